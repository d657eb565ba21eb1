"""bench.py's host-side pieces that need no GPU: the committed HBM-traffic profiles
of the FP64 Dslash and of the plain CG kernels match the current kernel sources
(otherwise the benchmark's roofline.traffic would silently become null), the
counter summary's calibration arithmetic, and --gpus above 1 is refused."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_traffic_profile_matches_the_dslash_sources():
    import bench
    with open(bench.TRAFFIC_FILE) as f:
        t = json.load(f)
    assert t["source_sha"] == bench.dslash_source_sha(), \
        "Dslash sources changed since the FETCH_SIZE/WRITE_SIZE runs: rerun them and regenerate the profile"
    vh = 32 ** 4 // 2
    assert t["vh"] == vh
    for shape, row in t["per_shape"].items():
        # calibrated HBM bytes of one launch: at least the algorithmic 2400 B per site, and not wildly above
        ratio = row["bytes_per_launch"] / (2400.0 * vh)
        assert 0.98 <= ratio <= 1.5, (shape, ratio)
        assert bench.traffic_from_profile(vh, int(shape)) == round(row["bytes_per_launch"])
    assert bench.traffic_from_profile(vh + 1, int(next(iter(t["per_shape"])))) is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_cg_traffic_profile_matches_the_cg_sources():
    """The plain CG kernels' committed traffic (the default line's roofline.traffic) belongs to the current
    sources, and every kernel moves at least its algorithmic bytes."""
    import bench
    with open(bench.CG_TRAFFIC_FILE) as f:
        t = json.load(f)
    assert t["source_sha"] == bench.dslash_source_sha(bench.CG_SOURCES), \
        "CG kernel sources changed since the FETCH_SIZE/WRITE_SIZE runs: rerun them and regenerate the profile"
    vh = 32 ** 4 // 2
    for name in ("k_cg_Ap_upd", "k_cg_Dp", "k_cg_p_norm"):
        row = t["kernels"][name]
        assert 0.98 <= row["bytes_per_launch"] / row["algorithmic_bytes"] <= 1.5, name
        assert bench.cg_traffic_from_profile(vh, name) == round(row["bytes_per_launch"])



def test_net_traffic_profile_matches_the_network_sources():
    """The network kernels' committed traffic belongs to the current sources, and every kernel moves at least
    its algorithmic bytes."""
    import bench
    with open(bench.NET_TRAFFIC_FILE) as f:
        t = json.load(f)
    assert t["source_sha"] == bench.dslash_source_sha(bench.NET_SOURCES), \
        "network kernel sources changed since the FETCH_SIZE/WRITE_SIZE runs: rerun them and regenerate the profile"
    for name, row in t["kernels"].items():
        assert 0.98 <= row["bytes_per_launch"] / row["algorithmic_bytes"] <= 3.0, name

def test_counter_summary_calibration(tmp_path, monkeypatch, capsys):
    """--counter-summary scales FETCH_SIZE and WRITE_SIZE (KiB per dispatch) by what they read for the 1 GiB
    device copy, averages per kernel and divides by the algorithmic bytes: checked on synthetic counter files."""
    import csv
    import bench
    head = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value", "Start_Timestamp", "End_Timestamp"]
    copy_kib = {"FETCH_SIZE": 524288.0, "WRITE_SIZE": 1048576.0}  # a copy reads as half its bytes in FETCH_SIZE
    layer = "void hisq::k_net_layer<16, 16>(hisq::Geom, char const*)"
    vals = {"FETCH_SIZE": [1.0e6, 1.2e6], "WRITE_SIZE": [3.0e5, 3.4e5]}
    for counter, sub in (("FETCH_SIZE", "f"), ("WRITE_SIZE", "w")):
        d = tmp_path / sub
        d.mkdir()
        with open(d / "x_counter_collection.csv", "w", newline="") as f:
            w = csv.writer(f)
            w.writerow(head)
            w.writerow([1, "__amd_rocclr_copyBuffer", counter, copy_kib[counter], 0, 1000])
            for i, v in enumerate(vals[counter]):
                w.writerow([2 + i, layer, counter, v, 0, 400000 + 20000 * i])
    out = tmp_path / "net.json"
    monkeypatch.setattr(bench, "NET_TRAFFIC_FILE", str(out))
    bench.summarize_counters("net", str(tmp_path / "f"), str(tmp_path / "w"))
    t = json.loads(out.read_text())
    assert t["fetch_factor"] == 2.0 and t["write_factor"] == 1.0
    row = t["kernels"]["k_net_layer<16,16>"]
    want = 1.1e6 * 1024 * 2.0 + 3.2e5 * 1024 * 1.0
    assert abs(row["bytes_per_launch"] - want) <= 1e-6 * want
    assert row["algorithmic_bytes"] == (4 * 72 + 32 * 24) * 16 ** 4 * 16
    assert abs(row["avg_us_under_counters"] - 410.0) < 1e-9
    assert "k_net_layer<16,16>" in capsys.readouterr().out
