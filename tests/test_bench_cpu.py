"""bench.py's host-side pieces that need no GPU: the committed HBM-traffic profile
of the FP64 Dslash matches the current kernel sources (otherwise the benchmark's
roofline.traffic would silently become null), and --gpus above 1 is refused."""
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
