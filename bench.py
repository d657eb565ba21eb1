#!/usr/bin/env python3
"""Benchmark of the HISQ Dslash and the even-odd CG it drives, on one MI355X.

Workload: 32^4 lattice, fat links 0.6 Haar SU(3) + 0.1 complex Gaussian noise,
long links Haar SU(3), staggered phases and antiperiodic time boundary folded
in, one complex Gaussian even-site source, mass 0.01, tol 1e-10 (synthetic,
seeded).  A step is one plain FP64 even-odd CG solve from x0 = 0 to a
recomputed residual |b - A x| / |b| <= 1e-10: the Dslash pair, the fused
normal-operator epilogue, the BLAS-1 updates with their reductions, the
convergence checks and the final FP64 residual.

Printed (one JSON line on stdout):
  value        sustained Dslash GB/s of the whole solve: algorithmic Dslash
               bytes (2400 B per output site per application: 16 FP64 links,
               one source and one output vector) over the wall time of the
               timed steps, inputs resident in HBM
  ms_per_step  seconds-to-1e-10 of plain FP64 CG, in ms
  roofline     the FP64 Dslash kernel alone, timed with HIP events on its stream
  cpu_baseline the CPU oracle on the host cores, same workload, bounded sample
  forms        time to 1e-10 of the chosen forms on the same problem
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

DIMS = (32, 32, 32, 32)
MASS = 0.01
TOL = 1e-10
CONFIG = 2  # seeds of the 32^4 workload
HBM_PEAK_GBS = 8000.0
DSLASH_SOURCES = ["paper_1411_2087_amd/csrc/hisq_common.hpp", "paper_1411_2087_amd/csrc/dslash_core.hpp",
                  "paper_1411_2087_amd/csrc/dslash.hip"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "dslash_f64_32x32x32x32_traffic.json")
# the plain CG's kernels: the Dslash core plus the fused CG epilogues
CG_SOURCES = DSLASH_SOURCES + ["paper_1411_2087_amd/csrc/cg_internal.hpp", "paper_1411_2087_amd/csrc/cg.hip"]
CG_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "cg_f64_32x32x32x32_traffic.json")
# algorithmic bytes per even site of the CG's dominant kernel, k_cg_Ap_upd: the parity-0 Dslash of t
# (16 FP64 matrices, t gathered once: 2304 + 48 B), p read at the site (48 B), x and r read and written
# (4 x 48 B); A p stays in registers
AP_UPD_BYTES = 2304 + 48 + 48 + 4 * 48
DP_BYTES = 2400  # k_cg_Dp: the parity-1 Dslash of p, t written


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def dslash_source_sha(sources=None):
    h = hashlib.sha256()
    for p in sources or DSLASH_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def cg_traffic_from_profile(vh, kernel):
    """HBM bytes per launch of the plain CG kernel `kernel` (k_cg_Dp / k_cg_Ap_upd) from committed rocprofv3
    FETCH_SIZE / WRITE_SIZE runs of the traffic probe, calibrated against a plain copy, or None if absent or
    taken on other kernel sources or another lattice."""
    try:
        with open(CG_TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("source_sha") != dslash_source_sha(CG_SOURCES) or t.get("vh") != vh:
        return None
    row = t.get("kernels", {}).get(kernel)
    return round(row["bytes_per_launch"]) if row else None


def traffic_from_profile(vh, shape):
    """HBM bytes per launch of the FP64 Dslash in launch shape `shape`, from committed
    rocprofv3 FETCH_SIZE / WRITE_SIZE runs (calibrated against a plain copy), or None
    if absent or taken on another version of the kernel or lattice."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("source_sha") != dslash_source_sha() or t.get("vh") != vh:
        return None
    row = t.get("per_shape", {}).get(str(shape))
    return round(row["bytes_per_launch"]) if row else None


NET_SOURCES = ["paper_1411_2087_amd/csrc/net.hip"]
NET_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "net_16x16x16x16_b16_c16_traffic.json")


def net_layer_bytes(cin, cout, sites):
    """Algorithmic bytes of one network layer (or its weight gradient) over `sites` (sites x batch): per site the
    four FP32 fat links it owns (each link serves two sites, 4 x 72 B) and the input and output features
    (24 B per channel: 3 complex64), links counted once per batch element."""
    return (4 * 72 + (cin + cout) * 24) * sites


def net_bwd_bytes(ci, co, sites):
    """Algorithmic bytes of the fused backward of a layer with CO input and CI output channels (input gradient
    through the adjoint layer and the weight gradient from the same transports): the links, the upstream
    gradient (CI channels), the layer input and the input gradient (CO channels each)."""
    return (4 * 72 + (ci + 2 * co) * 24) * sites


def summarize_counters(kind, fetch_dir, write_dir):
    """HBM traffic per launch from a pair of rocprofv3 --pmc runs (FETCH_SIZE, then WRITE_SIZE, in KiB per
    dispatch) of a traffic probe, each counter scaled by what it reads for the probe's 1 GiB device copy.
    kind "cg": the plain CG's k_cg_Dp / k_cg_Ap_upd / k_cg_p_norm on 32^4; kind "net": the network kernels on
    16^4, batch 16, C = 16; kind "dslash": the FP64 Dslash in every launch shape on 32^4 (the probe's tuner
    launches each shape 7 times in shape order; the first of the 7 is left out).  Writes the JSON summary under
    profiles/ and prints a markdown table."""
    import csv
    import glob
    import re

    def rows(d, counter):
        out = []
        for path in sorted(glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)):
            with open(path) as f:
                for r in csv.DictReader(f):
                    if r.get("Counter_Name") == counter:
                        us = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-3
                        out.append((int(r["Dispatch_Id"]), r["Kernel_Name"], float(r["Counter_Value"]), us))
        if not out:
            raise SystemExit(f"no {counter} rows under {d}")
        return [o[1:] for o in sorted(out)]  # dispatch order
    fetch, write = rows(fetch_dir, "FETCH_SIZE"), rows(write_dir, "WRITE_SIZE")
    copy_bytes = 1 << 30

    def copy_kib(rs):
        big = sorted(v for k, v, _ in rs if "copyBuffer" in k and v * 1024 > 0.25 * copy_bytes)
        if not big:
            raise SystemExit("no 1 GiB copy among the dispatches")
        return big[len(big) // 2]
    cf, cw = copy_kib(fetch), copy_kib(write)
    ff, wf = copy_bytes / (cf * 1024), copy_bytes / (cw * 1024)
    if kind == "cg":
        vh, sources, out_file = DIMS[0] * DIMS[1] * DIMS[2] * DIMS[3] // 2, CG_SOURCES, CG_TRAFFIC_FILE
        algo = {"k_cg_Ap_upd": AP_UPD_BYTES * vh, "k_cg_Dp": DP_BYTES * vh, "k_cg_p_norm": 3 * 48 * vh}

        def label(name):
            m = re.search(r"(k_cg_Ap_upd|k_cg_Dp|k_cg_p_norm)\b", name)
            return m.group(1) if m else None
    elif kind == "dslash":
        vh, sources, out_file = DIMS[0] * DIMS[1] * DIMS[2] * DIMS[3] // 2, DSLASH_SOURCES, TRAFFIC_FILE
        seq = {"fetch": [(n, v, us) for n, v, us in fetch if n.startswith("void hisq::k_dslash<hisq::PF64, ")],
               "write": [(n, v, us) for n, v, us in write if n.startswith("void hisq::k_dslash<hisq::PF64, ")]}
        import paper_1411_2087_amd as hq
        per = 7  # the tuner's 2 warm-up and 5 timed launches of each shape, in shape order
        nshapes = hq.hisq_dslash_shape(DIMS, hq.HISQ_F64, -2)
        if len(seq["fetch"]) < per * nshapes:
            raise SystemExit(f"{len(seq['fetch'])} FP64 Dslash dispatches, fewer than the tuner's {per * nshapes}")
        algo = {}

        def label(name):
            return None
    elif kind == "net":
        V, batch, sources, out_file = 16 ** 4, 16, NET_SOURCES, NET_TRAFFIC_FILE
        vh = V // 2
        algo = {}

        def label(name):
            m = re.search(r"(k_net_layer|k_net_wgrad|k_net_bwd)<(\d+), ?(\d+)", name)
            if not m:
                m1 = re.search(r"k_net_layer_mt<(\d+)>", name)  # the C -> 1 layer
                if not m1:
                    return None
                lab = f"k_net_layer_mt<{m1.group(1)}>"
                algo[lab] = net_layer_bytes(int(m1.group(1)), 1, V * batch)
                return lab
            lab = f"{m.group(1)}<{m.group(2)},{m.group(3)}>"
            nbytes = net_bwd_bytes if m.group(1) == "k_net_bwd" else net_layer_bytes
            algo[lab] = nbytes(int(m.group(2)), int(m.group(3)), V * batch)
            return lab
    else:
        raise SystemExit(f"unknown counter summary kind {kind}")
    groups = {}
    if kind == "dslash":
        for i in range(nshapes):
            lab = f"shape {i}"
            algo[lab] = 2400 * vh
            g_ = groups.setdefault(lab, {"fetch": [], "write": [], "us": []})
            for key in ("fetch", "write"):
                chunk = seq[key][per * i + 1:per * (i + 1)]
                g_[key] += [v for _, v, _ in chunk]
                if key == "fetch":
                    g_["us"] += [us for _, _, us in chunk]
                    g_["kernel"] = chunk[0][0].split("(")[0].replace("void hisq::", "")
    for rs, key in ((fetch, "fetch"), (write, "write")):
        for name, v, us in rs:
            lab = label(name)
            if lab:
                groups.setdefault(lab, {"fetch": [], "write": [], "us": []})[key].append(v)
                if key == "fetch":
                    groups[lab]["us"].append(us)
    table = {}
    for lab, g in sorted(groups.items(), key=lambda kv: (len(kv[0]), kv[0])):
        fk, wk = sum(g["fetch"]) / len(g["fetch"]), sum(g["write"]) / len(g["write"])
        fb, wb = fk * 1024 * ff, wk * 1024 * wf
        us = sum(g["us"]) / len(g["us"])
        table[lab] = {"kernel": g.get("kernel", lab), "dispatches": [len(g["fetch"]), len(g["write"])], "fetch_kib": fk, "write_kib": wk,
                      "fetch_bytes": fb, "write_bytes": wb, "bytes_per_launch": fb + wb,
                      "algorithmic_bytes": algo[lab], "ratio_to_algorithmic": (fb + wb) / algo[lab],
                      "avg_us_under_counters": us}
    res = {"kind": kind, "vh": vh, "source_sha": dslash_source_sha(sources), "copy_bytes": copy_bytes,
           "copy_fetch_kib": cf, "copy_write_kib": cw, "fetch_factor": ff, "write_factor": wf, "kernels": table}
    if kind == "dslash":  # keyed by launch shape, as traffic_from_profile reads it
        res["per_shape"] = {lab.split()[1]: t for lab, t in table.items()}
    with open(out_file, "w") as f:
        json.dump(res, f, indent=1)
    print(f"Calibration: a device copy of {copy_bytes} B reads as FETCH_SIZE {cf:.0f} KiB and WRITE_SIZE "
          f"{cw:.0f} KiB: one counter KiB is {ff:.3f} KiB fetched and {wf:.3f} KiB written.\n")
    print("| kernel | dispatches | FETCH_SIZE KiB | WRITE_SIZE KiB | HBM read GB | HBM written GB | algorithmic GB "
          "| traffic / algorithmic | avg us under counters |")
    print("|---|---|---|---|---|---|---|---|---|")
    for lab, t in table.items():
        print(f"| `{t['kernel'] if kind == 'dslash' else lab}`{' (' + lab + ')' if kind == 'dslash' else ''} | {t['dispatches'][0]} | {t['fetch_kib']:.0f} | {t['write_kib']:.0f} | "
              f"{t['fetch_bytes'] / 1e9:.4f} | {t['write_bytes'] / 1e9:.4f} | {t['algorithmic_bytes'] / 1e9:.4f} | "
              f"{t['ratio_to_algorithmic']:.3f} | {t['avg_us_under_counters']:.1f} |")
    print(f"\nKernel sources hash: `{res['source_sha']}`.")


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(fat, lng, b, vh, budget_s=15.0, cg_budget_s=45.0):
    """The CPU oracle on the host cores: its build for this machine (-O3 -march=native, compiled here), and
      - the value: CG iterations of the same 32^4 FP64 CG for about budget_s, as sustained Dslash GB/s;
      - the oracle Dslash on 8^4, 16^4, 32^4 and 48^3x96 (median of 5; of 3 single-threaded on the
        largest), with every thread and with one, as algorithmic GB/s and GFLOP/s (1146 flops per site);
      - the oracle CG to completion (1e-10) on 8^4 (m = 0.05) and 16^4 (m = 0.005), and 50 iterations on 48^3x96
        (m = 0.005) scaled to the GPU solve's 7610 iterations (marked extrapolated)."""
    import tempfile

    import numpy as np
    import oracle
    import synth
    from oracle import build as obuild
    lib = oracle.load_library(obuild.build_timing(os.path.join(tempfile.gettempdir(), "hisq_oracle_timing")))
    nthreads = oracle.num_threads(lib)
    t0 = time.perf_counter()
    oracle.apply_A(DIMS, MASS, fat, lng, b)
    t_A = time.perf_counter() - t0
    n_it = int(max(2, min(2000, (budget_s - 2 * t_A) / max(t_A, 1e-3))))
    log(f"[cpu] one A application {t_A:.2f}s -> {n_it} CG iterations")
    t0 = time.perf_counter()
    _, info = oracle.cg(DIMS, MASS, fat, lng, b, tol=1e-30, max_iter=n_it, lib=lib)
    dt = time.perf_counter() - t0
    n_dslash = 2 * info["iters"] + 4  # initial residual, 2 per iteration, final residual
    gbs = n_dslash * 2400.0 * vh / dt / 1e9
    out = {"value": round(gbs, 3), "unit": "GB/s", "cores": nthreads, "kind": "oracle",
           "sample": f"{info['iters']} iterations of the same 32^4 FP64 CG ({n_dslash} Dslash applications "
                     f"+ BLAS-1) in {dt:.1f} s; sustained algorithmic Dslash GB/s",
           "cpu_model": cpu_model(), "build": "gcc -O3 -march=native -fopenmp (plain loops, no intrinsics)"}
    # the oracle Dslash on every lattice of the workloads
    dsl = {}
    for dims in ((8, 8, 8, 8), (16, 16, 16, 16), (32, 32, 32, 32), (48, 48, 48, 96)):
        if dims == DIMS:
            f_, l_, s_ = fat, lng, b
        else:
            f_, l_ = synth.links(dims, synth.gauge_seed(3 if dims[3] == 96 else 1))
            s_ = synth.source(dims, synth.source_seed(1))
        vh_d = int(np.prod(dims)) // 2
        row = {}
        for th in (nthreads, 1):
            oracle.set_num_threads(th, lib)
            reps = 3 if (th == 1 and vh_d > 10 ** 6) else 5
            oracle.dslash(dims, f_, l_, s_, 1, lib=lib)
            ts = []
            for _ in range(reps):
                t1 = time.perf_counter()
                oracle.dslash(dims, f_, l_, s_, 1, lib=lib)
                ts.append(time.perf_counter() - t1)
            t = float(np.median(ts))
            row[f"threads_{th}"] = {"s": round(t, 5), "gbs": round(2400.0 * vh_d / t / 1e9, 2),
                                    "gflops": round(1146.0 * vh_d / t / 1e9, 2), "reps": reps}
        oracle.set_num_threads(nthreads, lib)
        dsl["x".join(map(str, dims))] = row
        log(f"[cpu] oracle dslash {'x'.join(map(str, dims))}: {row}")
        if dims != DIMS:
            del f_, l_, s_
    out["dslash"] = dsl
    # the oracle CG to completion on the two small workloads (16^4 at m = 0.005 needs ~7600 iterations: run
    # to completion when the oracle's measured Dslash rate says it fits cg_budget_s, else 200 iterations,
    # extrapolated to the GPU solve's iteration count and marked so)
    cgs = {}
    # 48^3x96 (m = 0.005, ~28 GB of traffic per iteration) is timed for 50 iterations and scaled to the GPU's
    # 7610, marked as extrapolated
    for dims, mass, cfg, gpu_iters, sample in (((8, 8, 8, 8), 0.05, 1, 753, 200),
                                               ((16, 16, 16, 16), 0.005, 5, 7582, 200),
                                               ((48, 48, 48, 96), 0.005, 3, 7610, 50)):
        f_, l_ = synth.links(dims, synth.gauge_seed(cfg))
        s_ = synth.source(dims, synth.source_seed(cfg))
        est = 2.2 * gpu_iters * dsl["x".join(map(str, dims))][f"threads_{nthreads}"]["s"]
        full = est <= cg_budget_s
        t1 = time.perf_counter()
        _, ci = oracle.cg(dims, mass, f_, l_, s_, tol=TOL if full else 1e-30, max_iter=100000 if full else sample,
                         lib=lib)
        t = time.perf_counter() - t1
        row = {"mass": mass, "iters": ci["iters"]}
        if full:
            row.update({"s": round(t, 3), "true_resid": ci["true_rel"], "converged": ci["converged"]})
        else:
            row.update({"s": round(t / ci["iters"] * gpu_iters, 3), "extrapolated": True,
                        "from": f"{ci['iters']} iterations in {t:.2f} s, scaled to {gpu_iters} iterations"})
        cgs["x".join(map(str, dims))] = row
        log(f"[cpu] oracle CG {'x'.join(map(str, dims))} m={mass}: {row}")
        del f_, l_, s_
    out["cg_to_1e-10"] = cgs
    return out


def form_batched(hq, dims, L64, L32, mode, n, log, cg_mode=0, seq_from=None):
    """Batched solve of n masses (log-spaced 0.002 - 0.2) against n sequential plain FP64 solves.
    cg_mode HISQ_CG_MIXED_F32C / HISQ_CG_MIXED_I16SC: L64 / L32 hold F64C / F32C or F64C / I16SC links.
    seq_from: a previous result of the same systems whose sequential plain FP64 time is reused."""
    import numpy as np
    import torch
    import synth
    masses = synth.log_masses(n, 0.002, 0.2)
    vh = int(np.prod(dims)) // 2
    if mode == hq.HISQ_MULTI_RHS:
        bs = np.stack([synth.source(dims, synth.source_seed(4, r)) for r in range(n)])
    else:
        bs = synth.source(dims, synth.source_seed(4))
    b = torch.from_numpy(bs).cuda()
    x = torch.zeros((n, vh, 3), dtype=torch.complex128, device="cuda")
    ws = hq.fields.workspace("cg_multi", dims, n, mode)
    opts = hq.CGOpts(mode=cg_mode, max_iter=0, check_every=0, use_graph=1, delta=0.0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = hq.cg_solve_multi(n, masses, TOL, mode, L64.fat, L64.lng, L32.fat, L32.lng, b, x, dims, opts, ws)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    del ws, x
    if seq_from is not None:
        seq, seq_iters = seq_from["sequential_plain_f64_s"], seq_from["sequential_plain_iters"]
    else:
        # the same systems one at a time with plain FP64 CG
        wsp = hq.fields.workspace("cg", dims)
        seq, seq_iters = 0.0, []
        for r in range(n):
            bb = (b[r] if mode == hq.HISQ_MULTI_RHS else b).contiguous()
            xx = torch.zeros_like(bb)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            s1 = hq.cg_solve(masses[r], TOL, L64.fat, L64.lng, None, None, bb, xx, dims, None, wsp)
            torch.cuda.synchronize()
            seq += time.perf_counter() - t1
            seq_iters.append(s1["iters"])
    name = ("multi_rhs" if mode == hq.HISQ_MULTI_RHS else "multi_shift") + f"_{n}"
    name += {hq.HISQ_CG_MIXED_F32C: "_f32c", hq.HISQ_CG_MIXED_I16SC: "_i16sc"}.get(cg_mode, "")
    log(f"[form {name}] {dt:.2f}s vs sequential plain FP64 {seq:.2f}s")
    return {"s": round(dt, 3), "n": n, "masses": "log-spaced 0.002-0.2", "iters": [s_["iters"] for s_ in st],
            "worst_true_resid": max(s_["true_resid"] for s_ in st), "sequential_plain_f64_s": round(seq, 3),
            "sequential_plain_iters": seq_iters, "speedup_vs_sequential_plain": round(seq / dt, 3)}


def polynomial_reference(hq, log, dims, mass, fat, lng, sources, C=4):
    """The network built, not trained, as K = p(A), p the Chebyshev-optimal quadratic on [4 m^2, lambda_max]
    (train.chebyshev_weights): exact on the naive operator (long links zero), where it shows what four fat-link
    layers can reach; on the HISQ operator the same weights miss the three-hop terms.  Flexible CG with it
    against plain FP64 CG on each operator and source."""
    import numpy as np
    import torch
    from paper_1411_2087_amd import train
    rows = {}
    for name, L in (("naive", np.zeros_like(lng)), ("hisq", lng)):
        L64 = hq.fields.Links.pack(fat, L, dims, hq.HISQ_F64)
        L32 = hq.fields.Links.pack(fat, L, dims, hq.HISQ_F32)
        lmax = train.lambda_max_estimate(L64, mass, dims)
        w, coef = train.chebyshev_weights(C, mass, lmax)
        wd = torch.from_numpy(w).cuda()
        wsc, wsf = hq.fields.workspace("cg", dims), hq.fields.workspace("fcg", dims, 1, 0, C)
        r = {"lambda_max": round(lmax, 3), "p_coeffs": [round(float(c), 6) for c in coef], "plain_iters": [],
             "plain_s": [], "fcg_iters": [], "fcg_s": [], "fallback_used": [], "fallback_iters": []}
        for src in sources:
            bd = torch.from_numpy(np.ascontiguousarray(src)).cuda()
            xp, xf = torch.zeros_like(bd), torch.zeros_like(bd)
            sp = hq.cg_solve(mass, TOL, L64.fat, L64.lng, None, None, bd, xp, dims, None, wsc)
            sf = hq.fcg_solve(mass, TOL, L64.fat, L64.lng, L32.fat, wd, C, bd, xf, dims, None, wsf)
            r["plain_iters"].append(sp["iters"])
            r["plain_s"].append(round(sp["time_s"], 4))
            r["fcg_iters"].append(sf["iters"])
            r["fcg_s"].append(round(sf["time_s"], 4))
            r["fallback_used"].append(sf["fallback_used"])
            r["fallback_iters"].append(sf["fallback_iters"])
        r["iteration_ratio_vs_plain"] = round(sum(r["fcg_iters"]) / sum(r["plain_iters"]), 3)
        log(f"[polynomial K, {name} operator] lambda_max {lmax:.3f}: plain {r['plain_iters']} {r['plain_s']}s, "
            f"fcg {r['fcg_iters']} {r['fcg_s']}s (fallback {r['fallback_used']})")
        rows[name] = r
    return rows


def trained_naive_reference(hq, log, dims, mass, fat, lng, sources, held, C=8, steps=1500):
    """A network trained where the fat-link layers can represent a good K: the naive operator (long links zero),
    the residual objective over a shuffled mix of Gaussian sources and normalised solutions x = A^-1 b (half
    each), from K = s 1; flexible CG with it against plain FP64 CG on the held-out sources."""
    import numpy as np
    import torch
    from paper_1411_2087_amd import train
    lng0 = np.zeros_like(lng)
    L64 = hq.fields.Links.pack(fat, lng0, dims, hq.HISQ_F64)
    L32 = hq.fields.Links.pack(fat, lng0, dims, hq.HISQ_F32)
    n = sources.shape[0]
    t0 = time.perf_counter()
    b, x, _, _ = train.make_pairs(dims, mass, L64, L32, sources)
    t_pairs = time.perf_counter() - t0
    nb = torch.linalg.vector_norm(b.reshape(n, -1), dim=1).reshape(-1, 1, 1)
    xn = x / torch.linalg.vector_norm(x.reshape(n, -1), dim=1).reshape(-1, 1, 1) * nb
    perm = torch.randperm(n, generator=torch.Generator().manual_seed(4)).cuda()
    inp = torch.cat([b[:n - n // 2], xn[:n // 2]])[perm]
    w0 = train.initial_weights(C, train.residual_scale(inp[:16], L32, mass, dims), 0.05, 99)
    tr = train.Trainer(dims, C, L32.fat, w0, batch=16, objective="residual", links32=L32, mass=mass)
    t0 = time.perf_counter()
    hist = tr.fit(inp[:-32], inp[:-32], steps=steps, lr=2e-3, log_every=500)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    wsc, wsf = hq.fields.workspace("cg", dims), hq.fields.workspace("fcg", dims, 1, 0, C)
    r = {"recipe": f"naive operator, C {C}, residual objective over {n - n // 2} Gaussian sources and {n // 2} "
                   f"normalised solutions, {steps} Adam steps", "pair_s": round(t_pairs, 2),
         "train_s": round(t_train, 2), "loss_log": [(s_, round(l, 4)) for s_, l in hist], "plain_iters": [],
         "plain_s": [], "fcg_iters": [], "fcg_s": [], "fallback_used": [], "fcg_true_resid": []}
    for src in held:
        bd = torch.from_numpy(np.ascontiguousarray(src)).cuda()
        xp, xf = torch.zeros_like(bd), torch.zeros_like(bd)
        sp = hq.cg_solve(mass, TOL, L64.fat, L64.lng, None, None, bd, xp, dims, None, wsc)
        sf = hq.fcg_solve(mass, TOL, L64.fat, L64.lng, L32.fat, tr.w, C, bd, xf, dims, None, wsf)
        r["plain_iters"].append(sp["iters"])
        r["plain_s"].append(round(sp["time_s"], 4))
        r["fcg_iters"].append(sf["iters"])
        r["fcg_s"].append(round(sf["time_s"], 4))
        r["fallback_used"].append(sf["fallback_used"])
        r["fcg_true_resid"].append(sf["true_resid"])
    r["iteration_ratio_vs_plain"] = round(sum(r["fcg_iters"]) / sum(r["plain_iters"]), 3)
    r["speedup_vs_plain"] = round(sum(r["plain_s"]) / sum(r["fcg_s"]), 3)
    log(f"[trained K, naive operator] pairs {t_pairs:.1f}s train {t_train:.1f}s: plain {r['plain_iters']} "
        f"{r['plain_s']}s, fcg {r['fcg_iters']} {r['fcg_s']}s (fallback {r['fallback_used']})")
    return r


def form_learned(hq, log, dims=(16, 16, 16, 16), mass=0.005, C=16, npairs=512, nheld=64, steps=600):
    """Learned preconditioner: 512 pairs from the batched CG (448 to train, 64 held out), GPU training with the
    residual objective, then flexible CG with the trained network, and with K = identity, against plain FP64 CG on
    a held-out source."""
    import numpy as np
    import torch
    import synth
    from paper_1411_2087_amd import train
    fat, lng = synth.links(dims, synth.gauge_seed(5))
    L64 = hq.fields.Links.pack(fat, lng, dims, hq.HISQ_F64)
    L32 = hq.fields.Links.pack(fat, lng, dims, hq.HISQ_F32)
    src = np.stack([synth.source(dims, synth.source_seed(5, i)) for i in range(npairs)])
    t0 = time.perf_counter()
    b, x, _, _ = train.make_pairs(dims, mass, L64, L32, src)
    t_pairs = time.perf_counter() - t0
    ntr = npairs - nheld
    tr = train.Trainer(dims, C, L32.fat, train.initial_weights(C, train.residual_scale(b[:16], L32, mass, dims), 0.05,
                                                               99), batch=16, objective="residual", links32=L32,
                       mass=mass)
    l0 = tr.evaluate(b[ntr:], x[ntr:])
    t0 = time.perf_counter()
    hist = tr.fit(b[:ntr], x[:ntr], steps=steps, lr=2e-3, log_every=200)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    l1 = tr.evaluate(b[ntr:], x[ntr:])
    bd = torch.from_numpy(src[ntr]).cuda()
    xp = torch.zeros_like(bd)
    sp = hq.cg_solve(mass, TOL, L64.fat, L64.lng, None, None, bd, xp, dims, None, hq.fields.workspace("cg", dims))
    wsf = hq.fields.workspace("fcg", dims, 1, 0, C)
    xf = torch.zeros_like(bd)
    sf = hq.fcg_solve(mass, TOL, L64.fat, L64.lng, L32.fat, tr.w, C, bd, xf, dims, None, wsf)
    xi = torch.zeros_like(bd)
    wid = torch.from_numpy(train.flatten(train.identity_weights(C))).cuda()
    si = hq.fcg_solve(mass, TOL, L64.fat, L64.lng, L32.fat, wid, C, bd, xi, dims, None, wsf)
    log(f"[form learned] pairs {t_pairs:.1f}s train {t_train:.1f}s (held-out loss {l0:.4f} -> {l1:.4f}); plain "
        f"{sp['iters']} it {sp['time_s']:.3f}s; fcg {sf['iters']} it (fallback {sf['fallback_used']}) "
        f"{sf['time_s']:.3f}s; fcg with K = 1 {si['iters']} it {si['time_s']:.3f}s")
    poly = polynomial_reference(hq, log, dims, mass, fat, lng, src[ntr:ntr + 1])
    naive = trained_naive_reference(hq, log, dims, mass, fat, lng, src[:256], src[ntr:ntr + 1])
    return {"workload": f"16^4, m {mass}, C {C}, residual objective, {npairs} pairs ({ntr} train / {nheld} held out)",
            "pairs": npairs, "pair_s": round(t_pairs, 2), "train_steps": steps, "train_s": round(t_train, 2),
            "held_out_loss": [round(l0, 4), round(l1, 4)], "loss_log": [(s_, round(l, 4)) for s_, l in hist],
            "plain_f64_s": round(sp["time_s"], 4), "plain_iters": sp["iters"], "fcg_s": round(sf["time_s"], 4),
            "fcg_iters": sf["iters"], "fallback_used": sf["fallback_used"], "fallback_iters": sf["fallback_iters"],
            "fcg_true_resid": sf["true_resid"], "fcg_identity_iters": si["iters"], "fcg_identity_s": round(si["time_s"], 4),
            "speedup_vs_plain": round(sp["time_s"] / sf["time_s"], 3),
            "iteration_ratio_vs_plain": round(sf["iters"] / sp["iters"], 3), "polynomial_K_C4": poly,
            "trained_naive_C8": naive}


def run_learned(args, dims=(16, 16, 16, 16), mass=0.005, npairs=512, nheld=64, steps=600, channels=(8, 16),
                nsolve=4):
    """The learned-preconditioner workload: 512 training pairs per gauge field (448 to train, 64 held out), the
    network trained on the GPU for each of `channels` with the residual objective, and flexible CG with the
    trained network against plain FP64 CG and against flexible CG with K = identity on `nsolve` held-out
    sources."""
    import numpy as np
    import torch

    import paper_1411_2087_amd as hq
    import synth
    from paper_1411_2087_amd import train
    fat, lng = synth.links(dims, synth.gauge_seed(5))
    L64 = hq.fields.Links.pack(fat, lng, dims, hq.HISQ_F64)
    L32 = hq.fields.Links.pack(fat, lng, dims, hq.HISQ_F32)
    src = np.stack([synth.source(dims, synth.source_seed(5, i)) for i in range(npairs)])
    t0 = time.perf_counter()
    b, x, _, _ = train.make_pairs(dims, mass, L64, L32, src, log=log if dims[0] > 16 else None)
    t_pairs = time.perf_counter() - t0
    log(f"[learned] {npairs} pairs in {t_pairs:.1f}s")
    ntrain = npairs - nheld
    held = [torch.from_numpy(src[ntrain + i]).cuda() for i in range(nsolve)]
    poly_src = src[ntrain:ntrain + 2].copy()
    del src

    def solve_all(fn):
        its, secs = [], []
        for bd in held:
            xx = torch.zeros_like(bd)
            st = fn(bd, xx)
            its.append(st["iters"])
            secs.append(st["time_s"])
        return its, secs, st
    wsp = hq.fields.workspace("cg", dims)
    p_its, p_s, _ = solve_all(lambda bd, xx: hq.cg_solve(mass, TOL, L64.fat, L64.lng, None, None, bd, xx, dims, None,
                                                           wsp))
    out = {"workload": f"{'x'.join(map(str, dims))}, m {mass}, {npairs} pairs ({ntrain} train / {nheld} held out), "
                       f"residual objective, {steps} Adam steps, batch 16",
           "pair_s": round(t_pairs, 2), "plain_f64": {"iters": p_its, "s": [round(v, 4) for v in p_s]}, "nets": {}}
    log(f"[learned] plain FP64 CG on {nsolve} held-out sources: {p_its} iterations, {sum(p_s):.3f}s")
    for C in channels:
        w0 = train.initial_weights(C, train.residual_scale(b[:16], L32, mass, dims), 0.05, 99)
        tr = train.Trainer(dims, C, L32.fat, w0, batch=16, objective="residual", links32=L32, mass=mass)
        l0 = tr.evaluate(b[ntrain:], x[ntrain:])
        t0 = time.perf_counter()
        hist = tr.fit(b[:ntrain], x[:ntrain], steps=steps, lr=2e-3, log_every=200 if dims[0] <= 16 else 50,
                      log=log if dims[0] > 16 else None)
        torch.cuda.synchronize()
        t_train = time.perf_counter() - t0
        l1 = tr.evaluate(b[ntrain:], x[ntrain:])
        wsf = hq.fields.workspace("fcg", dims, 1, 0, C)
        f_its, f_s, last = solve_all(lambda bd, xx: hq.fcg_solve(mass, TOL, L64.fat, L64.lng, L32.fat, tr.w, C, bd,
                                                                 xx, dims, None, wsf))
        wid = torch.from_numpy(train.flatten(train.identity_weights(C))).cuda()
        i_its, i_s, _ = solve_all(lambda bd, xx: hq.fcg_solve(mass, TOL, L64.fat, L64.lng, L32.fat, wid, C, bd, xx,
                                                              dims, None, wsf))
        out["nets"][f"C{C}"] = {"held_out_loss": [round(l0, 4), round(l1, 4)], "train_s": round(t_train, 2),
                                "loss_log": [(s_, round(l, 4)) for s_, l in hist],
                                "fcg_trained": {"iters": f_its, "s": [round(v, 4) for v in f_s],
                                                "fallback_used": last["fallback_used"],
                                                "fallback_iters": last["fallback_iters"]},
                                "fcg_identity": {"iters": i_its, "s": [round(v, 4) for v in i_s]},
                                "speedup_vs_plain": round(sum(p_s) / sum(f_s), 3)}
        log(f"[learned C={C}] held-out loss {l0:.4f} -> {l1:.4f}, train {t_train:.1f}s; fcg {f_its} "
            f"(fallback {last['fallback_used']}) {sum(f_s):.3f}s, identity {i_its}, plain {p_its} {sum(p_s):.3f}s")
    out["polynomial_K_C4"] = polynomial_reference(hq, log, dims, mass, fat, lng, poly_src)
    print(json.dumps({"metric": "CG s to 1e-10 resid, flexible CG with the trained network vs plain FP64 (report line)",
                      "unit": "s", "value": round(sum(out["nets"][f"C{channels[-1]}"]["fcg_trained"]["s"]), 4),
                      "n_gpus": 1,
                      "higher_is_better": False, "data": "synthetic", "config": {"workload": out["workload"]},
                      "learned": out}))


def run_shift_depth(args, n=8):
    """How deep the multi-shift CG's shifted phase should run before the batched refinement: 8 masses
    (log-spaced 0.002-0.2) at 32^4, one source, MULTI_SHIFT at several shift_tol against MULTI_RHS on the
    same systems, FP32 and two-row 16-bit inner links (report line)."""
    import numpy as np
    import torch

    import paper_1411_2087_amd as hq
    import synth
    fat, lng = synth.links(DIMS, synth.gauge_seed(4))
    fd, ld = torch.from_numpy(fat).cuda(), torch.from_numpy(lng).cuda()
    del fat, lng
    links = {p: hq.fields.Links.pack(fd, ld, DIMS, p)
             for p in (hq.HISQ_F64, hq.HISQ_F32, hq.HISQ_F64C, hq.HISQ_I16SC)}
    del fd, ld
    masses = synth.log_masses(n, 0.002, 0.2)
    b1 = torch.from_numpy(synth.source(DIMS, synth.source_seed(4))).cuda()
    bn = b1.unsqueeze(0).repeat(n, 1, 1).contiguous()
    vh = int(np.prod(DIMS)) // 2
    rows = {}
    for inner, mode, hi, lo in (("f32", hq.HISQ_CG_MIXED_F32, hq.HISQ_F64, hq.HISQ_F32),
                                ("i16sc", hq.HISQ_CG_MIXED_I16SC, hq.HISQ_F64C, hq.HISQ_I16SC)):
        H, L = links[hi], links[lo]
        for label, mmode, stol, b in [("multi_rhs", hq.HISQ_MULTI_RHS, 0.0, bn)] + \
                [(f"multi_shift_{t:.0e}", hq.HISQ_MULTI_SHIFT, t, b1) for t in (1e-3, 1e-4, 1e-5, 1e-6)]:
            ws = hq.fields.workspace("cg_multi", DIMS, n, mmode)
            x = torch.zeros((n, vh, 3), dtype=torch.complex128, device="cuda")
            o = hq.CGOpts(mode=mode, max_iter=0, check_every=0, use_graph=1, delta=0.0, shift_tol=stol)
            st = hq.cg_solve_multi(n, masses, TOL, mmode, H.fat, H.lng, L.fat, L.lng, b, x, DIMS, o, ws)
            r = {"s": round(st[0]["time_s"], 3), "iters": [s_["iters"] for s_ in st],
                 "worst_true_resid": max(s_["true_resid"] for s_ in st), "rc": st[0]["rc"]}
            if mmode == hq.HISQ_MULTI_SHIFT:
                # the shifted phase alone: its iterations and the FP64 true residuals it leaves
                x.zero_()
                o.shift_only = 1
                sp = hq.cg_solve_multi(n, masses, TOL, mmode, H.fat, H.lng, L.fat, L.lng, b, x, DIMS, o, ws)
                r["shifted_phase"] = {"s": round(sp[0]["time_s"], 3), "iters": [s_["iters"] for s_ in sp],
                                      "true_resid": [float(f"{s_['true_resid']:.2e}") for s_ in sp]}
            rows[f"{inner}/{label}"] = r
            log(f"[shift-depth] {inner} {label}: {r}")
            del ws, x
    print(json.dumps({"metric": "multi-shift CG s to 1e-10 by shifted-phase depth (report line)", "unit": "s",
                      "value": rows["f32/multi_shift_1e-03"]["s"], "n_gpus": 1, "higher_is_better": False,
                      "data": "synthetic",
                      "config": {"workload": "32^4, 8 masses 0.002-0.2, one source, tol 1e-10"}, "shift_depth": rows}))


def run_mdslash(args, nrhs=(8, 16), reps=20):
    """The multi-RHS FP32 Dslash alone at 32^4 (the kernel of the batched solves): every launch shape
    tuned, then the chosen one timed with HIP events; algorithmic bytes per site 1152 (16 FP32 links)
    + 48 N (N sources and N outputs of 24 bytes) (report line; the command of its counter profiles)."""
    import numpy as np
    import torch

    import paper_1411_2087_amd as hq
    import synth
    fat, lng = synth.links(DIMS, synth.gauge_seed(CONFIG))
    L = hq.fields.Links.pack(fat, lng, DIMS, hq.HISQ_F32)
    vh = int(np.prod(DIMS)) // 2
    ws = torch.empty(1 << 16, dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()
    rows = {}
    for n in nrhs:
        src = np.stack([synth.source(DIMS, synth.source_seed(CONFIG, r)) for r in range(n)], axis=1)
        s_ = torch.from_numpy(src.astype(np.complex64)).cuda().contiguous()
        d_ = torch.empty_like(s_)
        best, us = hq.hisq_tune_multi(L.fat, L.lng, s_, d_, DIMS, n, ws, reps=5)
        t = timed(lambda: hq.hisq_dslash_multi(L.fat, L.lng, s_, d_, 1, n, DIMS, ws), reps, stream)
        bps = 1152 + 48 * n
        rows[f"N{n}"] = {"shape": best, "shape_us": [round(u, 1) for u in us], "us": round(t, 1),
                         "bytes_per_site": bps, "gbs": round(bps * vh / t / 1e3, 1),
                         "frac": round(bps * vh / t / 1e3 / HBM_PEAK_GBS, 4)}
        log(f"[mdslash] N={n}: shape {best} {t:.1f} us {rows[f'N{n}']['gbs']} GB/s")
        del s_, d_
    print(json.dumps({"metric": "multi-RHS FP32 Dslash GB/s at 32^4 (report line)", "unit": "GB/s",
                      "value": rows[f"N{nrhs[0]}"]["gbs"], "n_gpus": 1, "higher_is_better": True,
                      "data": "synthetic", "config": {"workload": "32^4 multi-RHS FP32 Dslash"}, "mdslash": rows}))


def run_net_kernels(args, dims=(16, 16, 16, 16), C=16, batch=16, reps=5):
    """The network's kernels alone on the training shape: forward (4 layers) and backward (layers 4, 3, 2
    fused input and weight gradients, layer 1's weight gradient and input gradient) of a batch of 16
    sources at 16^4, C = 16, timed with HIP events on the stream they run on.  Algorithmic bytes per
    full-lattice site of a C_in -> C_out layer: the fat links (four FP32 matrices, each serving two sites)
    and the input and output features (24 bytes per channel); of a weight gradient the links, the input
    features and the upstream gradient; of a fused backward the links, the upstream gradient, the layer
    input and the input gradient."""
    import numpy as np
    import torch

    import paper_1411_2087_amd as hq
    import synth
    from paper_1411_2087_amd import train
    fat, lng = synth.links(dims, synth.gauge_seed(5))
    L32 = hq.fields.Links.pack(fat, lng, dims, hq.HISQ_F32)
    del fat, lng
    V = int(np.prod(dims))
    r = np.random.default_rng(7)
    w = torch.from_numpy(train.flatten(train.initial_weights(C, 1.0, 0.2, 7))).cuda()
    src = np.stack([synth.source(dims, synth.source_seed(5, i)) for i in range(batch)]).astype(np.complex64)
    b = torch.from_numpy(src).cuda()
    y = torch.empty_like(b)
    gout = torch.from_numpy((r.standard_normal(src.shape) + 1j * r.standard_normal(src.shape)).astype(np.complex64)).cuda()
    gin = torch.empty_like(b)
    gw = torch.empty(hq.net_weight_count(C), dtype=torch.complex64, device="cuda")
    acts = torch.empty(hq.net_act_bytes(dims, C, batch), dtype=torch.uint8, device="cuda")
    ws = torch.empty(hq.net_backward_ws_bytes(dims, C, batch), dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()
    if args.traffic_probe:  # counter calibration, then one forward and one backward
        cs = torch.ones((1 << 30) // 4, dtype=torch.float32, device="cuda")
        cd = torch.empty_like(cs)
        for _ in range(3):
            cd.copy_(cs)
        del cs, cd
        hq.net_forward(L32.fat, w, C, b, y, acts, batch, dims)
        hq.net_backward(L32.fat, w, C, acts, gout, gw, gin, batch, dims, ws)
        torch.cuda.synchronize()
        print(json.dumps({"traffic_probe": True, "copy_bytes": 1 << 30, "workload": "net-kernels"}))
        return

    def fwd():
        hq.net_forward(L32.fat, w, C, b, y, acts, batch, dims)

    def bwd():
        hq.net_backward(L32.fat, w, C, acts, gout, gw, gin, batch, dims, ws)
    fwd()
    bwd()
    t_f = timed(fwd, reps, stream) * 1e-6  # seconds per call
    t_b = timed(bwd, reps, stream) * 1e-6
    layer_bytes = lambda ci, co: net_layer_bytes(ci, co, V * batch)
    fwd_bytes = layer_bytes(1, C) + 2 * layer_bytes(C, C) + layer_bytes(C, 1)
    # backward: the fused layers 4, 3, 2, then layer 1's weight gradient and (grad_in given) input gradient
    bwd_bytes = (net_bwd_bytes(1, C, V * batch) + 2 * net_bwd_bytes(C, C, V * batch) + layer_bytes(1, C)
                 + layer_bytes(C, 1))
    out = {"workload": f"network forward / backward, {'x'.join(map(str, dims))}, C {C}, batch {batch}",
           "forward_ms": round(t_f * 1e3, 3), "backward_ms": round(t_b * 1e3, 3),
           "forward_gbs": round(fwd_bytes / t_f / 1e9, 1), "backward_gbs": round(bwd_bytes / t_b / 1e9, 1),
           "cc_layer_bytes": layer_bytes(C, C)}
    log(f"[net] forward {t_f * 1e3:.3f} ms ({out['forward_gbs']} GB/s), backward {t_b * 1e3:.3f} ms "
        f"({out['backward_gbs']} GB/s)")
    print(json.dumps({"metric": "network forward / backward time (report line)", "unit": "ms",
                      "value": out["forward_ms"] + out["backward_ms"], "n_gpus": 1, "higher_is_better": False,
                      "data": "synthetic", "config": {"workload": out["workload"]}, "net": out}))


LARGE_DIMS, LARGE_MASS = (48, 48, 48, 96), 0.005
# 48^3x96 CG kernels: k_cg_Dp moves the Dslash bytes, k_cg_Ap_upd those of AP_UPD_BYTES


def large_lattice(hq, log, precs, forms_list):
    """48^3 x 96, m = 0.005: each storage form's tuned Dslash (HIP events), then seconds to 1e-10 of the listed
    CG forms.  The plain FP64 solve runs with its kernels timed one by one (direct launches, HIP events), which
    gives the CG kernels' durations on the largest lattice."""
    import numpy as np
    import torch

    import synth
    dims, mass = LARGE_DIMS, LARGE_MASS
    vh = int(np.prod(dims)) // 2
    log("[setup] generating 48^3x96 links and source")
    fat, lng = synth.links(dims, synth.gauge_seed(3))
    b_np = synth.source(dims, synth.source_seed(3))
    fd, ld = torch.from_numpy(fat).cuda(), torch.from_numpy(lng).cuda()
    del fat, lng
    L = {p: hq.fields.Links.pack(fd, ld, dims, p) for p in precs}
    del fd, ld
    b = torch.from_numpy(b_np).cuda()
    dsl = {}
    for p in precs:
        dt = hq.fields.VEC_DTYPE[p]
        s_, d_ = b.to(dt), torch.empty(b.shape, dtype=dt, device="cuda")
        best, us = hq.hisq_tune_dslash(L[p].fat, L[p].lng, s_, d_, dims, p, reps=10)
        t = us[best] * 1e-6  # the shape the library runs
        gbs = hq.DSLASH_BYTES_PER_SITE[p] * vh / t / 1e9
        dsl[p] = {"us": round(t * 1e6, 1), "gbs": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4), "shape": best,
                  "us_per_shape": [round(u, 1) for u in us]}
        log(f"[dslash 48^3x96] prec {p}: {dsl[p]}")
        del s_, d_
    lo_of = {hq.HISQ_CG_MIXED_F32: hq.HISQ_F32, hq.HISQ_CG_MIXED_I16S: hq.HISQ_I16S,
             hq.HISQ_CG_MIXED_F32C: hq.HISQ_F32C, hq.HISQ_CG_MIXED_I16SC: hq.HISQ_I16SC,
             hq.HISQ_CG_MIXED_F16S: hq.HISQ_F16S}
    forms = {}
    for name, mode in forms_list:
        hi = L[hq.HISQ_F64C] if mode in (hq.HISQ_CG_PLAIN_F64C, hq.HISQ_CG_MIXED_F32C,
                                         hq.HISQ_CG_MIXED_I16SC) else L[hq.HISQ_F64]
        lo = L[lo_of[mode]] if mode in lo_of else None
        ws = hq.fields.workspace("cg", dims, 1, mode)
        x = torch.zeros_like(b)
        timing = mode == hq.HISQ_CG_PLAIN_F64
        o = hq.CGOpts(mode=mode, max_iter=0, check_every=0, use_graph=2 if timing else 1, delta=0.0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = hq.cg_solve(mass, TOL, hi.fat, hi.lng, lo.fat if lo is not None else None,
                         lo.lng if lo is not None else None, b, x, dims, o, ws)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        forms[name] = {"s": round(dt, 3), "iters": st["iters"], "reliable_updates": st["reliable_updates"],
                       "true_resid": st["true_resid"], "rc": st["rc"], "fallback_used": st["fallback_used"],
                       "fallback_iters": st["fallback_iters"]}
        if timing:
            t_dp, t_ap, t_pn = (u * 1e-6 for u in st["kernel_us"])
            forms[name]["kernels"] = {
                "k_cg_Dp": {"avg_us": round(t_dp * 1e6, 1), "gbs": round(DP_BYTES * vh / t_dp / 1e9, 1),
                            "frac": round(DP_BYTES * vh / t_dp / 1e9 / HBM_PEAK_GBS, 4)},
                "k_cg_Ap_upd": {"avg_us": round(t_ap * 1e6, 1), "gbs": round(AP_UPD_BYTES * vh / t_ap / 1e9, 1),
                                "frac": round(AP_UPD_BYTES * vh / t_ap / 1e9 / HBM_PEAK_GBS, 4)},
                "k_cg_p_norm": {"avg_us": round(t_pn * 1e6, 1)}}
        log(f"[48^3x96 {name}] {dt:.2f}s iters={st['iters']} resid={st['true_resid']:.2e} "
            f"fallback={st['fallback_used']} ({st['fallback_iters']} plain iterations) {forms[name].get('kernels', '')}")
        del ws, x
    base = forms["plain_f64"]["s"]
    for k in forms:
        forms[k]["speedup_vs_plain"] = round(base / forms[k]["s"], 3)
    del L
    torch.cuda.empty_cache()
    return {"dslash": {str(k): v for k, v in dsl.items()}, "forms": forms}


def run_large(args):
    """48^3 x 96, m = 0.005: seconds to 1e-10 of plain FP64 CG and of every mixed-precision form."""
    import paper_1411_2087_amd as hq
    precs = (hq.HISQ_F64, hq.HISQ_F32, hq.HISQ_I16S, hq.HISQ_F64C, hq.HISQ_F32C, hq.HISQ_I16SC, hq.HISQ_F16S)
    forms_list = (("plain_f64", hq.HISQ_CG_PLAIN_F64), ("plain_f64c", hq.HISQ_CG_PLAIN_F64C),
                  ("mixed_f32", hq.HISQ_CG_MIXED_F32), ("mixed_i16s", hq.HISQ_CG_MIXED_I16S),
                  ("mixed_f32c", hq.HISQ_CG_MIXED_F32C), ("mixed_i16sc", hq.HISQ_CG_MIXED_I16SC),
                  ("mixed_f16s", hq.HISQ_CG_MIXED_F16S))
    r = large_lattice(hq, log, precs, forms_list)
    print(json.dumps({"metric": "CG s to 1e-10 resid, FP64 plain vs chosen form (report line)", "unit": "s",
                      "value": r["forms"]["plain_f64"]["s"], "n_gpus": 1, "higher_is_better": False,
                      "data": "synthetic", "config": {"workload": "HISQ even-odd CG, 48^3x96, mass 0.005, tol 1e-10"},
                      "dslash": r["dslash"], "forms": r["forms"]}))


def traffic_probe_at(workload):
    """A 1 GiB copy (counter calibration) and 5 FP64 Dslash launches in each of launch shapes 6, 8, 10, 11 and 12
    (plain and default-blocked tile order at one term and 6 waves/SIMD; the FP64 default, two terms at 5
    waves/SIMD, in plain order and in blocks of 8 and of 4 t-planes by the whole z extent) on the lattice
    `workload` ("LxxLyxLzxLt"), for rocprofv3 counter runs."""
    import torch
    import paper_1411_2087_amd as hq
    import synth
    dims = tuple(int(v) for v in workload.split("x"))
    fat, lng = synth.links(dims, synth.gauge_seed(3))
    L = hq.fields.Links.pack(fat, lng, dims, hq.HISQ_F64)
    del fat, lng
    b = torch.from_numpy(synth.source(dims, synth.source_seed(3))).cuda()
    t = torch.empty_like(b)
    n = 1 << 30
    src = torch.ones(n // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    shapes = (6, 8, 10, 11, 12)
    for shape in shapes:  # 5 launches each
        hq.hisq_dslash_shape(dims, hq.HISQ_F64, shape)
        for _ in range(5):
            hq.dslash_apply(L.fat, L.lng, b, t, 1, dims, hq.HISQ_F64)
    torch.cuda.synchronize()
    print(json.dumps({"traffic_probe": True, "copy_bytes": n, "dslash_launches": 5, "vh": int(b.shape[0]),
                      "shapes": list(shapes), "workload": workload}))


def run_batched16(args):
    """16 masses log-spaced 0.002 - 0.2 on 32^4: batched multi-RHS (16 sources) and multi-shift (one source), on
    FP32, two-row FP32 and two-row 16-bit inner links, against 16 sequential plain FP64 solves of the same systems (a report line)."""
    import torch
    import paper_1411_2087_amd as hq
    import synth
    fat, lng = synth.links(DIMS, synth.gauge_seed(CONFIG))
    fd, ld = torch.from_numpy(fat).cuda(), torch.from_numpy(lng).cuda()
    del fat, lng
    L = {p: hq.fields.Links.pack(fd, ld, DIMS, p)
         for p in (hq.HISQ_F64, hq.HISQ_F32, hq.HISQ_F64C, hq.HISQ_F32C, hq.HISQ_I16SC)}
    del fd, ld
    forms = {}
    for mode, name in ((hq.HISQ_MULTI_RHS, "multi_rhs_16"), (hq.HISQ_MULTI_SHIFT, "multi_shift_16")):
        forms[name] = form_batched(hq, DIMS, L[hq.HISQ_F64], L[hq.HISQ_F32], mode, 16, log)
        forms[name + "_f32c"] = form_batched(hq, DIMS, L[hq.HISQ_F64C], L[hq.HISQ_F32C], mode, 16, log,
                                             hq.HISQ_CG_MIXED_F32C, forms[name])
        forms[name + "_i16sc"] = form_batched(hq, DIMS, L[hq.HISQ_F64C], L[hq.HISQ_I16SC], mode, 16, log,
                                              hq.HISQ_CG_MIXED_I16SC, forms[name])
    print(json.dumps({"workload": "batched solves of 16 masses 0.002-0.2, 32^4, tol 1e-10", "n_gpus": 1,
                      "forms": forms}))


PAPER_GRIDS = ((32, 32, 32, 128), (32, 40, 24, 96))
MATMUL_FLOPS = 198        # 3x3 complex product: 27 complex multiplies (6) + 18 complex adds (2)


def timed(fn, reps, stream):
    """Microseconds per call of fn() with HIP events on `stream` (2 warm-up calls)."""
    import torch
    fn()
    fn()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1) * 1e3 / reps


def link_construction(hq, dims, log):
    """Three-link products (Sec. 4) and the path-summed one-link matrices from Haar thin links."""
    import numpy as np
    import torch
    import synth
    V = int(np.prod(dims))
    U = torch.from_numpy(synth.thin_links(dims, synth.gauge_seed(7))).cuda()
    out = torch.empty_like(U)
    stream = torch.cuda.current_stream()
    us3 = timed(lambda: hq.hisq_three_link(U, out, dims), 20, stream)
    n = 4 * V
    row = {"three_link_us": round(us3, 1), "three_link_gflops": round(2 * MATMUL_FLOPS * n / us3 / 1e3, 1),
           "three_link_gbs": round(288.0 * n / us3 / 1e3, 1)}
    ws = hq.fields.workspace("fat_paths", dims)
    coeff = (1 / 8, 1 / 16, 1 / 64, 1 / 384, -1 / 16)
    us_f = timed(lambda: hq.hisq_fat_paths(U, coeff, out, dims, ws), 2, stream)
    # staple launches: per (mu, nu) one 3-staple, two 5-staples, two 7-staples and two signed
    # Lepage pairs, each with 4 (both signs) or 2 (one sign) products per site
    prods = 4 * 3 * (4 + 2 * 4 + 2 * 4 + 2 * (2 + 2))
    row.update({"fat_paths_ms": round(us_f / 1e3, 2), "fat_paths_gflops": round(prods * MATMUL_FLOPS * V / us_f / 1e3, 1),
                "fat_paths_coeff": "fat7 weights + Lepage -1/16"})
    log(f"[links {'x'.join(map(str, dims))}] {row}")
    del U, out, ws
    return row


def run_paper_grids(args):
    """Dslash alone on the two lattices of the paper's single-coprocessor runs (Sec. 4, Tables 1-2), every
    storage form: microseconds, GFLOP/s at 1146 flops per site, algorithmic GB/s."""
    import numpy as np
    import torch

    import paper_1411_2087_amd as hq
    import synth
    names = {hq.HISQ_F64: "f64", hq.HISQ_F32: "f32", hq.HISQ_F16S: "f16s", hq.HISQ_I16S: "i16s",
             hq.HISQ_F64C: "f64c", hq.HISQ_F32C: "f32c", hq.HISQ_I16SC: "i16sc"}
    grids = {}
    for dims in PAPER_GRIDS:
        vh = int(np.prod(dims)) // 2
        tag = "x".join(map(str, dims))
        log(f"[setup] generating {tag} links and source")
        fat, lng = synth.links(dims, synth.gauge_seed(6))
        b = torch.from_numpy(synth.source(dims, synth.source_seed(6))).cuda()
        fd, ld = torch.from_numpy(fat).cuda(), torch.from_numpy(lng).cuda()
        del fat, lng
        rows = {}
        for p in names:
            L = hq.fields.Links.pack(fd, ld, dims, p)
            dt = hq.fields.VEC_DTYPE[p]
            s_, d_ = b.to(dt), torch.empty(b.shape, dtype=dt, device="cuda")
            best, us = hq.hisq_tune_dslash(L.fat, L.lng, s_, d_, dims, p, reps=20)
            t = us[best] * 1e-6  # the shape the library runs
            rows[names[p]] = {"us": round(t * 1e6, 1), "gflops": round(1146.0 * vh / t / 1e9, 1),
                              "gbs": round(hq.DSLASH_BYTES_PER_SITE[p] * vh / t / 1e9, 1),
                              "bytes_per_site": hq.DSLASH_BYTES_PER_SITE[p], "shape": best}
            log(f"[dslash {tag}] {names[p]}: {rows[names[p]]}")
            del L, s_, d_
        del fd, ld, b
        torch.cuda.empty_cache()
        rows["link_construction"] = link_construction(hq, dims, log)
        grids[tag] = rows
        torch.cuda.empty_cache()
    print(json.dumps({"metric": "Dslash GFLOP/s and GB/s on the paper's lattices (report line)", "unit": "GFLOP/s",
                      "value": grids["32x32x32x128"]["f32"]["gflops"], "n_gpus": 1, "higher_is_better": True,
                      "data": "synthetic", "dtype": "f32",
                      "config": {"workload": "HISQ Dslash (one-link + Naik three-link), 32^3x128 and 32x40x24x96, "
                                             "parity 1, every link storage form"},
                      "paper_xeon_phi_sp_naik_gflops": {"uncompressed": "136-140", "compressed": "178-193"},
                      "grids": grids}))


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--dslash-reps", type=int, default=100)
    ap.add_argument("--no-forms", action="store_true", help="skip the chosen-form solves")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched (multi-RHS / multi-shift) forms")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-preconditioner form")
    ap.add_argument("--no-large", action="store_true", help="skip the 48^3x96 entries of the default line")
    ap.add_argument("--counter-summary", nargs=3, metavar=("KIND", "FETCH_DIR", "WRITE_DIR"),
                    help="on the host, after two rocprofv3 --pmc runs of a traffic probe (FETCH_SIZE, WRITE_SIZE): "
                         "write the calibrated per-launch HBM traffic of the plain CG kernels (KIND cg) or the "
                         "network kernels (KIND net) under profiles/ and print a markdown table")
    ap.add_argument("--workload", default="32x32x32x32",
                    help="32x32x32x32 (default: plain FP64 CG, the metric's workload), 48x48x48x96 "
                         "(mixed precision against plain FP64 on the large lattice), paper-grids (the Dslash "
                         "on 32^3x128 and 32x40x24x96), learned (512 training pairs on 16^4, C = 8 and 16), "
                         "learned-32 (the same on 32^4, C = 16, two held-out solves) or "
                         "batched-16 (16 masses, batched against sequential plain FP64 solves) or net-kernels "
                         "(the network's forward and backward kernels at 16^4, batch 16, C = 16) or shift-depth "
                         "(the multi-shift CG's shifted phase run to several depths) or mdslash (the multi-RHS "
                         "Dslash alone at 32^4, N = 8 and 16); "
                         "all but the first are report lines, not the metric")
    ap.add_argument("--traffic-probe", action="store_true",
                    help="only run a 1 GiB copy and the FP64 Dslash (for rocprofv3 counter runs); with --workload "
                         "LxxLyxLzxLt on that lattice")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the path has no multi-GPU "
              "decomposition; see the design notes on sharding)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1411_2087_amd as hq
    import synth

    if args.counter_summary:
        return summarize_counters(*args.counter_summary)
    if args.traffic_probe and args.workload == "net-kernels":
        return run_net_kernels(args)
    if args.traffic_probe and args.workload != "32x32x32x32":
        return traffic_probe_at(args.workload)
    if args.workload == "48x48x48x96":
        return run_large(args)
    if args.workload == "paper-grids":
        return run_paper_grids(args)
    if args.workload == "learned":
        return run_learned(args)
    if args.workload == "learned-32":
        return run_learned(args, dims=(32, 32, 32, 32), channels=(16,), nsolve=2)
    if args.workload == "batched-16":
        return run_batched16(args)
    if args.workload == "net-kernels":
        return run_net_kernels(args)
    if args.workload == "shift-depth":
        return run_shift_depth(args)
    if args.workload == "mdslash":
        return run_mdslash(args)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    vh = int(np.prod(DIMS)) // 2
    log(f"[setup] generating 32^4 links and source")
    fat, lng = synth.links(DIMS, synth.gauge_seed(CONFIG))
    b_np = synth.source(DIMS, synth.source_seed(CONFIG))
    fat_d, lng_d = torch.from_numpy(fat).to(dev), torch.from_numpy(lng).to(dev)
    L64 = hq.fields.Links.pack(fat_d, lng_d, DIMS, hq.HISQ_F64)
    L32 = hq.fields.Links.pack(fat_d, lng_d, DIMS, hq.HISQ_F32)
    L16 = hq.fields.Links.pack(fat_d, lng_d, DIMS, hq.HISQ_F16S)
    LI16 = hq.fields.Links.pack(fat_d, lng_d, DIMS, hq.HISQ_I16S)
    L64C = hq.fields.Links.pack(fat_d, lng_d, DIMS, hq.HISQ_F64C)
    L32C = hq.fields.Links.pack(fat_d, lng_d, DIMS, hq.HISQ_F32C)
    LI16C = hq.fields.Links.pack(fat_d, lng_d, DIMS, hq.HISQ_I16SC)
    del fat_d, lng_d
    torch.cuda.synchronize()
    b = torch.from_numpy(b_np).to(dev)
    x = torch.zeros_like(b)
    stream = torch.cuda.current_stream()

    if args.traffic_probe:
        n = 1 << 30
        src = torch.ones(n // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        tmp = torch.empty_like(b)
        for _ in range(3):
            dst.copy_(src)
        shape, _ = hq.hisq_tune_dslash(L64.fat, L64.lng, b, tmp, DIMS, hq.HISQ_F64, reps=5)
        for i in range(5):  # the last 5 FP64 Dslash dispatches are the measured ones
            hq.dslash_apply(L64.fat, L64.lng, b, tmp, 1, DIMS, hq.HISQ_F64)
        # and 6 iterations of the plain CG, launched directly (the kernels of the timed solve)
        wsp = hq.fields.workspace("cg", DIMS)
        xp = torch.zeros_like(b)
        op = hq.CGOpts(mode=hq.HISQ_CG_PLAIN_F64, max_iter=6, check_every=6, use_graph=0, delta=0.0)
        hq.cg_solve(MASS, TOL, L64.fat, L64.lng, None, None, b, xp, DIMS, op, wsp)
        torch.cuda.synchronize()
        print(json.dumps({"traffic_probe": True, "copy_bytes": n, "dslash_launches": 5, "cg_iterations": 6, "vh": vh,
                          "shape": shape}))
        return

    # autotune the Dslash launch shape of each precision on this lattice
    tuned = {}
    tmp = torch.empty_like(b)
    for name, prec, L in (("f64", hq.HISQ_F64, L64), ("f32", hq.HISQ_F32, L32), ("f16s", hq.HISQ_F16S, L16),
                          ("i16s", hq.HISQ_I16S, LI16), ("f64c", hq.HISQ_F64C, L64C), ("f32c", hq.HISQ_F32C, L32C),
                          ("i16sc", hq.HISQ_I16SC, LI16C)):
        dt = hq.fields.VEC_DTYPE[prec]
        s_, d_ = b.to(dt), torch.empty(b.shape, dtype=dt, device=dev)
        best, us = hq.hisq_tune_dslash(L.fat, L.lng, s_, d_, DIMS, prec, reps=20)
        tuned[name] = {"shape": best, "us": [round(u, 1) for u in us],
                       "gbs": round(hq.DSLASH_BYTES_PER_SITE[prec] * vh / (us[best] * 1e-6) / 1e9, 1)}
        log(f"[tune] {name}: shape {best}, us per shape {tuned[name]['us']}")
        del s_, d_

    ws = hq.fields.workspace("cg", DIMS, 1, hq.HISQ_CG_PLAIN_F64)
    opts = hq.CGOpts(mode=hq.HISQ_CG_PLAIN_F64, max_iter=0, check_every=0, use_graph=1, delta=0.0)

    def step():
        x.zero_()
        return hq.cg_solve(MASS, TOL, L64.fat, L64.lng, None, None, b, x, DIMS, opts, ws, raise_on_noconv=True)

    for i in range(args.warmup):
        st = step()
        log(f"[warmup {i}] iters={st['iters']} resid={st['true_resid']:.2e} {st['time_s']:.3f}s")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = [step() for _ in range(args.steps)]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    for i, st in enumerate(stats):
        log(f"[step {i}] iters={st['iters']} resid={st['true_resid']:.2e} {st['time_s']:.3f}s")
    n_dslash = sum(2 * st["iters"] + 4 + 4 * st["restarts"] for st in stats)
    value = n_dslash * 2400.0 * vh / wall / 1e9
    ms_per_step = wall / args.steps * 1e3
    x_np = x.cpu().numpy()

    # the solve's kernels timed one by one: the same solve with direct launches and HIP events around
    # its three main kernels, on the stream they run on
    x.zero_()
    st_k = hq.cg_solve(MASS, TOL, L64.fat, L64.lng, None, None, b, x,
                       DIMS, hq.CGOpts(mode=hq.HISQ_CG_PLAIN_F64, max_iter=0, check_every=0, use_graph=2, delta=0.0),
                       ws, raise_on_noconv=True)
    t_dp, t_ap, t_pn = (u * 1e-6 for u in st_k["kernel_us"])
    ap_achieved = AP_UPD_BYTES * vh / t_ap / 1e9
    log(f"[cg kernels] k_cg_Dp {t_dp * 1e6:.1f} us, k_cg_Ap_upd {t_ap * 1e6:.1f} us "
        f"({ap_achieved:.0f} GB/s), k_cg_p_norm {t_pn * 1e6:.1f} us over {st_k['iters']} iterations")

    # the FP64 Dslash kernel alone: HIP events on the stream it runs on
    for i in range(10):
        hq.dslash_apply(L64.fat, L64.lng, b, tmp, 1, DIMS, hq.HISQ_F64)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for i in range(args.dslash_reps):
        hq.dslash_apply(L64.fat, L64.lng, b, tmp, 1, DIMS, hq.HISQ_F64)
    e1.record(stream)
    e1.synchronize()
    t_dslash = e0.elapsed_time(e1) / 1e3 / args.dslash_reps
    achieved = 2400.0 * vh / t_dslash / 1e9
    # achievable HBM bandwidth on this machine: a plain 2 GiB device copy
    nbytes = 1 << 31
    cs = torch.empty(nbytes // 4, dtype=torch.float32, device=dev)
    cd = torch.empty_like(cs)
    cd.copy_(cs)
    e0.record(stream)
    for _ in range(5):
        cd.copy_(cs)
    e1.record(stream)
    e1.synchronize()
    copy_gbs = 2 * nbytes * 5 / (e0.elapsed_time(e1) / 1e3) / 1e9
    # and the achievable read rate: the library's nontemporal read stream over 4 GiB (reads dominate the Dslash)
    del cd
    rd = torch.ones(nbytes // 4 * 2, dtype=torch.float32, device=dev)
    sink = torch.empty(8192, dtype=torch.float64, device=dev)
    read_gbs = rd.numel() * 4 / hq.hisq_read_probe(rd, sink, reps=5) / 1e3
    del cs, rd, sink
    log(f"[dslash] f64 kernel {t_dslash * 1e6:.1f} us -> {achieved:.0f} GB/s; copy probe {copy_gbs:.0f} GB/s, "
        f"read probe {read_gbs:.0f} GB/s")

    forms = {"plain_f64": {"s": round(ms_per_step / 1e3, 4), "iters": stats[-1]["iters"],
                           "true_resid": stats[-1]["true_resid"]}}
    if not args.no_forms:
        for name, mode, Lhi, Llo in (("mixed_f32", hq.HISQ_CG_MIXED_F32, L64, L32),
                                     ("mixed_f16s", hq.HISQ_CG_MIXED_F16S, L64, L16),
                                     ("mixed_i16s", hq.HISQ_CG_MIXED_I16S, L64, LI16),
                                     ("plain_f64c", hq.HISQ_CG_PLAIN_F64C, L64C, None),
                                     ("mixed_f32c", hq.HISQ_CG_MIXED_F32C, L64C, L32C),
                                     ("mixed_i16sc", hq.HISQ_CG_MIXED_I16SC, L64C, LI16C)):
            wsm = hq.fields.workspace("cg", DIMS, 1, mode)
            om = hq.CGOpts(mode=mode, max_iter=0, check_every=0, use_graph=1, delta=0.0)
            xm = torch.zeros_like(b)
            lo_f, lo_l = (Llo.fat, Llo.lng) if Llo is not None else (None, None)
            hq.cg_solve(MASS, TOL, Lhi.fat, Lhi.lng, lo_f, lo_l, b, xm, DIMS, om, wsm)  # warm
            xm.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sm = hq.cg_solve(MASS, TOL, Lhi.fat, Lhi.lng, lo_f, lo_l, b, xm, DIMS, om, wsm)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            forms[name] = {"s": round(dt, 4), "iters": sm["iters"], "reliable_updates": sm["reliable_updates"],
                           "true_resid": sm["true_resid"], "speedup_vs_plain": round(ms_per_step / 1e3 / dt, 3),
                           "rc": sm["rc"], "fallback_used": sm["fallback_used"],
                           "fallback_iters": sm["fallback_iters"]}
            log(f"[form {name}] {dt:.3f}s iters={sm['iters']} updates={sm['reliable_updates']} "
                f"resid={sm['true_resid']:.2e}")
            del wsm, xm
    if not args.no_forms and not args.no_batched:
        forms["multi_rhs_8"] = form_batched(hq, DIMS, L64, L32, hq.HISQ_MULTI_RHS, 8, log)
        forms["multi_shift_8"] = form_batched(hq, DIMS, L64, L32, hq.HISQ_MULTI_SHIFT, 8, log)
        # the same with two-row long links on both levels
        forms["multi_rhs_8_f32c"] = form_batched(hq, DIMS, L64C, L32C, hq.HISQ_MULTI_RHS, 8, log,
                                                 hq.HISQ_CG_MIXED_F32C, forms["multi_rhs_8"])
        forms["multi_shift_8_f32c"] = form_batched(hq, DIMS, L64C, L32C, hq.HISQ_MULTI_SHIFT, 8, log,
                                                   hq.HISQ_CG_MIXED_F32C, forms["multi_shift_8"])
        # and with 16-bit fixed-point inner links (two-row long links)
        forms["multi_rhs_8_i16sc"] = form_batched(hq, DIMS, L64C, LI16C, hq.HISQ_MULTI_RHS, 8, log,
                                                  hq.HISQ_CG_MIXED_I16SC, forms["multi_rhs_8"])
        forms["multi_shift_8_i16sc"] = form_batched(hq, DIMS, L64C, LI16C, hq.HISQ_MULTI_SHIFT, 8, log,
                                                    hq.HISQ_CG_MIXED_I16SC, forms["multi_shift_8"])
        # 16 masses of one source (the multi-mass solve), against its 16 sequential plain FP64 solves
        forms["multi_shift_16"] = form_batched(hq, DIMS, L64, L32, hq.HISQ_MULTI_SHIFT, 16, log)
        forms["multi_shift_16_i16sc"] = form_batched(hq, DIMS, L64C, LI16C, hq.HISQ_MULTI_SHIFT, 16, log,
                                                     hq.HISQ_CG_MIXED_I16SC, forms["multi_shift_16"])
    del L16, LI16, L64C, L32C, LI16C
    torch.cuda.empty_cache()
    if not args.no_forms and not args.no_learned:
        forms["learned"] = form_learned(hq, log)
    large = None
    if not args.no_large:
        # the largest workload: its FP64 Dslash and CG kernels against the roofline, and the time to 1e-10 of
        # plain FP64 CG against the two-row FP32 and 16-bit forms
        large = large_lattice(hq, log, (hq.HISQ_F64, hq.HISQ_F64C, hq.HISQ_F32C, hq.HISQ_I16SC),
                              (("plain_f64", hq.HISQ_CG_PLAIN_F64), ("mixed_f32c", hq.HISQ_CG_MIXED_F32C),
                               ("mixed_i16sc", hq.HISQ_CG_MIXED_I16SC)))

    cpu = None
    if not args.no_cpu:
        import oracle
        # the oracle certifies the GPU solution and gives the host baseline
        tr = oracle.true_residual(DIMS, MASS, fat, lng, b_np, x_np)
        forms["plain_f64"]["oracle_true_resid"] = tr
        log(f"[cpu] oracle-recomputed residual of the GPU solution: {tr:.3e}")
        cpu = cpu_baseline(fat, lng, b_np, vh)

    traffic = cg_traffic_from_profile(vh, "k_cg_Ap_upd")
    out = {
        "metric": "Dslash GB/s (% HBM peak); CG s to 1e-10 resid, FP64 plain vs chosen form",
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "HISQ even-odd CG to 1e-10, 32^4, FP64, mass 0.01",
                   "lattice": "32x32x32x32", "mass": MASS, "tol": TOL, "global_batch": 1,
                   "seq_len": None, "parallelism": "single GPU"},
        "pct_hbm_peak": round(100 * value / HBM_PEAK_GBS, 2),
        "cg_s_to_1e-10": round(ms_per_step / 1e3, 4),
        "cg_iters": stats[-1]["iters"],
        "roofline": {"bound": "hbm", "achieved": round(ap_achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(ap_achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "kernel": "k_cg_Ap_upd<PF64> (the CG's dominant kernel: parity-0 Dslash, A p in registers, "
                               "x and r updates; 32^4)",
                     "avg_us": round(t_ap * 1e6, 2), "bytes_per_launch": AP_UPD_BYTES * vh,
                     "bytes_per_site": AP_UPD_BYTES,
                     "other_kernels": {
                         "k_cg_Dp": {"avg_us": round(t_dp * 1e6, 2), "bytes_per_site": DP_BYTES,
                                     "gbs": round(DP_BYTES * vh / t_dp / 1e9, 1),
                                     "traffic": cg_traffic_from_profile(vh, "k_cg_Dp")},
                         "k_cg_p_norm": {"avg_us": round(t_pn * 1e6, 2), "bytes_per_site": 3 * 48,
                                         "gbs": round(3 * 48 * vh / t_pn / 1e9, 1)},
                         "k_dslash_bare": {"avg_us": round(t_dslash * 1e6, 2), "bytes_per_site": 2400,
                                           "gbs": round(achieved, 1), "frac": round(achieved / HBM_PEAK_GBS, 4),
                                           "traffic": traffic_from_profile(vh, tuned["f64"]["shape"]),
                                           "gflops": round(1146.0 * vh / t_dslash / 1e9, 1)}},
                     "copy_probe_gbs": round(copy_gbs, 1), "read_probe_gbs": round(read_gbs, 1)},
        "cpu_baseline": cpu,
        "forms": forms,
        "large_48x48x48x96": large,
        "tuned_dslash_shapes": tuned,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
