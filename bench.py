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


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def dslash_source_sha():
    h = hashlib.sha256()
    for p in DSLASH_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_from_profile(vh, shape):
    """HBM bytes per Dslash launch from committed rocprofv3 counter runs, or None
    if absent or taken on another version or launch shape of the kernel."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("source_sha") != dslash_source_sha() or t.get("vh") != vh or t.get("shape") != shape:
        return None
    return t.get("bytes_per_launch")


def cpu_baseline(fat, lng, b, vh, budget_s=15.0):
    """Oracle CG on the host cores for a bounded number of iterations."""
    import numpy as np
    import oracle
    t0 = time.perf_counter()
    oracle.apply_A(DIMS, MASS, fat, lng, b)
    t_A = time.perf_counter() - t0
    n_it = int(max(2, min(2000, (budget_s - 2 * t_A) / max(t_A, 1e-3))))
    log(f"[cpu] one A application {t_A:.2f}s -> {n_it} CG iterations")
    t0 = time.perf_counter()
    _, info = oracle.cg(DIMS, MASS, fat, lng, b, tol=1e-30, max_iter=n_it)
    dt = time.perf_counter() - t0
    n_dslash = 2 * info["iters"] + 4  # initial residual, 2 per iteration, final residual
    gbs = n_dslash * 2400.0 * vh / dt / 1e9
    return {"value": round(gbs, 3), "unit": "GB/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"{info['iters']} iterations of the same 32^4 FP64 CG ({n_dslash} Dslash applications "
                      f"+ BLAS-1) in {dt:.1f} s; sustained algorithmic Dslash GB/s"}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--dslash-reps", type=int, default=100)
    ap.add_argument("--no-forms", action="store_true", help="skip the chosen-form solves")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline")
    ap.add_argument("--traffic-probe", action="store_true",
                    help="only run a 2 GiB copy and the FP64 Dslash (for rocprofv3 counter runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the path has no multi-GPU "
              "decomposition; see the design notes on sharding)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1411_2087_amd as hq
    import synth

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
        torch.cuda.synchronize()
        print(json.dumps({"traffic_probe": True, "copy_bytes": n, "dslash_launches": 5, "vh": vh, "shape": shape}))
        return

    # autotune the Dslash launch shape of each precision on this lattice
    tuned = {}
    tmp = torch.empty_like(b)
    for name, prec, L in (("f64", hq.HISQ_F64, L64), ("f32", hq.HISQ_F32, L32), ("f16s", hq.HISQ_F16S, L16),
                          ("i16s", hq.HISQ_I16S, LI16)):
        dt = hq.fields.VEC_DTYPE[prec]
        s_, d_ = b.to(dt), torch.empty(b.shape, dtype=dt, device=dev)
        best, us = hq.hisq_tune_dslash(L.fat, L.lng, s_, d_, DIMS, prec, reps=20)
        tuned[name] = {"shape": best, "us": [round(u, 1) for u in us]}
        log(f"[tune] {name}: shape {best}, us per shape {tuned[name]['us']}")
        del s_, d_

    ws = hq.fields.workspace("cg", DIMS, 1, hq.HISQ_CG_PLAIN_F64)
    opts = hq.CGOpts(mode=hq.HISQ_CG_PLAIN_F64, max_iter=0, check_every=0, use_graph=1, delta=0.1)

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
    del cs, cd
    log(f"[dslash] f64 kernel {t_dslash * 1e6:.1f} us -> {achieved:.0f} GB/s; copy probe {copy_gbs:.0f} GB/s")

    forms = {"plain_f64": {"s": round(ms_per_step / 1e3, 4), "iters": stats[-1]["iters"],
                           "true_resid": stats[-1]["true_resid"]}}
    if not args.no_forms:
        for name, mode, Llo in (("mixed_f32", hq.HISQ_CG_MIXED_F32, L32), ("mixed_f16s", hq.HISQ_CG_MIXED_F16S, L16),
                                ("mixed_i16s", hq.HISQ_CG_MIXED_I16S, LI16)):
            wsm = hq.fields.workspace("cg", DIMS, 1, mode)
            om = hq.CGOpts(mode=mode, max_iter=0, check_every=0, use_graph=1, delta=0.1)
            xm = torch.zeros_like(b)
            hq.cg_solve(MASS, TOL, L64.fat, L64.lng, Llo.fat, Llo.lng, b, xm, DIMS, om, wsm)  # warm
            xm.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sm = hq.cg_solve(MASS, TOL, L64.fat, L64.lng, Llo.fat, Llo.lng, b, xm, DIMS, om, wsm)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            forms[name] = {"s": round(dt, 4), "iters": sm["iters"], "reliable_updates": sm["reliable_updates"],
                           "true_resid": sm["true_resid"], "speedup_vs_plain": round(ms_per_step / 1e3 / dt, 3),
                           "rc": sm["rc"]}
            log(f"[form {name}] {dt:.3f}s iters={sm['iters']} updates={sm['reliable_updates']} "
                f"resid={sm['true_resid']:.2e}")
            del wsm, xm

    cpu = None
    if not args.no_cpu:
        import oracle
        # the oracle certifies the GPU solution and gives the host baseline
        tr = oracle.true_residual(DIMS, MASS, fat, lng, b_np, x_np)
        forms["plain_f64"]["oracle_true_resid"] = tr
        log(f"[cpu] oracle-recomputed residual of the GPU solution: {tr:.3e}")
        cpu = cpu_baseline(fat, lng, b_np, vh)

    traffic = traffic_from_profile(vh, tuned["f64"]["shape"])
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
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "kernel": "k_dslash<PF64> (parity 1, 32^4, tuned shape)", "avg_us": round(t_dslash * 1e6, 2),
                     "bytes_per_launch": 2400 * vh, "copy_probe_gbs": round(copy_gbs, 1),
                     "gflops": round(1146.0 * vh / t_dslash / 1e9, 1)},
        "cpu_baseline": cpu,
        "forms": forms,
        "tuned_dslash_shapes": tuned,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
