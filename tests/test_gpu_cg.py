"""GPU even-odd CG (plain FP64 and mixed precision) against the CPU oracle.

Every solution's residual |b - A x| / |b| is recomputed by the FP64 CPU oracle.
"""
import numpy as np
import pytest

from helpers import CG_TOL, fields, oracle, say, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hq():
    import torch
    import paper_1411_2087_amd as hq
    assert torch.cuda.is_available()
    return hq


def _solve(hq, dims, fat, lng, b, mass, mode, tol=CG_TOL, max_iter=0, use_graph=1, check_every=0, x0=None,
           delta=0.0):
    import torch
    L64 = hq.fields.Links.pack(fat, lng, dims, hq.HISQ_F64C if mode in (4, 5, 6) else hq.HISQ_F64)
    Llo = None
    if mode == 1:
        Llo = hq.fields.Links.pack(fat, lng, dims, 1)
    elif mode in (2, 3):
        Llo = hq.fields.Links.pack(fat, lng, dims, mode)
    elif mode == 5:
        Llo = hq.fields.Links.pack(fat, lng, dims, hq.HISQ_F32C)
    elif mode == 6:
        Llo = hq.fields.Links.pack(fat, lng, dims, hq.HISQ_I16SC)
    bd = torch.from_numpy(b).cuda()
    xd = torch.zeros_like(bd) if x0 is None else torch.from_numpy(x0).cuda()
    ws = hq.fields.workspace("cg", dims, 1, mode)
    opts = hq.CGOpts(mode=mode, max_iter=max_iter, check_every=check_every, use_graph=use_graph, delta=delta)
    st = hq.cg_solve(mass, tol, L64.fat, L64.lng, Llo.fat if Llo else None, Llo.lng if Llo else None, bd, xd, dims,
                     opts, ws)
    return xd.cpu().numpy(), st


def test_cg_config1_8_4(hq):
    """Plain FP64 CG on 8^4, mass 0.05, tol 1e-10 (the small workload)."""
    dims, mass = (8, 8, 8, 8), 0.05
    fat, lng = fields(dims, synth.gauge_seed(1))
    b = synth.source(dims, synth.source_seed(1))
    x, st = _solve(hq, dims, fat, lng, b, mass, 0)
    tr = oracle.true_residual(dims, mass, fat, lng, b, x)
    xo, info = oracle.cg(dims, mass, fat, lng, b, tol=CG_TOL)
    say(f"cg 8^4: gpu iters={st['iters']} gpu_resid={st['true_resid']:.3e} oracle_resid(gpu x)={tr:.3e} "
        f"oracle iters={info['iters']} time={st['time_s']:.4f}s")
    assert st["rc"] == 0 and tr <= CG_TOL
    assert abs(st["iters"] - info["iters"]) <= max(2, 0.02 * info["iters"])
    assert np.linalg.norm(x - xo) / np.linalg.norm(xo) < 1e-7
    # the recursion's own residual at exit met tol; the byte model: per iteration two Dslashes
    # (16 FP64 matrices = 2304 B per site each) and seven FP64 vector streams, plus the initial and
    # final true residuals (two Dslash link streams and six vectors each)
    assert st["iter_resid"] <= CG_TOL
    vh = int(np.prod(dims)) // 2
    assert st["bytes_moved"] == (st["iters"] * (2 * 2304 + 7 * 48) + 2 * (2 * 2304 + 6 * 48)) * vh


@pytest.mark.parametrize("use_graph", [0, 1])
def test_cg_graph_and_direct_agree(hq, use_graph):
    dims, mass = (6, 6, 6, 6), 0.1
    fat, lng = fields(dims)
    b = synth.source(dims, 77)
    x1, s1 = _solve(hq, dims, fat, lng, b, mass, 0, use_graph=use_graph, check_every=7)
    x2, s2 = _solve(hq, dims, fat, lng, b, mass, 0, use_graph=1 - use_graph, check_every=13)
    assert s1["iters"] == s2["iters"]
    assert np.array_equal(x1, x2)  # same kernels, same order: bitwise
    assert oracle.true_residual(dims, mass, fat, lng, b, x1) <= CG_TOL


@pytest.mark.parametrize("mode", [1, 2, 3, 4, 5, 6])
def test_cg_mixed(hq, mode):
    dims, mass = (8, 8, 8, 8), 0.05
    fat, lng = fields(dims, synth.gauge_seed(1))
    b = synth.source(dims, synth.source_seed(1))
    x, st = _solve(hq, dims, fat, lng, b, mass, mode)
    tr = oracle.true_residual(dims, mass, fat, lng, b, x)
    _, info = oracle.cg(dims, mass, fat, lng, b, tol=CG_TOL)
    say(f"cg mixed mode={mode} 8^4: iters={st['iters']} updates={st['reliable_updates']} gpu_resid="
        f"{st['true_resid']:.3e} oracle_resid={tr:.3e} fallback={st['fallback_used']} "
        f"(plain oracle iters {info['iters']})")
    assert st["rc"] == 0 and tr <= CG_TOL
    assert st["fallback_used"] == 0  # the inner operator (F16S included) carries the solve to tol
    # default trigger: 0.7 for the 16-bit inner links (an update every fall by 0.7, ~65 over
    # ten decades), 0.1 otherwise (~10)
    if mode in (2, 3, 6):
        assert st["reliable_updates"] >= 30
    else:
        assert st["reliable_updates"] <= 20


@pytest.mark.parametrize("mode,delta", [(1, 0.1), (3, 0.0), (3, 0.9)])
def test_cg_mixed_falls_back_on_a_wrong_inner_operator(hq, mode, delta):
    """Inner links of another gauge field: the inner solves converge to the wrong
    answer, reliable updates stop reducing the true residual, and plain FP64 CG
    on the outer links finishes the solve (also with frequent updates, whose
    stagnation test is scaled by delta)."""
    import torch
    dims, mass = (8, 8, 8, 8), 0.05
    fat, lng = fields(dims, synth.gauge_seed(1))
    fat_w, lng_w = fields(dims, synth.gauge_seed(12))
    b = synth.source(dims, synth.source_seed(1))
    L64 = hq.fields.Links.pack(fat, lng, dims, hq.HISQ_F64)
    Lw = hq.fields.Links.pack(fat_w, lng_w, dims, hq.HISQ_F32 if mode == 1 else hq.HISQ_I16S)
    bd = torch.from_numpy(b).cuda()
    xd = torch.zeros_like(bd)
    opts = hq.CGOpts(mode=mode, max_iter=0, check_every=0, use_graph=1, delta=delta)
    st = hq.cg_solve(mass, CG_TOL, L64.fat, L64.lng, Lw.fat, Lw.lng, bd, xd, dims, opts,
                     hq.fields.workspace("cg", dims, 1, mode))
    tr = oracle.true_residual(dims, mass, fat, lng, b, xd.cpu().numpy())
    say(f"cg mixed, wrong inner links: iters={st['iters']} updates={st['reliable_updates']} "
        f"fallback={st['fallback_used']} after {st['iters'] - st['fallback_iters']} inner iterations, "
        f"oracle_resid={tr:.3e}")
    assert st["rc"] == 0 and tr <= CG_TOL
    assert st["fallback_used"] == 1 and 0 < st["fallback_iters"] < st["iters"]


def test_cg_zero_source_and_limits(hq):
    dims, mass = (4, 4, 4, 4), 0.05
    fat, lng = fields(dims)
    b = np.zeros((128, 3), np.complex128)
    x, st = _solve(hq, dims, fat, lng, b, mass, 0, x0=np.ones((128, 3), np.complex128))
    assert st["rc"] == 0 and st["iters"] == 0 and not x.any()
    b = synth.source(dims, 5)
    x, st = _solve(hq, dims, fat, lng, b, mass, 0, max_iter=1)
    assert st["rc"] == -5 and st["iters"] == 1
    # warm start from the converged solution: zero iterations
    x, st = _solve(hq, dims, fat, lng, b, mass, 0)
    x2, st2 = _solve(hq, dims, fat, lng, b, mass, 0, x0=x)
    assert st2["iters"] == 0 and st2["rc"] == 0


def test_cg_nan_source_reports_breakdown(hq):
    dims, mass = (4, 4, 4, 4), 0.05
    fat, lng = fields(dims)
    b = synth.source(dims, 5)
    b[3, 1] = np.nan
    x, st = _solve(hq, dims, fat, lng, b, mass, 0)
    assert st["rc"] in (-5, -6)


def test_cg_32_4(hq):
    """Plain FP64 CG on 32^4, mass 0.01, tol 1e-10 (the bandwidth workload)."""
    dims, mass = (32, 32, 32, 32), 0.01
    fat, lng = fields(dims, synth.gauge_seed(2))
    b = synth.source(dims, synth.source_seed(2))
    x, st = _solve(hq, dims, fat, lng, b, mass, 0)
    tr = oracle.true_residual(dims, mass, fat, lng, b, x)
    say(f"cg 32^4: iters={st['iters']} gpu_resid={st['true_resid']:.3e} oracle_resid={tr:.3e} time={st['time_s']:.3f}s")
    assert st["rc"] == 0 and tr <= CG_TOL
    for mode in (1, 3, 4, 5, 6):
        xm, sm = _solve(hq, dims, fat, lng, b, mass, mode)
        trm = oracle.true_residual(dims, mass, fat, lng, b, xm)
        say(f"cg 32^4 mode {mode}: iters={sm['iters']} updates={sm['reliable_updates']} oracle_resid={trm:.3e} "
            f"time={sm['time_s']:.3f}s fallback={sm['fallback_used']}")
        assert sm["rc"] == 0 and trm <= CG_TOL and sm["fallback_used"] == 0


@pytest.mark.parametrize("mode", [0, 1])
def test_cg_blocked_tile_order(hq, mode):
    """CG with the fused kernels in the blocked (z, t) tile order (the order of Dslash
    shapes 7 and 8): same solution to tol, certified by the oracle."""
    dims, mass = (16, 16, 16, 16), 0.02
    fat, lng = fields(dims, synth.gauge_seed(13))
    b = synth.source(dims, synth.source_seed(13))
    before = {p: hq.hisq_dslash_shape(dims, p) for p in (hq.HISQ_F64, hq.HISQ_F32)}
    x0, s0 = _solve(hq, dims, fat, lng, b, mass, mode)
    for prec in before:
        hq.hisq_dslash_shape(dims, prec, 8)
    try:
        x1, s1 = _solve(hq, dims, fat, lng, b, mass, mode)
    finally:
        for prec, shape in before.items():
            hq.hisq_dslash_shape(dims, prec, shape)
    tr = oracle.true_residual(dims, mass, fat, lng, b, x1)
    say(f"cg blocked order 16^4 mode={mode}: iters {s1['iters']} (plain order {s0['iters']}), oracle_resid={tr:.3e}")
    assert s1["rc"] == 0 and tr <= CG_TOL
    assert abs(s1["iters"] - s0["iters"]) <= 3
