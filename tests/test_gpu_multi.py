"""GPU batched solves: multi-RHS Dslash parity, batched reliable-update CG and
multi-shift CG, every solution certified by the CPU oracle's FP64 residual."""
import numpy as np
import pytest

from helpers import CG_TOL, TOL_F32, fields, oracle, say, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hq():
    import torch
    import paper_1411_2087_amd as hq
    assert torch.cuda.is_available()
    return hq


@pytest.mark.parametrize("dims", [(6, 4, 4, 10), (8, 8, 8, 8)])
@pytest.mark.parametrize("nrhs", [1, 2, 4, 8, 16])
def test_dslash_multi_parity(hq, dims, nrhs):
    import torch
    fat, lng = fields(dims)
    L = hq.fields.Links.pack(fat, lng, dims, hq.HISQ_F32)
    vh = int(np.prod(dims)) // 2
    srcs = [synth.source(dims, 500 + r).astype(np.complex64).astype(np.complex128) for r in range(nrhs)]
    batched = np.stack(srcs, axis=1)  # [Vh][N][3]
    s = torch.from_numpy(batched.astype(np.complex64)).cuda().contiguous()
    ws = torch.empty(1 << 16, dtype=torch.uint8, device="cuda")
    outs = []
    for shape in range(hq.hisq_multi_shape(dims, nrhs, -2)):
        try:
            hq.hisq_multi_shape(dims, nrhs, shape)
        except hq.HisqError:
            continue
        d = torch.full_like(s, float("nan"))
        hq.hisq_dslash_multi(L.fat, L.lng, s, d, 1, nrhs, dims, ws)
        torch.cuda.synchronize()
        outs.append(d.cpu().numpy())
    for o in outs[1:]:
        assert np.array_equal(o.view(np.float32), outs[0].view(np.float32))  # every shape: same bits
    got = outs[0].astype(np.complex128)
    for r in range(nrhs):
        ref = oracle.dslash(dims, fat, lng, srcs[r], 1)
        err = oracle.componentwise_error(got[:, r], ref, oracle.dslash_scale(dims, fat, lng, srcs[r], 1))
        assert err <= TOL_F32, (r, err)
    best, us = hq.hisq_tune_multi(L.fat, L.lng, s, torch.empty_like(s), dims, nrhs, ws, reps=3)
    assert us[best] > 0
    say(f"dslash_multi dims={dims} nrhs={nrhs}: shapes {len(outs)}, tuned {best} {['%.1f' % u for u in us]} us")


# inner link storage of the batched solver: outer links, inner links, opts->mode
INNER = {"f32": ("HISQ_F64", "HISQ_F32", "HISQ_CG_MIXED_F32"),
         "f32c": ("HISQ_F64C", "HISQ_F32C", "HISQ_CG_MIXED_F32C"),  # two-row long links on both levels
         "i16s": ("HISQ_F64", "HISQ_I16S", "HISQ_CG_MIXED_I16S"),
         "i16sc": ("HISQ_F64C", "HISQ_I16SC", "HISQ_CG_MIXED_I16SC")}


def _solve_multi(hq, dims, fat, lng, bs, masses, mode, max_iter=0, inner="f32", delta=0.0):
    """Batched solve with the inner links `inner` (a key of INNER) and the reliable-update trigger `delta`
    (0: the default of the inner links)."""
    import torch
    po, pi, cg_mode = (getattr(hq, k) for k in INNER[inner])
    L64 = hq.fields.Links.pack(fat, lng, dims, po)
    Llo = hq.fields.Links.pack(fat, lng, dims, pi)
    n = len(masses)
    b = torch.from_numpy(np.ascontiguousarray(bs)).cuda()
    vh = int(np.prod(dims)) // 2
    x = torch.zeros((n, vh, 3), dtype=torch.complex128, device="cuda")
    ws = hq.fields.workspace("cg_multi", dims, n, mode)
    opts = hq.CGOpts(mode=cg_mode, max_iter=max_iter, check_every=0, use_graph=1, delta=delta)
    st = hq.cg_solve_multi(n, masses, CG_TOL, mode, L64.fat, L64.lng, Llo.fat, Llo.lng, b, x, dims, opts, ws)
    return x.cpu().numpy(), st


@pytest.mark.parametrize("n,inner", [(3, "f32"), (8, "f32"), (16, "f32"), (8, "f32c"), (8, "i16s"), (8, "i16sc")])
def test_cg_multi_rhs(hq, n, inner):
    dims = (8, 8, 8, 8)
    fat, lng = fields(dims, synth.gauge_seed(4))
    masses = synth.log_masses(n, 0.002, 0.2) if n > 1 else np.array([0.05])
    bs = np.stack([synth.source(dims, synth.source_seed(4, r)) for r in range(n)])
    if n == 3:
        bs[1] = 0.0  # a zero source inside the batch
    x, st = _solve_multi(hq, dims, fat, lng, bs, masses, hq.HISQ_MULTI_RHS, inner=inner)
    for r in range(n):
        tr = oracle.true_residual(dims, masses[r], fat, lng, bs[r], x[r]) if bs[r].any() else 0.0
        say(f"multi-rhs n={n} inner={inner} r={r} m={masses[r]:.4f}: iters={st[r]['iters']} "
            f"updates={st[r]['reliable_updates']} gpu={st[r]['true_resid']:.2e} oracle={tr:.2e}")
        assert st[r]["status"] == 0 and tr <= CG_TOL
        if not bs[r].any():
            assert not x[r].any()
    # agrees with independent single-mass solves of the oracle
    xo, _ = oracle.cg(dims, masses[0], fat, lng, bs[0], tol=1e-12)
    assert np.linalg.norm(x[0] - xo) / np.linalg.norm(xo) < 1e-6


@pytest.mark.parametrize("n,inner", [(4, "f32"), (8, "f32"), (4, "f32c"), (4, "i16sc")])
def test_cg_multi_shift(hq, n, inner):
    dims = (8, 8, 8, 8)
    fat, lng = fields(dims, synth.gauge_seed(4))
    masses = synth.log_masses(n, 0.002, 0.2)
    b = synth.source(dims, synth.source_seed(4))
    x, st = _solve_multi(hq, dims, fat, lng, b, masses, hq.HISQ_MULTI_SHIFT, inner=inner)
    for r in range(n):
        tr = oracle.true_residual(dims, masses[r], fat, lng, b, x[r])
        say(f"multi-shift n={n} inner={inner} m={masses[r]:.4f}: iters={st[r]['iters']} "
            f"updates={st[r]['reliable_updates']} oracle={tr:.2e}")
        assert st[r]["status"] == 0 and tr <= CG_TOL
    xo, _ = oracle.cg(dims, masses[-1], fat, lng, b, tol=1e-12)
    assert np.linalg.norm(x[-1] - xo) / np.linalg.norm(xo) < 1e-6


@pytest.mark.parametrize("inner,mode", [("f32", 0), ("i16sc", 0), ("f32", 1)])
def test_cg_multi_frequent_updates(hq, inner, mode):
    """delta = 0.9: reliable updates are due every few iterations for every RHS, so most
    captured runs end with several deferred updates at once (the direction of each updated
    RHS corrected by r_true - r_in); every solution is still certified by the oracle."""
    dims = (8, 8, 8, 8)
    fat, lng = fields(dims, synth.gauge_seed(4))
    n = 4
    masses = synth.log_masses(n, 0.002, 0.2)
    if mode == 0:
        bs = np.stack([synth.source(dims, synth.source_seed(4, r)) for r in range(n)])
    else:
        bs = synth.source(dims, synth.source_seed(4))
    x, st = _solve_multi(hq, dims, fat, lng, bs, masses, mode, inner=inner, delta=0.9)
    for r in range(n):
        b = bs[r] if mode == 0 else bs
        tr = oracle.true_residual(dims, masses[r], fat, lng, b, x[r])
        say(f"frequent updates inner={inner} mode={mode} m={masses[r]:.4f}: iters={st[r]['iters']} "
            f"updates={st[r]['reliable_updates']} oracle={tr:.2e}")
        assert st[r]["status"] == 0 and tr <= CG_TOL
    assert max(s_["reliable_updates"] for s_ in st) >= 20


def test_cg_multi_zero_source_and_limits(hq):
    dims = (4, 4, 4, 4)
    fat, lng = fields(dims)
    b = np.zeros((128, 3), np.complex128)
    x, st = _solve_multi(hq, dims, fat, lng, b, [0.1, 0.2], hq.HISQ_MULTI_SHIFT)
    assert all(s["status"] == 0 for s in st) and not x.any()
    bs = np.stack([synth.source(dims, 1), synth.source(dims, 2)])
    x, st = _solve_multi(hq, dims, fat, lng, bs, [0.01, 0.2], hq.HISQ_MULTI_RHS, max_iter=3)
    assert st[0]["rc"] == -5
    # half-float inner links are refused (argument check, before any launch)
    import torch
    L64 = hq.fields.Links.pack(fat, lng, dims, hq.HISQ_F64)
    LI = hq.fields.Links.pack(fat, lng, dims, hq.HISQ_F16S)
    b = torch.from_numpy(bs).cuda()
    xg = torch.zeros_like(b)
    ws = hq.fields.workspace("cg_multi", dims, 2, hq.HISQ_MULTI_RHS)
    opts = hq.CGOpts(mode=hq.HISQ_CG_MIXED_F16S, max_iter=0, check_every=0, use_graph=1, delta=0.1)
    with pytest.raises(hq.HisqError, match="HISQ_EINVAL"):
        hq.cg_solve_multi(2, [0.01, 0.2], 1e-10, hq.HISQ_MULTI_RHS, L64.fat, L64.lng, LI.fat, LI.lng, b, xg, dims,
                          opts, ws)


def test_cg_multi_16_4_timing(hq):
    """Batched N=16 on 16^4 against 16 sequential plain FP64 solves (timing printed)."""
    import time
    import torch
    dims = (16, 16, 16, 16)
    fat, lng = fields(dims, synth.gauge_seed(4))
    n = 16
    masses = synth.log_masses(n, 0.002, 0.2)
    bs = np.stack([synth.source(dims, synth.source_seed(4, r)) for r in range(n)])
    t0 = time.perf_counter()
    x, st = _solve_multi(hq, dims, fat, lng, bs, masses, hq.HISQ_MULTI_RHS)
    dt = time.perf_counter() - t0
    worst = max(oracle.true_residual(dims, masses[r], fat, lng, bs[r], x[r]) for r in range(n))
    L64 = hq.fields.Links.pack(fat, lng, dims, hq.HISQ_F64)
    ws = hq.fields.workspace("cg", dims)
    seq = 0.0
    for r in range(n):
        b = torch.from_numpy(bs[r]).cuda()
        xx = torch.zeros_like(b)
        s1 = hq.cg_solve(masses[r], CG_TOL, L64.fat, L64.lng, None, None, b, xx, dims, None, ws)
        seq += s1["time_s"]
    say(f"16^4 N=16 batched {st[0]['time_s']:.3f}s (wall {dt:.3f}s) vs sequential plain FP64 {seq:.3f}s; "
        f"worst oracle residual {worst:.2e}")
    assert worst <= CG_TOL
