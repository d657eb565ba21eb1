"""The full-size workloads: 48^3 x 96 mixed precision (FP32 / 16-bit links inside,
FP64 reliable updates) with the FP64 Dslash checked at every site, certified by
the CPU oracle."""
import numpy as np
import pytest

from helpers import CG_TOL, TOL_F64, fields, oracle, say, synth

pytestmark = pytest.mark.gpu

DIMS = (48, 48, 48, 96)
MASS = 0.005


@pytest.fixture(scope="module")
def big():
    import torch
    import paper_1411_2087_amd as hq
    fat, lng = fields(DIMS, synth.gauge_seed(3))
    b = synth.source(DIMS, synth.source_seed(3))
    fd, ld = torch.from_numpy(fat).cuda(), torch.from_numpy(lng).cuda()
    L = {p: hq.fields.Links.pack(fd, ld, DIMS, p)
         for p in (hq.HISQ_F64, hq.HISQ_F32, hq.HISQ_F16S, hq.HISQ_I16S, hq.HISQ_F64C, hq.HISQ_F32C, hq.HISQ_I16SC)}
    del fd, ld
    torch.cuda.synchronize()
    return hq, fat, lng, b, L


def test_dslash_f64_48x96(big):
    import torch
    hq, fat, lng, b, L = big
    s = torch.from_numpy(b).cuda()
    ref = oracle.dslash(DIMS, fat, lng, b, 1)
    scale = oracle.dslash_scale(DIMS, fat, lng, b, 1)
    for prec in (hq.HISQ_F64, hq.HISQ_F64C):
        d = torch.full_like(s, float("nan"))
        hq.dslash_apply(L[prec].fat, L[prec].lng, s, d, 1, DIMS, prec)
        err = oracle.componentwise_error(d.cpu().numpy(), ref, scale)
        say(f"dslash 48^3x96 prec={prec} parity 1: componentwise {err:.2e}")
        assert err <= TOL_F64


@pytest.mark.parametrize("mode", [1, 2, 3, 5, 6])
def test_mixed_cg_48x96(big, mode):
    """Every mixed form on the largest workload, FP16-links-with-per-matrix-scale (mode 2) included;
    none may need the plain-CG fallback."""
    import torch
    hq, fat, lng, b, L = big
    lo = {1: L[hq.HISQ_F32], 2: L[hq.HISQ_F16S], 3: L[hq.HISQ_I16S], 5: L[hq.HISQ_F32C],
          6: L[hq.HISQ_I16SC]}[mode]
    hi = L[hq.HISQ_F64C] if mode in (5, 6) else L[hq.HISQ_F64]
    bd = torch.from_numpy(b).cuda()
    x = torch.zeros_like(bd)
    ws = hq.fields.workspace("cg", DIMS, 1, mode)
    opts = hq.CGOpts(mode=mode, max_iter=0, check_every=0, use_graph=1, delta=0.0)
    st = hq.cg_solve(MASS, CG_TOL, hi.fat, hi.lng, lo.fat, lo.lng, bd, x, DIMS, opts, ws)
    tr = oracle.true_residual(DIMS, MASS, fat, lng, b, x.cpu().numpy())
    say(f"48^3x96 m={MASS} mode={mode}: iters={st['iters']} updates={st['reliable_updates']} "
        f"time={st['time_s']:.2f}s gpu={st['true_resid']:.2e} oracle={tr:.2e} fallback={st['fallback_used']}")
    assert st["rc"] == 0 and tr <= CG_TOL
    assert st["fallback_used"] == 0


# The two lattices of the paper's single-coprocessor Dslash runs (Sec. 4,
# Tables 1-2): every storage form compared with the oracle at every site.
PAPER_GRIDS = [(32, 32, 32, 128), (32, 40, 24, 96)]


@pytest.mark.parametrize("dims", PAPER_GRIDS, ids=lambda d: "x".join(map(str, d)))
def test_dslash_paper_grids(dims):
    import torch
    import paper_1411_2087_amd as hq
    from helpers import TOL_F16S, TOL_F32, TOL_I16S
    fat, lng = fields(dims, synth.gauge_seed(6))
    b = synth.source(dims, synth.source_seed(6))
    ref = oracle.dslash(dims, fat, lng, b, 1)
    scale = oracle.dslash_scale(dims, fat, lng, b, 1)
    fd, ld = torch.from_numpy(fat).cuda(), torch.from_numpy(lng).cuda()
    tols = {hq.HISQ_F64: TOL_F64, hq.HISQ_F32: TOL_F32, hq.HISQ_F16S: TOL_F16S, hq.HISQ_I16S: TOL_I16S,
            hq.HISQ_F64C: TOL_F64, hq.HISQ_F32C: TOL_F32, hq.HISQ_I16SC: TOL_I16S}
    for p, tol in tols.items():
        L = hq.fields.Links.pack(fd, ld, dims, p)
        dt = hq.fields.VEC_DTYPE[p]
        s = torch.from_numpy(b).cuda().to(dt)
        d = torch.full_like(s, float("nan"))
        hq.dslash_apply(L.fat, L.lng, s, d, 1, dims, p)
        got = d.cpu().numpy().astype(np.complex128)
        err = oracle.componentwise_error(got, ref, scale)
        say(f"dslash {'x'.join(map(str, dims))} prec={p}: componentwise {err:.2e}")
        assert err <= tol
        del L, s, d
