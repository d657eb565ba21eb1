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


# (8, 6, 6, 6): x rows of 4 sites and a ragged last tile (13.5 tiles per parity)
@pytest.mark.parametrize("dims", [(6, 4, 4, 10), (8, 8, 8, 8), (8, 6, 6, 6)])
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


def _solve_multi(hq, dims, fat, lng, bs, masses, mode, max_iter=0, inner="f32", delta=0.0, shift_tol=0.0,
                 shift_only=0):
    """Batched solve with the inner links `inner` (a key of INNER) and the reliable-update trigger `delta`
    (0: the default of the inner links); for MULTI_SHIFT the shifted phase's stop `shift_tol` and,
    with shift_only, its solutions without the refinement."""
    import torch
    po, pi, cg_mode = (getattr(hq, k) for k in INNER[inner])
    L64 = hq.fields.Links.pack(fat, lng, dims, po)
    Llo = hq.fields.Links.pack(fat, lng, dims, pi)
    n = len(masses)
    b = torch.from_numpy(np.ascontiguousarray(bs)).cuda()
    vh = int(np.prod(dims)) // 2
    x = torch.zeros((n, vh, 3), dtype=torch.complex128, device="cuda")
    ws = hq.fields.workspace("cg_multi", dims, n, mode)
    opts = hq.CGOpts(mode=cg_mode, max_iter=max_iter, check_every=0, use_graph=1, delta=delta, shift_tol=shift_tol,
                     shift_only=shift_only)
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


# (lattice, shifts, inner links, lightest mass): the oracle runs one FP64 CG per shift, so the lightest
# mass (the base system) is chosen to keep that to seconds (about 1600 iterations at 8^4, m = 0.01)
SHIFT_CASES = [((8, 8, 8, 8), 4, "f32", 0.01), ((8, 8, 8, 8), 8, "f32", 0.01), ((8, 8, 8, 8), 16, "f32", 0.01),
               ((8, 8, 8, 8), 8, "f32c", 0.01), ((16, 16, 16, 16), 4, "f32", 0.02),
               ((16, 16, 16, 16), 8, "f32", 0.03), ((16, 16, 16, 16), 16, "f32", 0.05)]


def _lambda_max(dims, fat, lng, iters=40):
    """Largest eigenvalue of A0 = -D_eo D_oe (mass 0) by power iteration with the oracle's operator,
    raised by 5 % (the iteration approaches it from below)."""
    v = synth.source(dims, 999)
    lam = 0.0
    for _ in range(iters):
        w = oracle.apply_A(dims, 0.0, fat, lng, v)
        lam = np.linalg.norm(w) / np.linalg.norm(v)
        v = w / np.linalg.norm(w)
    return 1.05 * lam


U32 = 2.0 ** -24  # FP32 unit roundoff


@pytest.mark.parametrize("dims,n,inner,m_lo", SHIFT_CASES)
def test_shifted_cg_phase(hq, dims, n, inner, m_lo):
    """The shifted-CG recurrences alone (Sec. 3: multishift CG over several masses), without the
    batched refinement.  The Krylov spaces of all shifted systems coincide, so after k iterations
    shift i holds the k-th CG iterate of A(m_i) x = b from x = 0, and its residual is zeta_i times
    the base residual.  For every shift the oracle runs exactly as many CG iterations in FP64 at
    m_i as the shift did (k), and:
      (1) the oracle's recursive residual has reached shift_tol at k (within 10 %) but not 2 % of
          the iterations earlier: the shift left the phase where plain CG would;
      (2) the GPU's recursive residual |zeta_i r| / |b| equals the oracle's at k within 10 % of
          shift_tol (the zeta, alpha, beta recurrences in FP64 scalars over FP32 vectors);
      (3) the FP64 true residual of the GPU's x_i (recomputed by the oracle), and its distance to
          the oracle's k-th iterate, stay within the FP32 recursion's drift: a residual gap of
          order u32 * kappa_i, kappa_i = lambda_max / (4 m_i^2), grows over the iterations
          (Greenbaum 1997); at m = 0.002 on 8^4 it reaches ~6e-2, which is why the phase is
          followed by the FP64 reliable-update refinement.
    A wrong zeta, alpha or beta recurrence breaks (1) and (2) for every shift but the base one."""
    tol_s = 1e-4
    fat, lng = fields(dims, synth.gauge_seed(4))
    masses = synth.log_masses(n, m_lo, 0.2)
    b = synth.source(dims, synth.source_seed(4))
    x, st = _solve_multi(hq, dims, fat, lng, b, masses, hq.HISQ_MULTI_SHIFT, inner=inner, shift_tol=tol_s,
                         shift_only=1)
    lmax = _lambda_max(dims, fat, lng)
    say(f"shifted CG dims={dims} n={n}: GPU done, iterations {[s_['iters'] for s_ in st]}; lambda_max {lmax:.2f}")
    rows = []
    import time
    for i in range(n):
        m = masses[i]
        k = st[i]["iters"]
        t0 = time.perf_counter()
        tr = oracle.true_residual(dims, m, fat, lng, b, x[i])
        xk, info = oracle.cg(dims, m, fat, lng, b, tol=0.0, max_iter=k, history=True)
        say(f"  shift {i} m={m:.4f}: oracle CG of {k} iterations in {time.perf_counter() - t0:.1f}s")
        hist = info["history"]
        slack = max(2, int(np.ceil(0.02 * k)))
        dx = np.linalg.norm(x[i] - xk) / np.linalg.norm(xk)
        drift = 2 * U32 * (lmax + 4 * m * m) / (4 * m * m)
        rows.append((round(m, 5), k, f"{hist[k]:.3e}", f"{st[i]['iter_resid']:.3e}", f"{tr:.2e}", f"{dx:.1e}",
                     f"{drift:.1e}"))
        assert st[i]["status"] == 0 and st[i]["rc"] == 0 and info["iters"] == k
        assert hist[k] <= 1.1 * tol_s, (m, k, hist[k])
        if k > slack:
            assert hist[:k - slack + 1].min() > tol_s, (m, k, hist[:k - slack + 1].min())
        assert abs(st[i]["iter_resid"] - hist[k]) <= 0.1 * tol_s, (m, st[i]["iter_resid"], hist[k])
        assert tr <= tol_s + drift, (m, tr, drift)
        assert dx <= tol_s + drift, (m, dx, drift)
    say(f"shifted CG dims={dims} n={n} inner={inner} shift_tol={tol_s} lambda_max={lmax:.2f}: (m, iters, oracle "
        f"recursive residual at iters, GPU recursive residual, oracle true residual of x, |x - x_k|/|x_k|, "
        f"drift bound) = {rows}")
    # shifts converge in mass order: a heavier mass never needs more iterations
    ks = [s_["iters"] for s_ in st]
    assert all(ks[i] >= ks[i + 1] for i in range(n - 1)), ks


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


@pytest.mark.parametrize("mode", ["rhs", "shift"])
def test_cg_multi_32_4_eight_masses(hq, mode):
    """The batched configuration at its full size, as the benchmark runs it: 32^4, 8 masses log-spaced
    0.002-0.2 (the lightest needs ~19 000 iterations), FP32 inner links with FP64 reliable updates; MULTI_RHS with
    8 sources, MULTI_SHIFT with one. Every solution certified by the oracle's FP64 residual."""
    dims = (32, 32, 32, 32)
    fat, lng = fields(dims, synth.gauge_seed(4))
    n = 8
    masses = synth.log_masses(n, 0.002, 0.2)
    if mode == "rhs":
        bs = np.stack([synth.source(dims, synth.source_seed(4, r)) for r in range(n)])
        x, st = _solve_multi(hq, dims, fat, lng, bs, masses, hq.HISQ_MULTI_RHS)
    else:
        b1 = synth.source(dims, synth.source_seed(4))
        bs = np.stack([b1] * n)
        x, st = _solve_multi(hq, dims, fat, lng, b1, masses, hq.HISQ_MULTI_SHIFT)
    worst = 0.0
    for r in range(n):
        tr = oracle.true_residual(dims, masses[r], fat, lng, bs[r], x[r])
        worst = max(worst, tr)
        assert st[r]["status"] == 0 and tr <= CG_TOL, (r, tr)
    say(f"32^4 multi-{mode} 8 masses: {st[0]['time_s']:.2f}s, iterations {[s_['iters'] for s_ in st]}, "
        f"worst oracle residual {worst:.2e}")
