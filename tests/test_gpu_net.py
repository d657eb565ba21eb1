"""GPU network kernels (transport + BF16 MFMA mixing, backward, loss, Adam) and
the flexible CG they precondition, against the CPU oracle."""
import numpy as np
import pytest

from helpers import CG_TOL, fields, oracle, say, synth
from oracle import lattice
from oracle import net as N

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hq():
    import torch
    import paper_1411_2087_amd as hq
    assert torch.cuda.is_available()
    return hq


def a256(v):
    return (v + 255) // 256 * 256


def eo_to_lex(dims, eo):
    """[C][2][Vh][3] (GPU layout) -> (C, V, 3) lex order."""
    C = eo.shape[0]
    V = int(np.prod(dims))
    out = np.zeros((C, V, 3), np.complex128)
    for p in (0, 1):
        out[:, lattice.parity_sites(dims, p)] = eo[:, p]
    return out


def acts_views(acts_np, dims, C, batch):
    """Layer inputs and output from the activation buffer (layout documented in hisq.h)."""
    vh = int(np.prod(dims)) // 2
    off = 4 * a256(32 * 288 * 2)
    chans = [1, C, C, C, 1]
    views = []
    for c in chans:
        nbytes = batch * c * 2 * vh * 3 * 8
        v = acts_np[off:off + nbytes].view(np.complex64).reshape(batch, c, 2, vh, 3)
        views.append(v.astype(np.complex128))
        off += a256(nbytes)
    return views


def rand_weights(C, seed, scale=0.4):
    r = np.random.default_rng(seed)
    Ws = []
    for co, ci in N.channels_of(C):
        Ws.append(((r.standard_normal((9, co, ci)) + 1j * r.standard_normal((9, co, ci))) * scale / np.sqrt(9 * ci)))
    return Ws


def gpu_forward(hq, dims, fat, Ws, C, bs):
    import torch
    from paper_1411_2087_amd import train
    L32 = hq.fields.Links.pack(fat, fat, dims, hq.HISQ_F32)
    w = torch.from_numpy(train.flatten([W.astype(np.complex64) for W in Ws])).cuda()
    B = len(bs)
    b = torch.from_numpy(np.stack(bs).astype(np.complex64)).cuda()
    y = torch.empty_like(b)
    acts = torch.empty(hq.net_act_bytes(dims, C, B), dtype=torch.uint8, device="cuda")
    hq.net_forward(L32.fat, w, C, b, y, acts, B, dims)
    torch.cuda.synchronize()
    return L32, w, b, y, acts


# Lattices of the layer tests: Vh = 288 ends in a half tile (ragged), Vh = 576 fills 9 tiles.
NET_DIMS = [(6, 6, 4, 4), (8, 4, 6, 6)]
TOL_MIX = 1e-5  # BF16 operands identical on both sides: only the FP32 accumulation differs


def grads_views(ws_np, dims, C, batch):
    """Per-layer gradients left in the backward workspace (layout documented in hisq.h):
    [dl/d in1, dl/d in2, dl/d in3, dl/d in4] and dl/d out, each (batch, channels, 2, Vh, 3)."""
    vh = int(np.prod(dims)) // 2
    off = 0
    gin = [None] * 4
    for l, c in ((3, C), (2, C), (1, C), (None, 1), (0, 1)):
        nbytes = batch * c * 2 * vh * 3 * 8
        v = ws_np[off:off + nbytes].view(np.complex64).reshape(batch, c, 2, vh, 3).astype(np.complex128)
        off += a256(nbytes)
        if l is None:
            gout = v
        else:
            gin[l] = v
    return gin, gout


def gpu_transport(hq, fat32_packed, feats, dims):
    """net_transport of a (batch, C, 2, Vh, 3) field: (batch, 9, C, 2, Vh, 3), the FP32 values the
    layer kernels round to BF16."""
    import torch
    B, C = feats.shape[:2]
    f = torch.from_numpy(np.ascontiguousarray(feats).astype(np.complex64)).cuda()
    out = torch.empty((B, 9) + tuple(feats.shape[1:]), dtype=torch.complex64, device="cuda")
    hq.net_transport(fat32_packed, f, out, C, B, dims)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.complex128)


def mix(W, T):
    """sum_k sum_b W[k, a, b] T[:, k, b] in FP64, for T (batch, 9, C_in, 2, Vh, 3), and the
    componentwise scale sum |W| |T| of each output."""
    out = np.einsum("kab,nkbpvc->napvc", W, T)
    scale = np.einsum("kab,nkbpvc->napvc", np.abs(W), np.abs(T))
    return out, scale


def cw_err(got, want, scale):
    return float(np.max(np.abs(got - want) / np.maximum(scale, 1e-300)))


TOL_FP32 = 1e-5  # FP32 products and sums of 16 channels and a 3x3 link: ~22 roundings of 2^-24


def fp32_layer_ref(dims, fat, W, feats):
    """The C -> 1 layer as the GPU computes it, in FP32 without BF16 operands: FP64
    out = sum_k sum_c W_k^c T_k x^c over the FP32-rounded weights and links, and the
    componentwise scale sum_k |T_k| (sum_c |W_k^c| |x^c|) (entrywise absolute links) that
    bounds its rounding.  feats: (batch, C, 2, Vh, 3); W: [9][1][C].  Returns (batch, 1, 2, Vh, 3)."""
    W32 = W.astype(np.complex64).astype(np.complex128)
    f32 = fat.astype(np.complex64).astype(np.complex128)
    afat = np.abs(f32)
    vh = int(np.prod(dims)) // 2
    outs, scales = [], []
    for n in range(feats.shape[0]):
        X = eo_to_lex(dims, feats[n])
        o = np.zeros(X.shape[1:], np.complex128)
        sc = np.zeros(X.shape[1:])
        for k in range(9):
            o += N.transport(dims, f32, np.einsum("c,cvs->vs", W32[k, 0], X), k)
            sc += N.transport(dims, afat, np.einsum("c,cvs->vs", np.abs(W32[k, 0]), np.abs(X)), k).real
        oe = np.zeros((1, 2, vh, 3), np.complex128)
        se = np.zeros((1, 2, vh, 3))
        for p in (0, 1):
            oe[0, p] = o[lattice.parity_sites(dims, p)]
            se[0, p] = sc[lattice.parity_sites(dims, p)]
        outs.append(oe)
        scales.append(se)
    return np.stack(outs), np.stack(scales)


@pytest.mark.parametrize("C", [4, 16])
@pytest.mark.parametrize("dims", NET_DIMS)
def test_net_transport(hq, C, dims):
    """The FP32 parallel transports against the FP64 oracle, componentwise at the FP32
    tolerance (scale sum_b |M_ab| |phi_b|, the links rounded to FP32 as the kernels read them)."""
    from helpers import TOL_F32
    fat, _ = fields(dims, 1000)
    L32 = hq.fields.Links.pack(fat, fat, dims, hq.HISQ_F32)
    r = np.random.default_rng(11)
    vh = int(np.prod(dims)) // 2
    x = (r.standard_normal((2, C, 2, vh, 3)) + 1j * r.standard_normal((2, C, 2, vh, 3))).astype(np.complex64)
    T = gpu_transport(hq, L32.fat, x, dims)
    fat32 = fat.astype(np.complex64).astype(np.complex128)
    worst = 0.0
    for bi in range(2):
        xl = eo_to_lex(dims, x[bi].astype(np.complex128))
        for k in range(9):
            got = eo_to_lex(dims, T[bi, k])
            for c in range(C):
                want = N.transport(dims, fat32, xl[c], k)
                scale = N.transport(dims, np.abs(fat32), np.abs(xl[c]), k)
                e = cw_err(got[c], want, scale)
                worst = max(worst, e)
                if k == 0:
                    assert np.array_equal(got[c], xl[c])
    say(f"net transport C={C} dims={dims}: componentwise {worst:.2e}")
    assert worst <= TOL_F32


@pytest.mark.parametrize("C", [4, 8, 16])
@pytest.mark.parametrize("dims", NET_DIMS)
def test_net_forward_layers(hq, C, dims):
    """Layers 1-3 against the FP64 mixing of the very BF16 operands the MFMA used: the
    GPU's own layer input, transported by the same device code (net_transport) and rounded
    to BF16 (round to nearest even, as the kernels convert), and the BF16-rounded weights;
    componentwise within TOL_MIX of sum |W| |T phi|: only the FP32 accumulation differs.  The
    C -> 1 layer (mixed in FP32, then transported) against the FP64 layer over the FP32 weights
    and links, componentwise within TOL_FP32.  The network output is the even part of the last
    layer, bit for bit."""
    fat, _ = fields(dims, 1000)
    Ws = rand_weights(C, 3)
    bs = [synth.source(dims, 60 + i) for i in range(2)]
    L32, w, b, y, acts = gpu_forward(hq, dims, fat, Ws, C, bs)
    views = acts_views(acts.cpu().numpy(), dims, C, 2)
    worst = 0.0
    for l in range(3):
        Tb = N._bf16c(gpu_transport(hq, L32.fat, views[l], dims).astype(np.complex64))
        Wb = N._bf16c(Ws[l].astype(np.complex64))
        want, scale = mix(Wb, Tb)
        e = cw_err(views[l + 1], want, scale)
        worst = max(worst, e)
        assert e <= TOL_MIX, (l, e)
    want, scale = fp32_layer_ref(dims, fat, Ws[3], views[3])
    e3 = cw_err(views[4], want, scale)
    assert e3 <= TOL_FP32, e3
    assert np.array_equal(y.cpu().numpy(), views[4][:, 0, 0].astype(np.complex64))
    # the first layer's input is the embedded source (odd sites zero)
    assert np.array_equal(views[0][:, 0, 0], np.stack(bs).astype(np.complex64).astype(np.complex128))
    assert not views[0][:, 0, 1].any()
    # end to end against pure FP64 (reported; BF16 rounding of every operand)
    ye, _ = N.net_forward(dims, fat, Ws, bs[0])
    e2e = np.linalg.norm(y.cpu().numpy()[0] - ye) / np.linalg.norm(ye)
    say(f"net forward C={C} dims={dims}: layers 1-3 vs BF16-operand FP64 mixing {worst:.2e}, layer 4 vs FP64 "
        f"{e3:.2e} (componentwise); end-to-end vs FP64 {e2e:.2e}")
    assert e2e < 5e-2


@pytest.mark.parametrize("C", [4, 8, 16])
@pytest.mark.parametrize("dims", NET_DIMS)
def test_net_backward(hq, C, dims):
    """Every layer's weight gradient and input gradient against FP64 sums of the BF16 operands
    the GPU used, componentwise within TOL_MIX, with x the GPU's layer input (acts) and g the
    GPU's upstream gradient (left in the workspace): dl/dx^c = sum_k sum_a
    bf16(conj(W_{adj k}^{ac})) bf16(T_k g^a) for layers 2-4, and for the first layer (its
    adjoint is a C -> 1 layer, mixed in FP32, then transported) the FP64 value over the FP32
    weights and links within TOL_FP32; the first layer's weight gradient
    dW_k^{ac} = sum conj(bf16(T_k x^c)) bf16(g^a), and that of layers 2-4, taken from the same
    transports of g as their input gradient, sum conj(bf16(x^c)) bf16(T_{adj k} g^a) (equal in
    exact arithmetic, T_k^dag = T_{adj k}).  The returned dl/d input is the even part of the
    first layer's input gradient, bit for bit."""
    import torch
    from paper_1411_2087_amd import train
    fat, _ = fields(dims, 1000)
    Ws = rand_weights(C, 5)
    B = 2
    bs = [synth.source(dims, 70 + i) for i in range(B)]
    L32, w, b, y, acts = gpu_forward(hq, dims, fat, Ws, C, bs)
    g = np.stack([synth.source(dims, 80 + i) for i in range(B)]).astype(np.complex64)
    gd = torch.from_numpy(g).cuda()
    gw = torch.zeros(hq.net_weight_count(C), dtype=torch.complex64, device="cuda")
    gin = torch.empty_like(gd)
    ws = torch.empty(hq.net_backward_ws_bytes(dims, C, B), dtype=torch.uint8, device="cuda")
    hq.net_backward(L32.fat, w, C, acts, gd, gw, gin, B, dims, ws)
    torch.cuda.synchronize()
    gws = train.unflatten(gw.cpu().numpy(), C)
    views = acts_views(acts.cpu().numpy(), dims, C, B)
    ginv, goutv = grads_views(ws.cpu().numpy(), dims, C, B)
    # the embedded output gradient: even part = grad_out, odd part zero
    assert np.array_equal(goutv[:, 0, 0], g.astype(np.complex128)) and not goutv[:, 0, 1].any()
    ups = [ginv[1], ginv[2], ginv[3], goutv]  # dl/d (output of layer l)
    ew, ex = [], []
    for l in range(4):
        Tg = N._bf16c(gpu_transport(hq, L32.fat, ups[l], dims).astype(np.complex64))
        if l == 0:
            gb = N._bf16c(ups[l].astype(np.complex64))
            Tx = N._bf16c(gpu_transport(hq, L32.fat, views[l], dims).astype(np.complex64))
            want = np.einsum("nkcpvs,napvs->kac", Tx.conj(), gb)
            scale = np.einsum("nkcpvs,napvs->kac", np.abs(Tx), np.abs(gb))
        else:
            xb = N._bf16c(views[l].astype(np.complex64))
            Tga = Tg[:, N.ADJOINT]
            want = np.einsum("ncpvs,nkapvs->kac", xb.conj(), Tga)
            scale = np.einsum("ncpvs,nkapvs->kac", np.abs(xb), np.abs(Tga))
        ew.append(cw_err(gws[l], want, scale))
        # input gradient: the adjoint layer on the upstream gradient
        if l == 0:
            Wadj = np.stack([np.conj(Ws[l][N.ADJOINT[k]]).T for k in range(9)])
            want_x, scale_x = fp32_layer_ref(dims, fat, Wadj, ups[l])
            ex0 = cw_err(ginv[l], want_x, scale_x)
            assert ex0 <= TOL_FP32, ex0
            ex.append(ex0)
        else:
            Wadj = N._bf16c(np.stack([np.conj(Ws[l][N.ADJOINT[k]]).T for k in range(9)]).astype(np.complex64))
            want_x, scale_x = mix(Wadj, Tg)
            ex.append(cw_err(ginv[l], want_x, scale_x))
    say(f"net backward C={C} dims={dims}: dW per layer {['%.1e' % v for v in ew]}, "
        f"d input per layer {['%.1e' % v for v in ex]} (componentwise, BF16 operands)")
    assert max(ew) <= TOL_MIX and max(ex[1:]) <= TOL_MIX
    assert np.array_equal(gin.cpu().numpy(), ginv[0][:, 0, 0].astype(np.complex64))


def test_net_many_units(hq):
    """The network on large grids: 8^4 with a batch of 32 gives 2048 (batch entry, tile, parity) units, one
    workgroup each in the layer kernels and two to three per resident workgroup of the persistent k_net_bwd
    and k_net_wgrad (the training shape runs ~21).  Every layer output, weight gradient and input gradient
    against the same BF16-operand (and, for the C -> 1 kernel, FP32) FP64 references as test_net_forward_layers
    and test_net_backward, componentwise; the sums over the batch are accumulated entry by entry."""
    import torch
    from paper_1411_2087_amd import train
    dims, C, B = (8, 8, 8, 8), 16, 32
    fat, _ = fields(dims, 1001)
    Ws = rand_weights(C, 6)
    bs = [synth.source(dims, 90 + i) for i in range(B)]
    L32, w, b, y, acts = gpu_forward(hq, dims, fat, Ws, C, bs)
    g = np.stack([synth.source(dims, 130 + i) for i in range(B)]).astype(np.complex64)
    gd = torch.from_numpy(g).cuda()
    gw = torch.zeros(hq.net_weight_count(C), dtype=torch.complex64, device="cuda")
    gin = torch.empty_like(gd)
    ws = torch.empty(hq.net_backward_ws_bytes(dims, C, B), dtype=torch.uint8, device="cuda")
    hq.net_backward(L32.fat, w, C, acts, gd, gw, gin, B, dims, ws)
    torch.cuda.synchronize()
    gws = train.unflatten(gw.cpu().numpy(), C)
    views = acts_views(acts.cpu().numpy(), dims, C, B)
    ginv, goutv = grads_views(ws.cpu().numpy(), dims, C, B)
    # the forward layers on the same 2048-workgroup grids
    ef = []
    for l in range(4):
        e_l = 0.0
        for n in range(B):
            if l < 3:
                Tb = N._bf16c(gpu_transport(hq, L32.fat, views[l][n:n + 1], dims).astype(np.complex64))
                Wb = N._bf16c(Ws[l].astype(np.complex64))
                wf = np.einsum("kab,nkbpvc->napvc", Wb, Tb, optimize=True)
                sf = np.einsum("kab,nkbpvc->napvc", np.abs(Wb), np.abs(Tb), optimize=True)
            else:
                wf, sf = fp32_layer_ref(dims, fat, Ws[3], views[3][n:n + 1])
            e_l = max(e_l, cw_err(views[l + 1][n:n + 1], wf, sf))
        ef.append(e_l)
    ups = [ginv[1], ginv[2], ginv[3], goutv]
    ew, ex = [], []
    for l in range(4):
        want = np.zeros(gws[l].shape, np.complex128)
        scale = np.zeros(gws[l].shape)
        ex_l = 0.0
        Wadj = np.stack([np.conj(Ws[l][N.ADJOINT[k]]).T for k in range(9)])
        Wadj_b = N._bf16c(Wadj.astype(np.complex64))
        for n in range(B):
            un = ups[l][n:n + 1]
            Tg = N._bf16c(gpu_transport(hq, L32.fat, un, dims).astype(np.complex64))
            if l == 0:
                gb = N._bf16c(un.astype(np.complex64))
                Tx = N._bf16c(gpu_transport(hq, L32.fat, views[l][n:n + 1], dims).astype(np.complex64))
                want += np.einsum("nkcpvs,napvs->kac", Tx.conj(), gb, optimize=True)
                scale += np.einsum("nkcpvs,napvs->kac", np.abs(Tx), np.abs(gb), optimize=True)
                wx, sx = fp32_layer_ref(dims, fat, Wadj, un)
                ex_l = max(ex_l, cw_err(ginv[l][n:n + 1], wx, sx))
            else:
                xb = N._bf16c(views[l][n:n + 1].astype(np.complex64))
                Tga = Tg[:, N.ADJOINT]
                want += np.einsum("ncpvs,nkapvs->kac", xb.conj(), Tga, optimize=True)
                scale += np.einsum("ncpvs,nkapvs->kac", np.abs(xb), np.abs(Tga), optimize=True)
                wx = np.einsum("kab,nkbpvc->napvc", Wadj_b, Tg, optimize=True)
                sx = np.einsum("kab,nkbpvc->napvc", np.abs(Wadj_b), np.abs(Tg), optimize=True)
                ex_l = max(ex_l, cw_err(ginv[l][n:n + 1], wx, sx))
        ew.append(cw_err(gws[l], want, scale))
        ex.append(ex_l)
    say(f"net, 8^4 x 32 (several units per workgroup): forward per layer {['%.1e' % v for v in ef]}, "
        f"dW per layer {['%.1e' % v for v in ew]}, d input per layer {['%.1e' % v for v in ex]} (componentwise)")
    assert max(ef[:3]) <= TOL_MIX and ef[3] <= TOL_FP32
    assert max(ew) <= TOL_MIX and max(ex[1:]) <= TOL_MIX and ex[0] <= TOL_FP32


def test_net_loss_and_adam(hq):
    import torch
    dims = (4, 4, 4, 6)
    vh = 192
    r = np.random.default_rng(1)
    y = (r.standard_normal((3, vh, 3)) + 1j * r.standard_normal((3, vh, 3))).astype(np.complex64)
    x = (r.standard_normal((3, vh, 3)) + 1j * r.standard_normal((3, vh, 3))).astype(np.complex64)
    yd, xd = torch.from_numpy(y).cuda(), torch.from_numpy(x).cuda()
    gd = torch.empty_like(yd)
    ws = torch.empty(1 << 16, dtype=torch.uint8, device="cuda")
    loss = hq.net_loss(yd, xd, 3, dims, gd, ws)
    lo, gr = N.loss_and_grad(list(y.astype(np.complex128)), list(x.astype(np.complex128)))
    assert abs(loss - lo) < 1e-12 * lo
    assert np.abs(gd.cpu().numpy() - np.stack(gr)).max() < 1e-6 * np.abs(np.stack(gr)).max()
    # Adam: two steps against the oracle's
    n = 50
    w = (r.standard_normal(n) + 1j * r.standard_normal(n))
    g1 = (r.standard_normal(n) + 1j * r.standard_normal(n))
    g2 = (r.standard_normal(n) + 1j * r.standard_normal(n))
    wd = torch.from_numpy(w.astype(np.complex64)).cuda()
    m = torch.zeros(2 * n, dtype=torch.float32, device="cuda")
    v = torch.zeros_like(m)
    wo, mo, vo = [w.copy()], [np.zeros(n, complex)], [np.zeros(n, complex)]
    for t, gg in ((1, g1), (2, g2)):
        hq.net_adam_step(wd, torch.from_numpy(gg.astype(np.complex64)).cuda(), m, v, n, 1e-2, t)
        N.adam_step(wo, [gg.astype(np.complex64).astype(complex)], mo, vo, t, 1e-2)
    assert np.abs(wd.cpu().numpy() - wo[0]).max() < 1e-5


def test_training_reduces_loss(hq):
    """Both objectives run on the GPU kernels; the residual (approximate-inverse) objective learns.  The error
    objective |K b - x|^2 / |x|^2 is dominated by the low modes a four-hop network cannot represent and is not
    claimed to decrease (reported only)."""
    import torch
    from paper_1411_2087_amd import train
    dims, mass, C = (8, 8, 8, 8), 0.05, 8
    fat, lng = fields(dims, synth.gauge_seed(5))
    L64 = hq.fields.Links.pack(fat, lng, dims, hq.HISQ_F64)
    L32 = hq.fields.Links.pack(fat, lng, dims, hq.HISQ_F32)
    src = np.stack([synth.source(dims, synth.source_seed(5, i)) for i in range(64)])
    b, x, secs, x64 = train.make_pairs(dims, mass, L64, L32, src)
    # the pairs solve A x = b (oracle check on two of them)
    for i in (0, 63):
        assert oracle.true_residual(dims, mass, fat, lng, src[i], x64[i].cpu().numpy()) < 1e-8
    sr = train.residual_scale(b[:16], L32, mass, dims)
    tr = train.Trainer(dims, C, L32.fat, train.initial_weights(C, sr, 0.05, 99), batch=16, objective="residual",
                       links32=L32, mass=mass)
    l0 = tr.evaluate(b[48:], x[48:])
    hist = tr.fit(b[:48], x[:48], steps=200, lr=2e-3, log_every=50)
    l1 = tr.evaluate(b[48:], x[48:])
    s = train.least_squares_scale(b, x)
    te = train.Trainer(dims, C, L32.fat, train.initial_weights(C, s, 0.05, 99), batch=16)
    e0 = te.evaluate(b[48:], x[48:])
    te.fit(b[:48], x[:48], steps=100, lr=2e-3, log_every=50)
    e1 = te.evaluate(b[48:], x[48:])
    say(f"training 8^4 C={C}: residual objective held-out {l0:.4f} -> {l1:.4f} "
        f"(log {[(s_, round(l, 4)) for s_, l in hist]}); error objective {e0:.4f} -> {e1:.4f}")
    assert l1 < 0.7 * l0
    assert np.isfinite(e1)


def test_fcg_trained_gain_16_4(hq):
    """Learned-preconditioner workload on 16^4, m = 0.005: pairs from the batched CG, training on the GPU with
    the residual objective, then flexible CG on held-out sources against plain FP64 CG and against flexible CG
    with K = identity.  What is established (parity of the gain itself unpinned): every solution is certified
    by the oracle; K = 1 tracks plain CG within 1 %; the trained network does not cut the iteration count by
    more than 10 % (measured 1.0-2.1 times plain CG's iterations, by width and training length: the residual
    objective fits the bulk of the spectrum, not its low end, and the fat-link layers cannot reach the three-hop
    terms of the operator)."""
    import torch
    from paper_1411_2087_amd import train
    dims, mass, C = (16, 16, 16, 16), 0.005, 16
    fat, lng = fields(dims, synth.gauge_seed(5))
    L64 = hq.fields.Links.pack(fat, lng, dims, hq.HISQ_F64)
    L32 = hq.fields.Links.pack(fat, lng, dims, hq.HISQ_F32)
    src = np.stack([synth.source(dims, synth.source_seed(5, i)) for i in range(64 + 2)])
    b, x, secs, _ = train.make_pairs(dims, mass, L64, L32, src[:64])
    tr = train.Trainer(dims, C, L32.fat, train.initial_weights(C, train.residual_scale(b[:16], L32, mass, dims),
                                                               0.05, 99), batch=16, objective="residual",
                       links32=L32, mass=mass)
    hist = tr.fit(b, x, steps=300, lr=2e-3, log_every=100)
    w = tr.w.cpu().numpy()
    ws_c = hq.fields.workspace("cg", dims)
    rows = []
    for i in (64, 65):
        _, stc = _cg_plain(hq, dims, mass, L64, src[i], ws_c)
        xf, stf = _fcg(hq, dims, mass, fat, lng, src[i], w, C)
        xi, sti = _fcg(hq, dims, mass, fat, lng, src[i], train.flatten(train.identity_weights(C)), C)
        tr_res = oracle.true_residual(dims, mass, fat, lng, src[i], xf)
        rows.append((stc["iters"], round(stc["time_s"], 3), sti["iters"], stf["iters"], stf["fallback_used"],
                     stf["fallback_iters"], round(stf["time_s"], 3), tr_res))
        assert stf["rc"] == 0 and tr_res <= CG_TOL
        assert oracle.true_residual(dims, mass, fat, lng, src[i], xi) <= CG_TOL
        assert abs(sti["iters"] - stc["iters"]) <= 0.01 * stc["iters"]
        assert stf["iters"] >= 0.9 * stc["iters"]
    say(f"learned 16^4 m={mass} C={C}: pairs {secs:.1f}s, train log {[(s_, round(l, 4)) for s_, l in hist]}; "
        f"(plain iters, plain s, K=1 iters, fcg iters, fallback, fallback iters, fcg s, resid) = {rows}")


def test_fcg_trained_gain_naive(hq):
    """What a trained network gains where the fat-link layers can represent a good K: the naive operator (long
    links zero), 16^4, m = 0.005, C = 8.  The residual objective over a shuffled mix of 128 Gaussian sources and
    128 normalised solutions x = A^-1 b (Gaussian sources alone weight the bulk of the spectrum and give
    1.9-2.6x plain CG's iterations), 1500 Adam steps: flexible CG with the trained network needs fewer iterations
    than plain CG (measured 2474-2479 against 3958, 0.63x; asserted below 0.8x), every solution certified by the
    oracle.  It is still slower in time (each iteration applies the network), and the same recipe on the HISQ
    operator gives 1.3-3.3x: the layers cannot reach its three-hop terms."""
    import torch
    from paper_1411_2087_amd import train
    dims, mass, C, npairs = (16, 16, 16, 16), 0.005, 8, 256
    fat, lng = fields(dims, synth.gauge_seed(5))
    lng0 = np.zeros_like(lng)
    L64 = hq.fields.Links.pack(fat, lng0, dims, hq.HISQ_F64)
    L32 = hq.fields.Links.pack(fat, lng0, dims, hq.HISQ_F32)
    src = np.stack([synth.source(dims, synth.source_seed(5, i)) for i in range(npairs + 2)])
    b, x, secs, _ = train.make_pairs(dims, mass, L64, L32, src[:npairs])
    nb = torch.linalg.vector_norm(b.reshape(npairs, -1), dim=1).reshape(-1, 1, 1)
    xn = x / torch.linalg.vector_norm(x.reshape(npairs, -1), dim=1).reshape(-1, 1, 1) * nb
    k = npairs // 2
    perm = torch.randperm(npairs, generator=torch.Generator().manual_seed(4)).cuda()
    inp = torch.cat([b[:npairs - k], xn[:k]])[perm]
    w0 = train.initial_weights(C, train.residual_scale(inp[:16], L32, mass, dims), 0.05, 99)
    tr = train.Trainer(dims, C, L32.fat, w0, batch=16, objective="residual", links32=L32, mass=mass)
    hist = tr.fit(inp[:-32], inp[:-32], steps=1500, lr=2e-3, log_every=300)
    w = tr.w.cpu().numpy()
    ws_c = hq.fields.workspace("cg", dims)
    rows = []
    for i in (npairs, npairs + 1):
        _, stc = _cg_plain(hq, dims, mass, L64, src[i], ws_c)
        xf, stf = _fcg(hq, dims, mass, fat, lng0, src[i], w, C)
        tr_res = oracle.true_residual(dims, mass, fat, lng0, src[i], xf)
        rows.append((stc["iters"], round(stc["time_s"], 3), stf["iters"], stf["fallback_used"], stf["fallback_iters"],
                     round(stf["time_s"], 3), tr_res))
        assert stf["rc"] == 0 and tr_res <= CG_TOL
        assert stf["iters"] < 0.8 * stc["iters"]
    say(f"trained on the naive operator 16^4 m={mass} C={C}: pairs {secs:.1f}s, train log "
        f"{[(s_, round(l, 4)) for s_, l in hist]}; (plain iters, plain s, fcg iters, fallback, fallback iters, "
        f"fcg s, resid) = {rows}")


def test_polynomial_network_naive(hq):
    """The reach of the architecture.  With the long links zero, the four fat-link layers represent any quadratic
    p(A) exactly; train.chebyshev_weights builds the one that minimises max |1 - l p(l)| on [lambda_max / 30,
    lambda_max] (which keeps K well away from singular under BF16 rounding).  The network's K b matches the
    oracle's p(A) b (FP64 operator; BF16 weights and features in the network: measured 5e-3, bound 2e-2), and
    flexible CG with this K needs less than half of plain CG's iterations (16^4, m = 0.005; plain CG 3956-3965),
    every solution certified."""
    import torch
    from paper_1411_2087_amd import train
    dims, mass, C = (16, 16, 16, 16), 0.005, 4
    fat, lng = fields(dims, synth.gauge_seed(5))
    lng0 = np.zeros_like(lng)
    L64 = hq.fields.Links.pack(fat, lng0, dims, hq.HISQ_F64)
    L32 = hq.fields.Links.pack(fat, lng0, dims, hq.HISQ_F32)
    lmax = train.lambda_max_estimate(L64, mass, dims)
    w, (c0, c1, c2) = train.chebyshev_weights(C, mass, lmax)
    b = synth.source(dims, synth.source_seed(5, 600))
    bd = torch.from_numpy(b.astype(np.complex64)).cuda().unsqueeze(0).contiguous()
    y = torch.empty_like(bd)
    acts = torch.empty(hq.net_act_bytes(dims, C, 1), dtype=torch.uint8, device="cuda")
    hq.net_forward(L32.fat, torch.from_numpy(w).cuda(), C, bd, y, acts, 1, dims)
    ab = oracle.apply_A(dims, mass, fat, lng0, b)
    want = c0 * b + c1 * ab + c2 * oracle.apply_A(dims, mass, fat, lng0, ab)
    rel = np.linalg.norm(y.cpu().numpy()[0] - want) / np.linalg.norm(want)
    assert rel < 2e-2, rel
    ws_c = hq.fields.workspace("cg", dims)
    rows = []
    for i in (600, 601):
        src = synth.source(dims, synth.source_seed(5, i))
        _, stc = _cg_plain(hq, dims, mass, L64, src, ws_c)
        xf, stf = _fcg(hq, dims, mass, fat, lng0, src, w, C)
        tr_res = oracle.true_residual(dims, mass, fat, lng0, src, xf)
        rows.append((stc["iters"], round(stc["time_s"], 3), stf["iters"], stf["fallback_used"], round(stf["time_s"], 3),
                     tr_res))
        say(f"polynomial network: lambda_max {lmax:.4f}, K b vs p(A) b {rel:.2e}, source {i}: plain {stc}, fcg {stf}")
        assert stf["rc"] == 0 and tr_res <= CG_TOL
        assert stf["iters"] < 0.5 * stc["iters"]
    say(f"polynomial network, naive operator 16^4 m={mass}: lambda_max {lmax:.3f}, p = {c0:.4f} + {c1:.4f} A + "
        f"{c2:.5f} A^2, K b vs oracle p(A) b {rel:.2e}; (plain iters, plain s, fcg iters, fallback, fcg s, resid) "
        f"= {rows}")


def _cg_plain(hq, dims, mass, L64, b, ws):
    import torch
    bd = torch.from_numpy(b).cuda()
    xd = torch.zeros_like(bd)
    st = hq.cg_solve(mass, CG_TOL, L64.fat, L64.lng, None, None, bd, xd, dims, None, ws)
    return xd.cpu().numpy(), st


def _fcg(hq, dims, mass, fat, lng, b, w, C, max_iter=0):
    import torch
    L64 = hq.fields.Links.pack(fat, lng, dims, hq.HISQ_F64)
    L32 = hq.fields.Links.pack(fat, lng, dims, hq.HISQ_F32)
    bd = torch.from_numpy(b).cuda()
    xd = torch.zeros_like(bd)
    ws = hq.fields.workspace("fcg", dims, 1, 0, C)
    wd = torch.from_numpy(w.astype(np.complex64)).cuda()
    opts = hq.CGOpts(mode=0, max_iter=max_iter, check_every=0, use_graph=1, delta=0.1)
    st = hq.fcg_solve(mass, CG_TOL, L64.fat, L64.lng, L32.fat, wd, C, bd, xd, dims, opts, ws)
    return xd.cpu().numpy(), st


def test_fcg_identity_is_cg(hq):
    from paper_1411_2087_amd import train
    dims, mass, C = (8, 8, 8, 8), 0.05, 4
    fat, lng = fields(dims, synth.gauge_seed(1))
    b = synth.source(dims, synth.source_seed(1))
    x, st = _fcg(hq, dims, mass, fat, lng, b, train.flatten(train.identity_weights(C)), C)
    tr = oracle.true_residual(dims, mass, fat, lng, b, x)
    _, info = oracle.cg(dims, mass, fat, lng, b, tol=CG_TOL)
    say(f"fcg K=1: iters={st['iters']} fallback={st['fallback_used']} oracle resid={tr:.2e}; plain CG {info['iters']}")
    assert st["rc"] == 0 and tr <= CG_TOL
    # K = 1 up to the BF16 rounding of the mixing operands: FCG tracks CG
    assert abs(st["iters"] - info["iters"]) <= max(3, 0.10 * info["iters"])


def test_fcg_falls_back_on_a_bad_network(hq):
    from paper_1411_2087_amd import train
    dims, mass, C = (8, 8, 8, 8), 0.05, 4
    fat, lng = fields(dims, synth.gauge_seed(1))
    b = synth.source(dims, synth.source_seed(1))
    x, st = _fcg(hq, dims, mass, fat, lng, b, train.flatten(train.identity_weights(C, scale=-1.0)), C)
    assert st["fallback_used"] == 1 and st["rc"] == 0
    assert oracle.true_residual(dims, mass, fat, lng, b, x) <= CG_TOL
    w = train.flatten(train.identity_weights(C))
    w[3] = np.nan
    x, st = _fcg(hq, dims, mass, fat, lng, b, w, C)
    assert st["fallback_used"] in (1, 2) and st["rc"] == 0
    assert oracle.true_residual(dims, mass, fat, lng, b, x) <= CG_TOL
