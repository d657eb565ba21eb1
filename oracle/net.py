"""Gauge-covariant linear network: FP64 reference (test infrastructure only).

A parallel-transport convolution layer maps C_in colour-vector fields on the
full lattice to C_out fields:

    out^a(x) = sum_b sum_{k=0..8} W_k^{ab} (T_k in^b)(x)

with T_0 = 1, T_{+mu} phi(x) = F_mu(x) phi(x + mu), T_{-mu} phi(x) =
F_mu(x - mu)^dag phi(x - mu), F the folded fat links (the one-link field of
the paper's operator, Sec. 3) and W complex scalars, so every layer commutes
with gauge transformations.  The network has four such layers with channels
1 -> C -> C -> C -> 1 and no nonlinearity.  Acting on an even-site vector r_e
it embeds r_e on the full lattice (odd sites zero) and returns the even part
of the last layer's output: K(r_e).

Gradients use the convention dl/dz = dl/dRe z + i dl/dIm z for every complex
quantity z.  For out = sum_k W_k T_k in:
    dl/dW_k^{ab} = sum_x <(T_k in^b)(x), g^a(x)>          (<u,v> = u^dag v)
    dl/din^b     = sum_{k,a} conj(W_k^{ab}) T_k^dag g^a,   T_{+mu}^dag = T_{-mu}.
"""
from __future__ import annotations

import numpy as np

from . import lattice

N_TRANSPORT = 9
ADJOINT = [0, 5, 6, 7, 8, 1, 2, 3, 4]   # T_k^dag = T_ADJOINT[k]


def _grid(dims, phi):
    Lx, Ly, Lz, Lt = dims
    return phi.reshape(Lt, Lz, Ly, Lx, 3)


AXIS = {0: 3, 1: 2, 2: 1, 3: 0}          # lattice direction -> axis of the (t,z,y,x) grid


def transport(dims, fat, phi, k):
    """(T_k phi) for a full-lattice field phi (V, 3)."""
    if k == 0:
        return phi.copy()
    Lx, Ly, Lz, Lt = dims
    mu = (k - 1) % 4
    ax = AXIS[mu]
    U = fat[mu].reshape(Lt, Lz, Ly, Lx, 3, 3)
    p = _grid(dims, phi)
    if k <= 4:   # U_mu(x) phi(x + mu)
        nb = np.roll(p, -1, axis=ax)
        out = np.einsum("...ab,...b->...a", U, nb)
    else:        # U_mu(x - mu)^dag phi(x - mu)
        Ub = np.roll(U, 1, axis=ax)
        nb = np.roll(p, 1, axis=ax)
        out = np.einsum("...ba,...b->...a", Ub.conj(), nb)
    return out.reshape(-1, 3)


def bf16_round(a):
    """Round float32 values to bfloat16 (round to nearest, ties to even); returns float32."""
    a = np.ascontiguousarray(a, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    out = (r & 0xFFFFFFFF).astype(np.uint32).view(np.float32)
    return np.where(np.isnan(a), a, out)


def _bf16c(z):
    """Complex array with real and imaginary parts rounded FP32 -> BF16."""
    z = np.asarray(z)
    return bf16_round(z.real.astype(np.float32)).astype(np.float64) + 1j * bf16_round(
        z.imag.astype(np.float32)).astype(np.float64)


def layer_forward(dims, fat, W, x, bf16=False):
    """out (C_out, V, 3) = sum_k W_k T_k x for x (C_in, V, 3), W (9, C_out, C_in).

    bf16=True rounds the weights and the transported features to BF16 (via
    FP32) before the mixing, as the MFMA operands are."""
    feats = np.stack([np.stack([transport(dims, fat, x[b], k) for b in range(x.shape[0])]) for k in range(9)])
    if bf16:
        feats = _bf16c(feats.astype(np.complex64))
        W = _bf16c(np.asarray(W).astype(np.complex64))
    return np.einsum("kab,kbvc->avc", W, feats)


def adjoint_weights(W):
    """W'_{k}^{ba} = conj(W_{k^dag}^{ab}): the layer whose forward map is the input gradient."""
    W = np.asarray(W)
    return np.stack([np.conj(W[ADJOINT[k]]).T for k in range(9)])


def layer_backward(dims, fat, W, x, g, bf16=False):
    """(dl/dx, dl/dW) of one layer given x (C_in, V, 3) and g = dl/dout (C_out, V, 3).

    bf16=True rounds the operands of the weight-gradient product (the
    transported features and g) to BF16 via FP32, as the MFMA kernel does."""
    Cin = x.shape[0]
    gW = np.zeros_like(np.asarray(W, dtype=np.complex128))
    gg = _bf16c(np.asarray(g).astype(np.complex64)) if bf16 else g
    for k in range(9):
        for b in range(Cin):
            f = transport(dims, fat, x[b], k)
            if bf16:
                f = _bf16c(f.astype(np.complex64))
            gW[k, :, b] = np.einsum("vc,avc->a", f.conj(), gg)
    gx = np.zeros_like(x, dtype=np.complex128)
    for k in range(9):
        for a in range(g.shape[0]):
            tg = transport(dims, fat, g[a], ADJOINT[k])
            gx += np.conj(W[k, a, :])[:, None, None] * tg[None]
    return gx, gW


def embed_even(dims, r_e):
    return lattice.merge(dims, even=r_e)[None]


def net_forward(dims, fat, Ws, r_e, bf16=False):
    """K(r_e) and the input of every layer."""
    x = embed_even(dims, r_e)
    acts = []
    for W in Ws:
        acts.append(x)
        x = layer_forward(dims, fat, W, x, bf16=bf16)
    y_e, _ = lattice.split(dims, x[0])
    return y_e, acts


def net_backward(dims, fat, Ws, acts, g_e):
    """dl/dr_e and [dl/dW_l] given dl/dK(r_e) = g_e."""
    g = embed_even(dims, g_e)
    grads = [None] * len(Ws)
    for l in range(len(Ws) - 1, -1, -1):
        g, grads[l] = layer_backward(dims, fat, Ws[l], acts[l], g)
    g_in, _ = lattice.split(dims, g[0])
    return g_in, grads


def loss_and_grad(ys, xs):
    """l = mean_i |y_i - x_i|^2 / |x_i|^2 and dl/dy_i."""
    B = len(ys)
    loss = 0.0
    grads = []
    for y, x in zip(ys, xs):
        nx = np.vdot(x, x).real
        d = y - x
        loss += np.vdot(d, d).real / nx
        grads.append(2.0 * d / (nx * B))
    return loss / B, grads


def adam_step(w, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba 2014) on the real and imaginary parts, in place; t counts from 1."""
    for arr_w, arr_g, arr_m, arr_v in zip(w, g, m, v):
        for part in ("real", "imag"):
            wp, gp = getattr(arr_w, part), getattr(arr_g, part)
            mp, vp = getattr(arr_m, part), getattr(arr_v, part)
            mp *= b1
            mp += (1 - b1) * gp
            vp *= b2
            vp += (1 - b2) * gp * gp
            mhat = mp / (1 - b1 ** t)
            vhat = vp / (1 - b2 ** t)
            wp -= lr * mhat / (np.sqrt(vhat) + eps)


def channels_of(C):
    return [(C, 1), (C, C), (C, C), (1, C)]


def identity_weights(C):
    """Weights for which K is the identity on even vectors."""
    Ws = []
    for co, ci in channels_of(C):
        W = np.zeros((9, co, ci), np.complex128)
        for a in range(min(co, ci)):
            W[0, a, a] = 1.0
        Ws.append(W)
    return Ws
