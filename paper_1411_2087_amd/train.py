"""Training of the gauge-covariant preconditioner on the GPU.

Sequences the library's kernels (net_forward, net_loss, net_backward,
net_adam_step, hisq_apply_A, hisq_dot) over batches of (b, x) pairs with
A x = b produced by the library's own CG.  Two objectives:
  "error"    mean_i |K(b_i) - x_i|^2 / |x_i|^2         (fits K to A^-1 on the pairs)
  "residual" mean_i |A K(b_i) - b_i|^2 / |b_i|^2       (approximate-inverse objective;
             its gradient with respect to K(b_i) is A applied to the residual, A Hermitian)
Every arithmetic step runs in libhisq; this module only orders the calls and
owns the device buffers.
"""
from __future__ import annotations

import numpy as np
import torch

from . import (HISQ_F32, HISQ_F64, HISQ_MULTI_RHS, CGOpts, cg_solve_multi, hisq_apply_A, hisq_dot,
               hisq_workspace_bytes, net_act_bytes,
               net_adam_step, net_backward, net_backward_ws_bytes, net_forward, net_loss, net_weight_count)
from .fields import Links, workspace

LAYER_SHAPES = lambda C: [(C, 1), (C, C), (C, C), (1, C)]  # (C_out, C_in) per layer


def identity_weights(C, scale=1.0):
    """Weights with K = scale * identity (every layer passes channel 0 through T_0)."""
    Ws = []
    for i, (co, ci) in enumerate(LAYER_SHAPES(C)):
        W = np.zeros((9, co, ci), np.complex64)
        W[0, 0, 0] = scale if i == 3 else 1.0
        for a in range(1, min(co, ci)):
            W[0, a, a] = 1.0
        Ws.append(W)
    return Ws


def flatten(Ws):
    return np.concatenate([W.reshape(-1) for W in Ws]).astype(np.complex64)


def unflatten(w, C):
    out, o = [], 0
    for co, ci in LAYER_SHAPES(C):
        n = 9 * co * ci
        out.append(np.asarray(w[o:o + n]).reshape(9, co, ci))
        o += n
    return out


def initial_weights(C, scale, noise, noise_seed):
    """scale * identity plus complex Gaussian noise of size `noise` (drawn by the input generator)."""
    import synth
    w = flatten(identity_weights(C, scale))
    z = synth.gauss(noise_seed, 7, w.size).astype(np.complex64)
    return w + noise * z


def lambda_max_estimate(links64: Links, mass, dims, steps=60, seed=999):
    """The largest eigenvalue of A(mass) by power iteration on the FP64 operator: sqrt(|A^(k+1) v|^2 / |A^k v|^2)
    after `steps` applications to a Gaussian v (no normalisation needed in FP64 for |lambda| < 1e6), raised by 5 %
    (the iteration approaches it from below)."""
    import synth
    v = torch.from_numpy(synth.source(dims, seed)).cuda()
    w, tmp = torch.empty_like(v), torch.empty_like(v)
    ws = torch.empty(hisq_workspace_bytes("dot", dims), dtype=torch.uint8, device=v.device)
    n = v.shape[0] * 3
    prev = hisq_dot(v, v, n, HISQ_F64, ws).real
    lam = 0.0
    for _ in range(steps):
        hisq_apply_A(mass, links64.fat, links64.lng, v, w, tmp, dims, HISQ_F64)
        cur = hisq_dot(w, w, n, HISQ_F64, ws).real
        lam = float(np.sqrt(cur / prev))
        prev = cur
        v, w = w, v
    return 1.05 * lam


def chebyshev_weights(C, mass, lambda_max, lambda_lo=None):
    """Weights with which the network computes K = p(A) exactly when the operator's long links are zero (its
    Dslash is then D = sum_mu T_{+mu} - T_{-mu} over the fat-link transports the layers already apply), p the
    quadratic for which 1 - l p(l) is the degree-3 Chebyshev polynomial shifted to [lambda_lo, lambda_max] and
    normalised to 1 at l = 0, the quadratic that minimises max |1 - l p(l)| on that interval.  On [4 m^2,
    lambda_max] it would divide the condition number by (d + 1)^2 = 9, but p then nearly vanishes where
    1 - l p(l) touches its upper bound inside the spectrum (p_min / p_max ~ 1e-5 at m = 0.005), and the BF16
    rounding of the network (~5e-3 of K) can make K indefinite.  The default lambda_lo = max(4 m^2,
    lambda_max / 30) keeps p_min / p_max ~ 0.04 and costs ~5 % of the condition-number gain.  With
    D^2 = 4 m^2 - A on the even sites the layers carry phi, D phi -> phi, D^2 phi -> phi, D^3 phi,
    D^2 phi -> alpha phi + beta D^2 phi + gamma D^4 phi (C >= 4).  A reference for the trained networks: it is
    built, not learned."""
    from numpy.polynomial import Polynomial
    b = float(lambda_max)
    a = max(4.0 * mass * mass, b / 30.0) if lambda_lo is None else float(lambda_lo)
    y = Polynomial([(b + a) / (b - a), -2.0 / (b - a)])   # [a, b] -> [1, -1]
    t3 = Polynomial([0.0, -3.0, 0.0, 4.0])                 # T_3(y) = 4 y^3 - 3 y
    q = t3(y) / t3((b + a) / (b - a))                      # q(0) = 1
    c0, c1, c2 = -q.coef[1], -q.coef[2], -q.coef[3]        # p(l) = (1 - q(l)) / l
    m4 = 4.0 * mass * mass                                 # K = p(A), A = m4 - D^2 on the even sites
    alpha, beta, gamma = c0 + m4 * c1 + m4 * m4 * c2, -c1 - 2 * m4 * c2, c2
    Ws = [np.zeros((9, co, ci), np.complex64) for co, ci in LAYER_SHAPES(C)]
    sgn = [0.0, 1.0, 1.0, 1.0, 1.0, -1.0, -1.0, -1.0, -1.0]  # D: +1 on the forward hops, -1 on the backward ones
    Ws[0][0, 0, 0] = 1.0
    Ws[0][:, 1, 0] = sgn                                   # ch0 = phi, ch1 = D phi
    Ws[1][0, 0, 0] = 1.0
    Ws[1][:, 1, 1] = sgn                                   # ch0 = phi, ch1 = D^2 phi
    Ws[2][0, 0, 0] = 1.0
    Ws[2][:, 1, 1] = sgn
    Ws[2][0, 2, 1] = 1.0                                   # ch0 = phi, ch1 = D^3 phi, ch2 = D^2 phi
    Ws[3][0, 0, 0] = alpha
    Ws[3][0, 0, 2] = beta
    Ws[3][:, 0, 1] = np.asarray(sgn) * gamma               # out = alpha phi + beta D^2 phi + gamma D^4 phi
    return flatten(Ws), (c0, c1, c2)


def make_pairs(dims, mass, links64: Links, links32: Links, sources: np.ndarray, tol=1e-8, device="cuda", log=None):
    """x_i = A(mass)^-1 b_i for every source, by the batched reliable-update CG, 16 at a time.
    Returns (b, x) as device complex64 tensors [n][Vh][3], the total solve time and x in complex128.
    log (optional): called with a progress line after each batch."""
    n = sources.shape[0]
    vh = sources.shape[1]
    bs = torch.from_numpy(np.ascontiguousarray(sources)).to(device)
    xs = torch.zeros_like(bs)
    opts = CGOpts(mode=0, max_iter=0, check_every=0, use_graph=1, delta=0.1)
    seconds = 0.0
    for s in range(0, n, 16):
        k = min(16, n - s)
        ws = workspace("cg_multi", dims, k, HISQ_MULTI_RHS)
        b = bs[s:s + k].contiguous()
        x = torch.zeros_like(b)
        st = cg_solve_multi(k, [mass] * k, tol, HISQ_MULTI_RHS, links64.fat, links64.lng, links32.fat, links32.lng, b,
                            x, dims, opts, ws, raise_on_noconv=True)
        seconds += st[0]["time_s"]
        xs[s:s + k] = x
        if log is not None:
            log(f"[pairs] {s + k}/{n}: {max(r['iters'] for r in st)} iterations, {st[0]['time_s']:.2f}s")
    return bs.to(torch.complex64), xs.to(torch.complex64), seconds, xs


class Trainer:
    """Adam on the network weights; buffers sized for `batch` sources."""

    def __init__(self, dims, C, fat32, weights: np.ndarray, batch=16, device="cuda", objective="error",
                 links32: Links | None = None, mass: float | None = None):
        self.dims, self.C, self.fat32, self.batch = tuple(dims), C, fat32, batch
        assert objective in ("error", "residual")
        self.objective, self.links32, self.mass = objective, links32, mass
        if objective == "residual":
            assert links32 is not None and mass is not None
        n = net_weight_count(C)
        assert weights.size == n
        self.n = n
        self.w = torch.from_numpy(weights.astype(np.complex64)).to(device)
        self.m = torch.zeros(2 * n, dtype=torch.float32, device=device)
        self.v = torch.zeros(2 * n, dtype=torch.float32, device=device)
        self.gw = torch.zeros(n, dtype=torch.complex64, device=device)
        vh = int(np.prod(dims)) // 2
        self.acts = torch.empty(net_act_bytes(dims, C, batch), dtype=torch.uint8, device=device)
        self.ws = torch.empty(net_backward_ws_bytes(dims, C, batch), dtype=torch.uint8, device=device)
        self.lws = torch.empty(2048 * (batch + 1) + 4096, dtype=torch.uint8, device=device)
        self.y = torch.empty((batch, vh, 3), dtype=torch.complex64, device=device)
        self.gy = torch.empty_like(self.y)
        self.ay = torch.empty_like(self.y)
        self.g1 = torch.empty_like(self.y)
        self.tmp = torch.empty((vh, 3), dtype=torch.complex64, device=device)
        self.step_count = 0

    def _apply_A(self, src, dst):
        for i in range(src.shape[0]):
            hisq_apply_A(self.mass, self.links32.fat, self.links32.lng, src[i], dst[i], self.tmp, self.dims, HISQ_F32)

    def forward(self, b):
        k = b.shape[0]
        net_forward(self.fat32, self.w, self.C, b, self.y[:k], self.acts, k, self.dims)
        return self.y[:k]

    def loss(self, b, x):
        k = b.shape[0]
        y = self.forward(b)
        if self.objective == "residual":
            self._apply_A(y, self.ay[:k])
            return net_loss(self.ay[:k], b, k, self.dims, None, self.lws)
        return net_loss(y, x, k, self.dims, None, self.lws)

    def step(self, b, x, lr, sync=False):
        """One Adam step on a batch; returns the batch loss before the step if sync."""
        k = b.shape[0]
        assert k <= self.batch
        y = self.forward(b)
        if self.objective == "residual":
            self._apply_A(y, self.ay[:k])
            loss = net_loss(self.ay[:k], b, k, self.dims, self.g1[:k], self.lws, sync=sync)
            self._apply_A(self.g1[:k], self.gy[:k])
        else:
            loss = net_loss(y, x, k, self.dims, self.gy[:k], self.lws, sync=sync)
        net_backward(self.fat32, self.w, self.C, self.acts, self.gy[:k], self.gw, None, k, self.dims, self.ws)
        self.step_count += 1
        net_adam_step(self.w, self.gw, self.m, self.v, self.n, lr, self.step_count)
        return loss

    def fit(self, b_train, x_train, steps, lr=1e-3, log_every=50, seed=0, log=None):
        """`steps` Adam steps over shuffled batches; returns [(step, loss)] at log points."""
        rng = np.random.default_rng(seed)
        n = b_train.shape[0]
        hist = []
        order = rng.permutation(n)
        pos = 0
        for s in range(1, steps + 1):
            if pos + self.batch > n:
                order = rng.permutation(n)
                pos = 0
            idx = torch.from_numpy(order[pos:pos + self.batch]).to(b_train.device)
            pos += self.batch
            sync = (s % log_every == 0) or s == 1
            l = self.step(b_train[idx].contiguous(), x_train[idx].contiguous(), lr, sync=sync)
            if sync:
                hist.append((s, l))
                if log:
                    log(f"[train] step {s} loss {l:.5f}")
        return hist

    def evaluate(self, b, x):
        losses = []
        for s in range(0, b.shape[0], self.batch):
            bb, xx = b[s:s + self.batch].contiguous(), x[s:s + self.batch].contiguous()
            losses.append(self.loss(bb, xx) * bb.shape[0])
        return float(np.sum(losses) / b.shape[0])


def _dot_workspace(like):
    return torch.empty(hisq_workspace_bytes("dot", (4, 4, 4, 4)), dtype=torch.uint8, device=like.device)


def least_squares_scale(b, x):
    """The scalar s minimising sum |s b - x|^2 (starting point of K = s 1 for the error objective)."""
    n = b.shape[1] * 3
    ws = _dot_workspace(b)
    num = sum(hisq_dot(b[i], x[i], n, HISQ_F32, ws).real for i in range(b.shape[0]))
    den = sum(hisq_dot(b[i], b[i], n, HISQ_F32, ws).real for i in range(b.shape[0]))
    return num / den


def residual_scale(b, links32: Links, mass, dims):
    """The scalar s minimising sum |s A b - b|^2 (starting point for the residual objective)."""
    n = b.shape[1] * 3
    ab = torch.empty_like(b[0])
    tmp = torch.empty_like(b[0])
    ws = _dot_workspace(b)
    num = den = 0.0
    for i in range(b.shape[0]):
        hisq_apply_A(mass, links32.fat, links32.lng, b[i].contiguous(), ab, tmp, dims, HISQ_F32)
        num += hisq_dot(ab, b[i].contiguous(), n, HISQ_F32, ws).real
        den += hisq_dot(ab, ab, n, HISQ_F32, ws).real
    return num / den
