"""Flexible CG with a preconditioner K, plain FP64 (test infrastructure only).

Flexible conjugate gradient (Notay 2000, FCG with one stored direction; the
Polak-Ribiere form of the direction update of Golub & Ye 1999), solving the
even-odd system A x = b of the staggered operator (Sec. 3 CG, Sec. 4
even-odd):

    r_0 = b - A x_0, z_0 = K(r_0), p_0 = z_0
    alpha_k = Re<z_k, r_k> / Re<p_k, A p_k>
    x_{k+1} = x_k + alpha_k p_k,  r_{k+1} = r_k - alpha_k A p_k
    z_{k+1} = K(r_{k+1})
    beta_k  = Re<z_{k+1}, r_{k+1} - r_k> / Re<z_k, r_k>
    p_{k+1} = z_{k+1} + beta_k p_k

With K = 1 the iterates are those of CG; with K = A^-1 one step solves.  If
Re<z, r> <= 0 or Re<p, A p> <= 0 (K not positive on r), or the residual has
not fallen for `stall` iterations, the solve continues from the current x
with plain CG (the fallback).
"""
from __future__ import annotations

import numpy as np

from . import apply_A, cg


def fcg(dims, mass, fat, lng, b, K, tol=1e-10, max_iter=10000, stall=50, x0=None):
    bb = np.vdot(b, b).real
    x = np.zeros_like(b) if x0 is None else x0.copy()
    r = b - apply_A(dims, mass, fat, lng, x)
    hist = [np.sqrt(np.vdot(r, r).real / bb)]
    z = K(r)
    p = z.copy()
    zr = np.vdot(z, r).real
    best, since = hist[0], 0
    it = 0
    fallback = False
    while it < max_iter and hist[-1] > tol:
        ap = apply_A(dims, mass, fat, lng, p)
        pap = np.vdot(p, ap).real
        if not (zr > 0 and pap > 0):
            fallback = True
            break
        alpha = zr / pap
        x = x + alpha * p
        r_new = r - alpha * ap
        it += 1
        hist.append(np.sqrt(np.vdot(r_new, r_new).real / bb))
        if hist[-1] < best:
            best, since = hist[-1], 0
        else:
            since += 1
            if since >= stall:
                fallback = True
                r = r_new
                break
        z = K(r_new)
        zr_new = np.vdot(z, r_new).real
        beta = np.vdot(z, r_new - r).real / zr
        p = z + beta * p
        r, zr = r_new, zr_new
    info = {"iters": it, "history": np.array(hist), "fallback": fallback}
    if fallback:
        x, cinfo = cg(dims, mass, fat, lng, b, tol=tol, max_iter=max(1, max_iter - it), x0=x)
        info["fallback_iters"] = cinfo["iters"]
    return x, info
