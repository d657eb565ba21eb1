"""Link construction for the improved staggered operator: FP64 reference
(TEST INFRASTRUCTURE ONLY: used by tests/, never by the library).

Sec. 4 of the paper builds the three-link (Naik) matrices from the thin
links and notes that this is matrix-matrix work:

    L_mu(n) = U_mu(n) U_mu(n + mu) U_mu(n + 2 mu).

The one-link matrices of the improved action are sums of products of thin
links along paths from n to n + mu (smearing).  The paper does not give the
paths or their weights; this reference takes the weights as inputs and
sums the usual path families, each over every direction and sign:

    one-link     U_mu(n)
    3-staple     U_nu(n) U_mu(n+nu) U_nu(n+mu)^dag                          (nu = +-1 of 3 axes: 6 paths)
    5-staple     a 3-staple in rho whose middle link is replaced by a
                 3-staple in nu, nu != rho                                   (24 paths)
    7-staple     the same once more with a third axis                       (48 paths)
    Lepage       a 3-staple in nu whose middle link is a 3-staple in the
                 same nu with the same sign (reaches two steps out)         (6 paths)

A backward staple (sign -) is U_nu(n-nu)^dag V(n-nu) U_nu(n-nu+mu).  The
staggered phases and the time boundary sign are folded in afterwards, by
`fold`, with hop 1 for one-link and 3 for three-link matrices.

Fields are canonical complex128 arrays (4, V, 3, 3), V in lex order
(x fastest), periodic indexing.
"""
from __future__ import annotations

import numpy as np

from . import lattice

AXIS = {0: 3, 1: 2, 2: 1, 3: 0}          # lattice direction -> axis of the (t, z, y, x) grid
PATH_COUNTS = {"one": 1, "3": 6, "5": 24, "7": 48, "lepage": 6}


def shift(dims, f, mu, k):
    """g(n) = f(n + k mu) for a (V, 3, 3) field."""
    Lx, Ly, Lz, Lt = dims
    g = f.reshape(Lt, Lz, Ly, Lx, 3, 3)
    return np.roll(g, -k, axis=AXIS[mu]).reshape(-1, 3, 3)


def dag(a):
    return np.conj(np.swapaxes(a, -1, -2))


def three_link(dims, U):
    """L_mu(n) = U_mu(n) U_mu(n+mu) U_mu(n+2mu) for all mu."""
    return np.stack([U[mu] @ shift(dims, U[mu], mu, 1) @ shift(dims, U[mu], mu, 2) for mu in range(4)])


def staple(dims, U, V, mu, nu, sign):
    """The staple of the field V (standing in for the mu-link) in direction nu with the given sign (+1, -1)."""
    if sign > 0:
        return U[nu] @ shift(dims, V, nu, 1) @ dag(shift(dims, U[nu], mu, 1))
    B = dag(U[nu]) @ V @ shift(dims, U[nu], mu, 1)     # the backward staple rooted at n - nu
    return shift(dims, B, nu, -1)


def staple_both(dims, U, V, mu, nu):
    return staple(dims, U, V, mu, nu, +1) + staple(dims, U, V, mu, nu, -1)


def fat_paths(dims, U, c):
    """sum over path families of c[k] times their path sums; c = (one-link, 3-, 5-, 7-staple, Lepage)."""
    c1, c3, c5, c7, cl = (float(v) for v in c)
    out = np.zeros_like(U)
    for mu in range(4):
        F = c1 * U[mu]
        others = [d for d in range(4) if d != mu]
        for nu in others:
            S3 = staple_both(dims, U, U[mu], mu, nu)
            F = F + c3 * S3
            for s in (+1, -1):
                F = F + cl * staple(dims, U, staple(dims, U, U[mu], mu, nu, s), mu, nu, s)
            for rho in others:
                if rho == nu:
                    continue
                S5 = staple_both(dims, U, S3, mu, rho)
                F = F + c5 * S5
                for sig in others:
                    if sig in (nu, rho):
                        continue
                    F = F + c7 * staple_both(dims, U, S5, mu, sig)
        out[mu] = F
    return out


def fold(dims, links, hop, antiperiodic_t=True):
    """eta_mu(n) b_mu(n) links_mu(n): MILC staggered phases (eta_x = 1, eta_y = (-1)^x,
    eta_z = (-1)^(x+y), eta_t = (-1)^(x+y+z)) and, for antiperiodic time, -1 on the
    t-links whose hop of `hop` sites crosses the last time slice."""
    e = lattice.eta(dims)                       # (V, 4)
    t = lattice.coords(dims)[:, 3]
    out = np.array(links, dtype=np.complex128, copy=True)
    for mu in range(4):
        s = e[:, mu].copy()
        if mu == 3 and antiperiodic_t:
            s[t + hop >= dims[3]] *= -1
        out[mu] *= s[:, None, None]
    return out


# ------------------------------------------------------------------ explicit path walker
def walk(dims, U, n, steps):
    """Product of links along a path from site n (coordinate 4-vector) taking the
    signed unit steps in `steps` (e.g. [(+1, nu), (+1, mu), (-1, nu)]): a step
    +d multiplies U_d(here), a step -d multiplies U_d(here - d)^dag."""
    here = np.array(n, dtype=int)
    P = np.eye(3, dtype=np.complex128)
    for s, d in steps:
        if s > 0:
            P = P @ U[d, int(lattice.lex_of(here, dims))]
            here[d] = (here[d] + 1) % dims[d]
        else:
            here[d] = (here[d] - 1) % dims[d]
            P = P @ dag(U[d, int(lattice.lex_of(here, dims))])
    return P, here


def path_list(mu):
    """Every path of every family for direction mu, as (family, steps)."""
    others = [d for d in range(4) if d != mu]
    out = [("one", [(+1, mu)])]

    def wrap(inner, s, d):
        return [(s, d)] + inner + [(-s, d)]
    for nu in others:
        for s in (+1, -1):
            out.append(("3", wrap([(+1, mu)], s, nu)))
            out.append(("lepage", wrap(wrap([(+1, mu)], s, nu), s, nu)))
            for rho in others:
                if rho == nu:
                    continue
                for r in (+1, -1):
                    out.append(("5", wrap(wrap([(+1, mu)], s, nu), r, rho)))
                    for sig in others:
                        if sig in (nu, rho):
                            continue
                        for q in (+1, -1):
                            out.append(("7", wrap(wrap(wrap([(+1, mu)], s, nu), r, rho), q, sig)))
    return out
