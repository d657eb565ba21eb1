"""Brute-force dense staggered Dslash for tiny lattices (test infrastructure only).

Assembles the 3V x 3V complex matrix of the operator term by term from its
definition (Sec. 3 of the paper: at every site, for each of the 8 directions
+-mu, a one-link matrix on the nearest neighbour and a three-link matrix on
the third-nearest neighbour), with no reuse of the C oracle's code:

  D[n, n+mu]   += F_mu(n)         D[n, n-mu]   -= F_mu(n-mu)^dag
  D[n, n+3mu]  += L_mu(n)         D[n, n-3mu]  -= L_mu(n-3mu)^dag

Blocks are accumulated, never assigned: on a lattice of extent 4, n+3mu and
n-mu are the same site.
"""
from __future__ import annotations

import numpy as np

from . import lattice


def dense_D(dims, fat, lng):
    dims = tuple(dims)
    V = int(np.prod(dims))
    c = lattice.coords(dims)
    D = np.zeros((3 * V, 3 * V), np.complex128)
    for n in range(V):
        for mu in range(4):
            for hop, U in ((1, fat), (3, lng)):
                fwd = c[n].copy()
                fwd[mu] = (fwd[mu] + hop) % dims[mu]
                bwd = c[n].copy()
                bwd[mu] = (bwd[mu] - hop) % dims[mu]
                f = int(lattice.lex_of(fwd, dims))
                b = int(lattice.lex_of(bwd, dims))
                D[3 * n:3 * n + 3, 3 * f:3 * f + 3] += U[mu, n]
                D[3 * n:3 * n + 3, 3 * b:3 * b + 3] -= U[mu, b].conj().T
    return D


def color_index(dims, p):
    """Row/column indices of D for the colour components of parity-p sites, h order."""
    s = lattice.parity_sites(dims, p)
    return (3 * s[:, None] + np.arange(3)[None, :]).reshape(-1)


def blocks(dims, D):
    """(D_eo, D_oe): even rows x odd columns and odd rows x even columns."""
    e = color_index(dims, 0)
    o = color_index(dims, 1)
    return D[np.ix_(e, o)], D[np.ix_(o, e)]


def dense_A(dims, D, mass):
    """A = 4 m^2 - D_eo D_oe on the even sites."""
    Deo, Doe = blocks(dims, D)
    return 4.0 * mass * mass * np.eye(Deo.shape[0]) - Deo @ Doe
