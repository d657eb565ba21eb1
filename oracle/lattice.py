"""Site bookkeeping for the NumPy parts of the oracle (test infrastructure only).

lex = x + Lx*(y + Ly*(z + Lz*t)); a full-lattice field is (V, 3) in lex order,
a one-parity field is (Vh, 3) ordered by h = lex >> 1.
"""
from __future__ import annotations

import numpy as np


def coords(dims):
    """(V, 4) integer coordinates (x, y, z, t) of every site, lex order."""
    Lx, Ly, Lz, Lt = dims
    lex = np.arange(Lx * Ly * Lz * Lt)
    return np.stack([lex % Lx, (lex // Lx) % Ly, (lex // (Lx * Ly)) % Lz, lex // (Lx * Ly * Lz)], axis=1)


def lex_of(c, dims):
    Lx, Ly, Lz, Lt = dims
    c = np.asarray(c)
    return c[..., 0] + Lx * (c[..., 1] + Ly * (c[..., 2] + Lz * c[..., 3]))


def parity(dims):
    return coords(dims).sum(axis=1) % 2


def parity_sites(dims, p):
    """lex indices of the sites of parity p, in h order."""
    return np.nonzero(parity(dims) == p)[0]


def split(dims, full):
    """Full-lattice (V, ...) field -> (even (Vh, ...), odd (Vh, ...))."""
    return full[parity_sites(dims, 0)], full[parity_sites(dims, 1)]


def merge(dims, even=None, odd=None, tail=(3,)):
    V = int(np.prod(dims))
    out = np.zeros((V,) + tuple(tail), np.complex128)
    if even is not None:
        out[parity_sites(dims, 0)] = even
    if odd is not None:
        out[parity_sites(dims, 1)] = odd
    return out


def eta(dims):
    """(V, 4) staggered phases, the MILC convention: eta_x = 1, eta_y = (-1)^x,
    eta_z = (-1)^(x+y), eta_t = (-1)^(x+y+z)."""
    c = coords(dims)
    e = np.ones((c.shape[0], 4))
    e[:, 1] = (-1.0) ** c[:, 0]
    e[:, 2] = (-1.0) ** (c[:, 0] + c[:, 1])
    e[:, 3] = (-1.0) ** (c[:, 0] + c[:, 1] + c[:, 2])
    return e
