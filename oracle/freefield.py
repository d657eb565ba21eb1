"""Closed forms of the staggered operator with constant links (test infrastructure only).

With fat links c1 * 1 and long links c3 * 1 (phases folded in), a plane wave
psi(n) = exp(i p.n) chi satisfies, at every site n,

  (D psi)(n) = 2 i sum_mu eta_mu(n) (c1 sin p_mu + c3 sin 3 p_mu) psi(n),

because eta_mu does not depend on the mu coordinate.  Writing s_mu(p) for the
bracket, eta_mu(n) exp(i p.n) is a plane wave of momentum p + pi*zeta_mu with
s_nu(p + pi*zeta_mu) = -+ s_nu(p); the cross terms of D^2 cancel in pairs and

  A psi_e = (4 m^2 + 4 sum_mu s_mu(p)^2) psi_e

on the even projection psi_e.  Antiperiodic time boundaries shift the allowed
p_t to (2k+1) pi / Lt.  A = 4m^2 - D^2 is then diagonal in momentum space, so
the even-odd system is solved exactly by one FFT.
"""
from __future__ import annotations

import numpy as np

from . import lattice


def momentum(dims, k, antiperiodic_t=True):
    p = np.array([2 * np.pi * k[mu] / dims[mu] for mu in range(4)], dtype=np.float64)
    if antiperiodic_t:
        p[3] = (2 * k[3] + 1) * np.pi / dims[3]
    return p


def plane_wave(dims, k, chi, antiperiodic_t=True):
    """Full-lattice (V, 3) field exp(i p.n) chi."""
    p = momentum(dims, k, antiperiodic_t)
    c = lattice.coords(dims)
    ph = np.exp(1j * (c @ p))
    return ph[:, None] * np.asarray(chi, np.complex128)[None, :]


def s_mu(p, c1, c3):
    return c1 * np.sin(p) + c3 * np.sin(3 * p)


def dslash_plane_wave(dims, k, chi, c1, c3, antiperiodic_t=True):
    """Closed-form (D psi)(n) on the full lattice for psi = plane_wave(k, chi)."""
    p = momentum(dims, k, antiperiodic_t)
    psi = plane_wave(dims, k, chi, antiperiodic_t)
    e = lattice.eta(dims)
    fac = 2j * (e @ s_mu(p, c1, c3))
    return fac[:, None] * psi


def A_eigenvalue(dims, k, mass, c1, c3, antiperiodic_t=True):
    p = momentum(dims, k, antiperiodic_t)
    return 4 * mass * mass + 4 * np.sum(s_mu(p, c1, c3) ** 2)


def fft_solve(dims, b_even, mass, c1, c3, antiperiodic_t=True):
    """Exact solution x_e of A x_e = b_e for constant links, via FFT.

    The even source is embedded on the full lattice (odd sites zero); A acts
    as 4 m^2 - D^2, which is diagonal in momentum space and maps even-only
    fields to even-only fields.
    """
    Lx, Ly, Lz, Lt = dims
    full = lattice.merge(dims, even=b_even)  # (V, 3) lex order, x fastest
    f = full.reshape(Lt, Lz, Ly, Lx, 3)
    t = np.arange(Lt)
    twist = np.exp(-1j * np.pi * t / Lt) if antiperiodic_t else np.ones(Lt)
    f = f * twist[:, None, None, None, None]
    F = np.fft.fftn(f, axes=(0, 1, 2, 3))
    # momentum of each FFT bin (periodic part) plus the antiperiodic shift pi/Lt
    px = 2 * np.pi * np.fft.fftfreq(Lx) 
    py = 2 * np.pi * np.fft.fftfreq(Ly)
    pz = 2 * np.pi * np.fft.fftfreq(Lz)
    pt = 2 * np.pi * np.fft.fftfreq(Lt) + (np.pi / Lt if antiperiodic_t else 0.0)
    S = (s_mu(pt, c1, c3) ** 2)[:, None, None, None] + (s_mu(pz, c1, c3) ** 2)[None, :, None, None] \
        + (s_mu(py, c1, c3) ** 2)[None, None, :, None] + (s_mu(px, c1, c3) ** 2)[None, None, None, :]
    lam = 4 * mass * mass + 4 * S
    X = F / lam[..., None]
    x = np.fft.ifftn(X, axes=(0, 1, 2, 3)) / twist[:, None, None, None, None]
    x = x.reshape(-1, 3)
    xe, xo = lattice.split(dims, x)
    return xe, xo
