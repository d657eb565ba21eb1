"""Pins of the link-construction part of the oracle (three-link products and
path-summed one-link matrices, Sec. 4 of the paper).

Checked against closed forms (unit links, pure-gauge fields), gauge
covariance, an explicit walk along every path of every family at sampled
sites, the independent phase folding of the input generator, and planted
mistakes that the pins must catch."""
import numpy as np
import pytest

import synth
from oracle import lattice
from oracle import links as K

DIMS = (4, 6, 4, 8)
FAT7 = (1 / 8, 1 / 16, 1 / 64, 1 / 384, 0.0)
ODD = (0.3, -0.11, 0.037, 0.0071, -0.052)     # weights with no special relation


def unit(dims):
    V = int(np.prod(dims))
    return np.broadcast_to(np.eye(3, dtype=np.complex128), (4, V, 3, 3)).copy()


def pure_gauge(dims, seed):
    V = int(np.prod(dims))
    g = synth.haar(seed, V)
    U = np.empty((4, V, 3, 3), np.complex128)
    for mu in range(4):
        U[mu] = g @ K.dag(K.shift(dims, g, mu, 1))
    return g, U


def weight_sum(c):
    n = K.PATH_COUNTS
    return c[0] * n["one"] + c[1] * n["3"] + c[2] * n["5"] + c[3] * n["7"] + c[4] * n["lepage"]


def test_path_counts_by_enumeration():
    for mu in range(4):
        fam = [f for f, _ in K.path_list(mu)]
        for k, n in K.PATH_COUNTS.items():
            assert fam.count(k) == n
    # fat7 weights are normalised: unit links give the identity
    assert abs(weight_sum(FAT7) - 1.0) < 1e-15


def test_unit_links():
    U = unit(DIMS)
    assert np.allclose(K.three_link(DIMS, U), U, atol=0, rtol=0)
    F = K.fat_paths(DIMS, U, ODD)
    assert np.max(np.abs(F - weight_sum(ODD) * U)) < 1e-14


def test_pure_gauge_closed_form():
    """U_mu(n) = g(n) g(n+mu)^dag: every path from n to n+k mu multiplies to g(n) g(n+k mu)^dag."""
    g, U = pure_gauge(DIMS, 11)
    L = K.three_link(DIMS, U)
    F = K.fat_paths(DIMS, U, ODD)
    for mu in range(4):
        ref3 = g @ K.dag(K.shift(DIMS, g, mu, 3))
        ref1 = g @ K.dag(K.shift(DIMS, g, mu, 1))
        assert np.max(np.abs(L[mu] - ref3)) < 1e-13
        assert np.max(np.abs(F[mu] - weight_sum(ODD) * ref1)) < 1e-12


def test_gauge_covariance():
    V = int(np.prod(DIMS))
    U = synth.thin_links(DIMS, 21)
    g = synth.haar(22, V)
    Ug = np.stack([g @ U[mu] @ K.dag(K.shift(DIMS, g, mu, 1)) for mu in range(4)])
    L, Lg = K.three_link(DIMS, U), K.three_link(DIMS, Ug)
    F, Fg = K.fat_paths(DIMS, U, ODD), K.fat_paths(DIMS, Ug, ODD)
    for mu in range(4):
        assert np.max(np.abs(Lg[mu] - g @ L[mu] @ K.dag(K.shift(DIMS, g, mu, 3)))) < 1e-13
        assert np.max(np.abs(Fg[mu] - g @ F[mu] @ K.dag(K.shift(DIMS, g, mu, 1)))) < 1e-12


@pytest.mark.parametrize("family", ["one", "3", "5", "7", "lepage"])
def test_explicit_walk(family):
    """Each family on its own (weight 1, others 0) equals the sum of explicit walks along its paths."""
    U = synth.thin_links(DIMS, 31)
    c = [0.0] * 5
    c[["one", "3", "5", "7", "lepage"].index(family)] = 1.0
    F = K.fat_paths(DIMS, U, c)
    coords = lattice.coords(DIMS)
    rng = np.random.default_rng(5)
    for n in rng.choice(len(coords), 6, replace=False):
        for mu in range(4):
            acc = np.zeros((3, 3), np.complex128)
            for fam, steps in K.path_list(mu):
                if fam != family:
                    continue
                P, end = K.walk(DIMS, U, coords[n], steps)
                want = coords[n].copy()
                want[mu] = (want[mu] + 1) % DIMS[mu]
                assert np.array_equal(end, want)
                acc += P
            assert np.max(np.abs(F[mu, n] - acc)) < 1e-13
    if family == "one":
        return
    # the three-link product is the walk of three forward steps
    L = K.three_link(DIMS, U)
    for n in rng.choice(len(coords), 4, replace=False):
        for mu in range(4):
            P, _ = K.walk(DIMS, U, coords[n], [(+1, mu)] * 3)
            assert np.max(np.abs(L[mu, n] - P)) < 1e-14


@pytest.mark.parametrize("anti", [True, False])
def test_fold_matches_the_input_generator(anti):
    """The oracle's folding (from lattice.eta) against the input generator's C folding."""
    fat, lng = synth.links(DIMS, 41, fold=False)
    f2, l2 = fat.copy(), lng.copy()
    synth.fold(DIMS, f2, l2, antiperiodic_t=anti)
    assert np.array_equal(K.fold(DIMS, fat, 1, anti), f2)
    assert np.array_equal(K.fold(DIMS, lng, 3, anti), l2)


def test_pins_reject_planted_mistakes(monkeypatch):
    """Plant a dropped backward staple, a wrong shift and a missing dagger in the
    oracle; the closed forms and the walk must notice each."""
    U = synth.thin_links(DIMS, 51)
    g, Ug = pure_gauge(DIMS, 52)
    good_staple = K.staple

    def no_backward(dims, U_, V, mu, nu, sign):
        return good_staple(dims, U_, V, mu, nu, +1) if sign > 0 else np.zeros_like(V)

    def wrong_shift(dims, U_, V, mu, nu, sign):
        if sign > 0:
            return U_[nu] @ K.shift(dims, V, nu, 1) @ K.dag(K.shift(dims, U_[nu], nu, 1))
        return good_staple(dims, U_, V, mu, nu, sign)

    def no_dagger(dims, U_, V, mu, nu, sign):
        if sign > 0:
            return U_[nu] @ K.shift(dims, V, nu, 1) @ K.shift(dims, U_[nu], mu, 1)
        return good_staple(dims, U_, V, mu, nu, sign)

    for bad in (no_backward, wrong_shift, no_dagger):
        monkeypatch.setattr(K, "staple", bad)
        F = K.fat_paths(DIMS, Ug, ODD)
        ref1 = g @ K.dag(K.shift(DIMS, g, 0, 1))
        closed_ok = np.max(np.abs(F[0] - weight_sum(ODD) * ref1)) < 1e-12
        Fw = K.fat_paths(DIMS, U, (0, 1, 0, 0, 0))
        n = 7
        acc = sum(K.walk(DIMS, U, lattice.coords(DIMS)[n], st)[0] for f, st in K.path_list(0) if f == "3")
        walk_ok = np.max(np.abs(Fw[0, n] - acc)) < 1e-13
        assert not (closed_ok and walk_ok), bad.__name__
    monkeypatch.setattr(K, "staple", good_staple)
