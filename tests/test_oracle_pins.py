"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

None of these compares the oracle with itself: each check is a closed form,
an invariant, a brute-force dense matrix, or a published test vector.
"""
import numpy as np
import pytest

import oracle
import synth
from oracle import dense, freefield, lattice

DIMS_SMALL = [(4, 4, 4, 4), (4, 6, 8, 10), (6, 4, 4, 8)]


def rng(seed):
    return np.random.default_rng(seed)


def cvec(r, shape):
    return (r.standard_normal(shape) + 1j * r.standard_normal(shape)) / np.sqrt(2)


# ---------------------------------------------------------------- generator
def test_philox_known_answers():
    # Known-answer vectors published with the Random123 library (Salmon et al. 2011).
    assert synth.philox4x32_10((0, 0, 0, 0), (0, 0)) == (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)
    assert synth.philox4x32_10((0xFFFFFFFF,) * 4, (0xFFFFFFFF,) * 2) == (0x408F276D, 0x41C83B0E, 0xA20BC7C6,
                                                                            0x6D5451FD)
    assert synth.philox4x32_10((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0)) == (
        0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)


def test_haar_su3_and_moments():
    n = 100000
    u = synth.haar(7, n)
    eye = np.eye(3)
    assert np.abs(u @ u.conj().transpose(0, 2, 1) - eye).max() < 1e-14
    assert np.abs(np.linalg.det(u) - 1).max() < 1e-14
    tr = np.trace(u, axis1=1, axis2=2)
    # Haar SU(3): E tr U = 0, E |tr U|^2 = 1, E |U_ij|^2 = 1/3
    assert abs(tr.mean()) < 5 / np.sqrt(n)
    assert abs((np.abs(tr) ** 2).mean() - 1) < 0.02
    assert np.abs((np.abs(u) ** 2).mean(axis=0) - 1 / 3).max() < 0.01
    # E tr(U)^3 = 1 for SU(3) (one singlet in 3x3x3), = 0 for U(3): checks the det fix
    assert abs((tr ** 3).mean() - 1) < 0.05


def test_links_generator_statistics():
    dims = (4, 4, 4, 8)
    fat, lng = synth.links(dims, 1001, fold=False)
    # long links are SU(3); fat = 0.6 U + 0.1 Z has E|F_ij|^2 = 0.36/3 + 0.01
    assert np.abs(lng @ lng.conj().transpose(0, 1, 3, 2) - np.eye(3)).max() < 1e-14
    m2 = (np.abs(fat) ** 2).mean()
    assert abs(m2 - (0.36 / 3 + 0.01)) < 0.01
    # reproducible from the seed, different for another seed
    fat2, _ = synth.links(dims, 1001, fold=False)
    assert np.array_equal(fat, fat2)
    fat3, _ = synth.links(dims, 1002, fold=False)
    assert not np.allclose(fat, fat3)


def test_fold_signs():
    dims = (4, 6, 4, 8)
    fat, lng = synth.unit_links(dims, 1.0, 1.0, fold=True, antiperiodic_t=True)
    c = lattice.coords(dims)
    x, y, z, t = c.T
    eta = [np.ones_like(x), (-1) ** x, (-1) ** (x + y), (-1) ** (x + y + z)]
    for mu in range(4):
        bf = np.where((mu == 3) & (t == dims[3] - 1), -1, 1)
        bl = np.where((mu == 3) & (t >= dims[3] - 3), -1, 1)
        assert np.array_equal(fat[mu, :, 0, 0].real, eta[mu] * bf)
        assert np.array_equal(lng[mu, :, 0, 0].real, eta[mu] * bl)


# ---------------------------------------------------------------- counts (Sec. 3)
def test_paper_counts():
    matvec = 36 + 30          # 36 real multiplies + 30 real adds
    flops = 16 * matvec + 15 * 6
    assert flops == oracle.FLOPS_PER_SITE == 1146
    assert 16 * 18 + 16 * 6 == oracle.INPUT_OPERANDS_PER_SITE == 384
    assert oracle.BYTES_DP_VECTOR == 3 * 2 * 8 and oracle.BYTES_DP_MATRIX == 3 * oracle.BYTES_DP_VECTOR
    # memory model of the multishift solver, (36 + 2 Nm) 48 V bytes: 2592 and 2784 B per site
    assert (36 + 2 * 9) * 48 == 2592 and (36 + 2 * 11) * 48 == 2784


# ---------------------------------------------------------------- free field
@pytest.mark.parametrize("dims", DIMS_SMALL)
@pytest.mark.parametrize("anti", [True, False])
def test_free_field_plane_wave(dims, anti):
    r = rng(hash((dims, anti)) % 2 ** 31)
    c1, c3 = 0.7, -0.25
    fat, lng = synth.unit_links(dims, c1, c3, antiperiodic_t=anti)
    for _ in range(3):
        k = [int(r.integers(0, dims[mu])) for mu in range(4)]
        chi = cvec(r, 3)
        psi = freefield.plane_wave(dims, k, chi, anti)
        want = freefield.dslash_plane_wave(dims, k, chi, c1, c3, anti)
        pe, po = lattice.split(dims, psi)
        we, wo = lattice.split(dims, want)
        assert np.abs(oracle.dslash(dims, fat, lng, po, 0) - we).max() < 1e-13
        assert np.abs(oracle.dslash(dims, fat, lng, pe, 1) - wo).max() < 1e-13


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (4, 6, 8, 10)])
def test_free_field_A_eigen_and_one_step_cg(dims):
    r = rng(5)
    c1, c3, mass = 0.6, 0.3, 0.05
    fat, lng = synth.unit_links(dims, c1, c3)
    k = [int(r.integers(0, dims[mu])) for mu in range(4)]
    psi = freefield.plane_wave(dims, k, cvec(r, 3))
    be, _ = lattice.split(dims, psi)
    lam = freefield.A_eigenvalue(dims, k, mass, c1, c3)
    assert np.abs(oracle.apply_A(dims, mass, fat, lng, be) - lam * be).max() < 1e-13 * lam
    x, info = oracle.cg(dims, mass, fat, lng, be, tol=1e-12)
    assert info["iters"] == 1 and info["converged"]
    assert np.abs(x - be / lam).max() < 1e-12 * np.abs(be / lam).max()


@pytest.mark.parametrize("anti", [True, False])
def test_free_field_cg_vs_fft(anti):
    dims = (4, 6, 8, 10)
    c1, c3, mass = 0.8, 0.2, 0.1
    fat, lng = synth.unit_links(dims, c1, c3, antiperiodic_t=anti)
    b = synth.source(dims, 2001)
    xe, xo = freefield.fft_solve(dims, b, mass, c1, c3, anti)
    assert np.abs(xo).max() < 1e-12 * np.abs(xe).max()  # even source -> even solution
    x, info = oracle.cg(dims, mass, fat, lng, b, tol=1e-12)
    assert info["converged"] and info["true_rel"] <= 1e-12
    assert np.linalg.norm(x - xe) / np.linalg.norm(xe) < 1e-10


# ---------------------------------------------------------------- invariants
@pytest.mark.parametrize("dims", DIMS_SMALL)
def test_antihermiticity(dims):
    fat, lng = synth.links(dims, 1000)
    r = rng(11)
    Vh = int(np.prod(dims)) // 2
    xe, yo = cvec(r, (Vh, 3)), cvec(r, (Vh, 3))
    lhs = np.vdot(yo, oracle.dslash(dims, fat, lng, xe, 1))       # <y_o, D_oe x_e>
    rhs = -np.vdot(oracle.dslash(dims, fat, lng, yo, 0), xe)      # -<D_eo y_o, x_e>
    assert abs(lhs - rhs) <= 1e-13 * np.linalg.norm(yo) * np.linalg.norm(oracle.dslash(dims, fat, lng, xe, 1))
    # A Hermitian and bounded below by 4 m^2
    m = 0.05
    ue, ve = cvec(r, (Vh, 3)), cvec(r, (Vh, 3))
    a1 = np.vdot(ue, oracle.apply_A(dims, m, fat, lng, ve))
    a2 = np.vdot(oracle.apply_A(dims, m, fat, lng, ue), ve)
    assert abs(a1 - a2) <= 1e-12 * abs(a1)
    q = np.vdot(ue, oracle.apply_A(dims, m, fat, lng, ue))
    assert abs(q.imag) < 1e-10 * abs(q) and q.real >= 4 * m * m * np.vdot(ue, ue).real


def gauge_transform(dims, fat, lng, g):
    """F_mu(n) -> g(n) F_mu(n) g(n+mu)^dag, L_mu(n) -> g(n) L_mu(n) g(n+3mu)^dag."""
    c = lattice.coords(dims)
    f2, l2 = np.empty_like(fat), np.empty_like(lng)
    for mu in range(4):
        for hop, U, out in ((1, fat, f2), (3, lng, l2)):
            d = c.copy()
            d[:, mu] = (d[:, mu] + hop) % dims[mu]
            nb = lattice.lex_of(d, dims)
            out[mu] = g @ U[mu] @ g[nb].conj().transpose(0, 2, 1)
    return f2, l2


@pytest.mark.parametrize("dims", DIMS_SMALL)
def test_gauge_covariance(dims):
    fat, lng = synth.links(dims, 1000)
    V = int(np.prod(dims))
    g = synth.haar(99, V)
    f2, l2 = gauge_transform(dims, fat, lng, g)
    r = rng(3)
    psi = cvec(r, (V, 3))
    gpsi = np.einsum("nab,nb->na", g, psi)
    for p in (0, 1):
        src = lattice.split(dims, psi)[1 - p]
        gsrc = lattice.split(dims, gpsi)[1 - p]
        gp = lattice.split(dims, g)[p]
        lhs = oracle.dslash(dims, f2, l2, gsrc, p)
        rhs = np.einsum("nab,nb->na", gp, oracle.dslash(dims, fat, lng, src, p))
        assert np.abs(lhs - rhs).max() < 1e-13 * np.abs(rhs).max()


# ---------------------------------------------------------------- brute force 4^4
@pytest.fixture(scope="module")
def dense44():
    dims = (4, 4, 4, 4)
    fat, lng = synth.links(dims, 1000)
    return dims, fat, lng, dense.dense_D(dims, fat, lng)


def test_dense_antihermitian_and_matvec(dense44):
    dims, fat, lng, D = dense44
    assert np.abs(D + D.conj().T).max() < 1e-15
    Deo, Doe = dense.blocks(dims, D)
    r = rng(1)
    Vh = 128
    for p, blk in ((0, Deo), (1, Doe)):
        src = cvec(r, (Vh, 3))
        got = oracle.dslash(dims, fat, lng, src, p).reshape(-1)
        assert np.abs(got - blk @ src.reshape(-1)).max() < 1e-13
    # parity blocks are the only nonzero blocks
    e, o = dense.color_index(dims, 0), dense.color_index(dims, 1)
    assert np.abs(D[np.ix_(e, e)]).max() == 0 and np.abs(D[np.ix_(o, o)]).max() == 0


def test_dense_cg_vs_lu_and_spectrum(dense44):
    dims, fat, lng, D = dense44
    mass = 0.05
    A = dense.dense_A(dims, D, mass)
    ev = np.linalg.eigvalsh(A)
    assert ev.min() >= 4 * mass * mass * (1 - 1e-12)
    b = synth.source(dims, 2064)
    x_lu = np.linalg.solve(A, b.reshape(-1)).reshape(-1, 3)
    x, info = oracle.cg(dims, mass, fat, lng, b, tol=1e-13)
    assert info["converged"]
    kappa = ev.max() / ev.min()
    assert np.linalg.norm(x - x_lu) / np.linalg.norm(x_lu) <= kappa * 1e-13
    # A applied by the oracle equals the dense A
    assert np.abs(oracle.apply_A(dims, mass, fat, lng, b).reshape(-1) - A @ b.reshape(-1)).max() < 1e-12


def test_dense_multishift(dense44):
    """Multi-shift reference: one source, several masses, each an independent CG (Sec. 3)."""
    dims, fat, lng, D = dense44
    b = synth.source(dims, 2064)
    for m in synth.log_masses(4, 0.02, 0.2):
        A = dense.dense_A(dims, D, m)
        x_lu = np.linalg.solve(A, b.reshape(-1)).reshape(-1, 3)
        x, info = oracle.cg(dims, m, fat, lng, b, tol=1e-12)
        assert info["converged"] and info["true_rel"] <= 1e-12
        assert np.linalg.norm(x - x_lu) / np.linalg.norm(x_lu) < 1e-9


# ---------------------------------------------------------------- the pins catch mistakes
def test_pins_reject_planted_mistakes(dense44):
    """Mistakes planted in a copy of the dense operator are caught by the pins above."""
    dims, fat, lng, D = dense44
    # transposed link: gauge covariance fails
    V = 256
    g = synth.haar(5, V)
    f2, l2 = gauge_transform(dims, fat, lng, g)
    Dt = dense.dense_D(dims, fat.transpose(0, 1, 3, 2).copy(), lng)
    Dt2 = dense.dense_D(dims, f2.transpose(0, 1, 3, 2).copy(), l2)
    G = np.zeros((3 * V, 3 * V), complex)
    for n in range(V):
        G[3 * n:3 * n + 3, 3 * n:3 * n + 3] = g[n]
    assert np.abs(Dt2 @ G - G @ Dt).max() > 1e-3
    # wrong sign on the backward terms: anti-hermiticity fails
    c = lattice.coords(dims)
    Dfwd = np.zeros_like(D)
    for n in range(V):
        for mu in range(4):
            for hop, U in ((1, fat), (3, lng)):
                d = c[n].copy()
                d[mu] = (d[mu] + hop) % dims[mu]
                f = int(lattice.lex_of(d, dims))
                Dfwd[3 * n:3 * n + 3, 3 * f:3 * f + 3] += U[mu, n]
    Dbad = 2 * Dfwd - D  # forward terms kept, backward terms with flipped sign
    assert np.abs(Dbad + Dbad.conj().T).max() > 1e-1
    # dropped Naik term: the free-field closed form fails
    fat_u, lng_u = synth.unit_links(dims, 0.7, 0.3)
    Ds = dense.dense_D(dims, fat_u, lng_u * 0)
    Dw = dense.dense_D(dims, fat_u, lng_u)
    assert np.abs(Ds - Dw).max() > 0.1  # dropped Naik term changes the free field
    k = [1, 0, 2, 1]
    psi = freefield.plane_wave(dims, k, [1, 0.5j, -0.2])
    want = freefield.dslash_plane_wave(dims, k, [1, 0.5j, -0.2], 0.7, 0.3)
    assert np.abs(Ds @ psi.reshape(-1) - want.reshape(-1)).max() > 1e-2
    assert np.abs(Dw @ psi.reshape(-1) - want.reshape(-1)).max() < 1e-13


# ---------------------------------------------------------------- the componentwise error scale
def _walk_scale(dims, fat, lng, src, p, h, dagger=True):
    """Error scale of the output components at site (parity p, index h), by an
    explicit walk over the 16 terms of the operator (Sec. 3): each term is the
    matrix T that multiplies a neighbour vector -- F_mu(n) at n+mu,
    -F_mu(n-mu)^dag at n-mu, L_mu(n) at n+3mu, -L_mu(n-3mu)^dag at n-3mu --
    and contributes sum_b |T_ab| |psi_b| to component a.  The backward
    matrices are formed as explicit conjugate transposes; dagger=False plants
    the mistake of using the untransposed matrix there."""
    c = lattice.coords(dims)
    n = int(lattice.parity_sites(dims, p)[h])
    out = np.zeros(3)
    for mu in range(4):
        for hop, U in ((1, fat), (3, lng)):
            for sgn in (+1, -1):
                d = c[n].copy()
                d[mu] = (d[mu] + sgn * hop) % dims[mu]
                m = int(lattice.lex_of(d, dims))
                if sgn > 0:
                    T = U[mu, n]
                else:
                    T = -(U[mu, m].conj().T if dagger else U[mu, m])
                psi = src[m >> 1]
                out += np.abs(T) @ np.abs(psi)
    return out


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (6, 4, 4, 8), (8, 8, 8, 8)])
def test_scale_bounds_the_output(dims):
    """|(D psi)_i| <= a_i: the scale sums the moduli of the very products that D adds."""
    fat, lng = synth.links(dims, 1200)
    src = synth.source(dims, 1201)
    for p in (0, 1):
        y = oracle.dslash(dims, fat, lng, src, p)
        a = oracle.dslash_scale(dims, fat, lng, src, p)
        assert np.all(np.abs(y) <= a * (1 + 1e-14))
        assert np.all(a > 0)


def test_scale_free_field_closed_form():
    """Unit links c1*1 and c3*1 (phases folded, so each term is +-|c| times the
    identity): a(n)_a = 8 (|c1| + |c3|) |psi_a| summed over the 8 one-hop and
    the 8 three-hop neighbours' a-th components."""
    dims = (8, 8, 8, 8)
    c1, c3 = 0.7, -0.3
    fat, lng = synth.unit_links(dims, c1, c3)
    # a source of unit modulus in every component: the neighbours' moduli are all 1
    r = rng(5)
    src = np.exp(2j * np.pi * r.random((int(np.prod(dims)) // 2, 3)))
    for p in (0, 1):
        a = oracle.dslash_scale(dims, fat, lng, src, p)
        assert np.abs(a - 8 * (abs(c1) + abs(c3))).max() < 1e-13


@pytest.mark.parametrize("dims", [(8, 8, 8, 8), (8, 10, 8, 12)])
def test_scale_matches_an_explicit_walk(dims):
    """Every extent >= 8 (and not 6), so the 16 neighbours of a site are distinct
    and no two terms alias; the oracle's scale equals the walk at sampled sites,
    and the two planted mistakes (untransposed backward matrices, every term
    counted twice) are far from it."""
    fat, lng = synth.links(dims, 1300)
    src = synth.source(dims, 1301)
    vh = int(np.prod(dims)) // 2
    r = rng(9)
    worst_planted = 0.0
    for p in (0, 1):
        a = oracle.dslash_scale(dims, fat, lng, src, p)
        for h in r.choice(vh, 24, replace=False):
            want = _walk_scale(dims, fat, lng, src, p, h)
            assert np.abs(a[h] - want).max() <= 1e-13 * want.max(), (p, h)
            planted = _walk_scale(dims, fat, lng, src, p, h, dagger=False)
            worst_planted = max(worst_planted, np.abs(a[h] - planted).max() / want.max())
            assert np.abs(2 * want - a[h]).max() > 0.5 * want.max()
    assert worst_planted > 1e-2


# ---------------------------------------------------------------- golden: the paper's printed counts
def test_golden_paper_counts():
    """The counts and sizes printed in Sec. 3-5 (tests/golden/paper_counts.json),
    derived again here, and the byte model behind every GB/s the library reports."""
    import json
    import os
    import paper_1411_2087_amd as hq
    with open(os.path.join(os.path.dirname(__file__), "golden", "paper_counts.json")) as f:
        g = json.load(f)
    d, s = g["dslash_per_site"], g["storage"]
    # a 3x3 complex matrix times a 3-vector: 9 complex products (4 mul + 2 add each)
    # and 6 complex accumulations (2 add each)
    assert 9 * 4 == d["matvec_real_multiplies"] and 9 * 2 + 6 * 2 == d["matvec_real_adds"]
    assert 3 * 2 == d["vector_add_real_adds"]
    assert d["matrices"] * d["matvec_real_multiplies"] == d["real_multiplies"]
    flops = d["matrices"] * (d["matvec_real_multiplies"] + d["matvec_real_adds"]) + \
        d["vector_adds"] * d["vector_add_real_adds"]
    assert flops == d["flops"] == oracle.FLOPS_PER_SITE
    # the printed "576 real adds" is a slip: the adds are 16*30 + 15*6 = 570
    assert flops - d["real_multiplies"] == 570
    operands = d["matrices"] * 18 + d["vectors_in"] * 6
    assert operands == d["input_operands"]
    assert round(flops / operands, 2) == d["flops_per_operand"]
    assert round(flops / (4 * operands), 2) == d["flops_per_byte_sp"]
    assert int(100 * flops / (8 * operands)) / 100 == d["flops_per_byte_dp"]
    assert 3 * 2 * 8 == s["dp_vector_bytes"] and 3 * s["dp_vector_bytes"] == s["dp_matrix_bytes"]
    for nm, b in g["multishift"]["bytes_per_site"].items():
        assert (36 + 2 * int(nm)) * s["dp_vector_bytes"] == b
    # algorithmic bytes per output site: links once, the 16 neighbour vectors
    # counted as one source read, one output write
    vec, mat = s["dp_vector_bytes"], s["dp_matrix_bytes"]
    two_row = mat * s["grows_compressed"] // s["grows_uncompressed"]
    assert hq.DSLASH_BYTES_PER_SITE[hq.HISQ_F64] == d["matrices"] * mat + 2 * vec == 2400
    assert hq.DSLASH_BYTES_PER_SITE[hq.HISQ_F32] == (d["matrices"] * mat + 2 * vec) // 2
    assert hq.DSLASH_BYTES_PER_SITE[hq.HISQ_F64C] == 8 * mat + 8 * two_row + 2 * vec == 2016
    assert hq.DSLASH_BYTES_PER_SITE[hq.HISQ_F32C] == (8 * mat + 8 * two_row + 2 * vec) // 2
    # 16-bit links: 18 half-words + one FP32 scale per matrix, FP32 vectors
    assert hq.DSLASH_BYTES_PER_SITE[hq.HISQ_F16S] == hq.DSLASH_BYTES_PER_SITE[hq.HISQ_I16S] == \
        d["matrices"] * (18 * 2 + 4) + 2 * vec // 2 == 688
