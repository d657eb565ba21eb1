"""GPU parity of the HISQ Dslash, the even-odd operator and the reductions
against the CPU oracle (through the C ABI)."""
import numpy as np
import pytest

from helpers import TOL_F16S, TOL_F32, TOL_F64, TOL_I16S, fields, oracle, say, synth, vh

pytestmark = pytest.mark.gpu

# 4^4: +3 aliases -1; 4x6x8x10: non-cubic (catches axis-order bugs);
# 6x6x6x6 and 6x4x4x10: Vh not a multiple of the 64-site tile (ragged tail)
DIMS = [(4, 4, 4, 4), (4, 6, 8, 10), (6, 6, 6, 6), (6, 4, 4, 10), (8, 8, 8, 8), (16, 8, 8, 12)]


@pytest.fixture(scope="module")
def hq():
    import torch
    import paper_1411_2087_amd as hq
    assert torch.cuda.is_available()
    return hq


def _dslash_gpu(hq, dims, fat, lng, src, parity, prec):
    import torch
    L = hq.fields.Links.pack(fat, lng, dims, prec)
    dt = hq.fields.VEC_DTYPE[prec]
    s = torch.from_numpy(src).to(dt).cuda()
    d = torch.full_like(s, float("nan"))
    hq.dslash_apply(L.fat, L.lng, s, d, parity, dims, prec)
    torch.cuda.synchronize()
    return d.cpu().numpy().astype(np.complex128)


@pytest.mark.parametrize("dims", DIMS)
@pytest.mark.parametrize("prec,tol", [(0, TOL_F64), (1, TOL_F32), (2, TOL_F16S), (3, TOL_I16S), (4, TOL_F64),
                                      (5, TOL_F32), (6, TOL_I16S)])
def test_dslash_parity(hq, dims, prec, tol):
    fat, lng = fields(dims, 1000 + sum(dims))
    r = np.random.default_rng(7)
    for parity in (0, 1):
        src = synth.source(dims, 3000 + parity)
        if prec not in (0, 4):
            # the FP32 kernel sees FP32 vectors; the oracle gets the same rounded values
            src = src.astype(np.complex64).astype(np.complex128)
        ref = oracle.dslash(dims, fat, lng, src, parity)
        scale = oracle.dslash_scale(dims, fat, lng, src, parity)
        got = _dslash_gpu(hq, dims, fat, lng, src, parity, prec)
        assert np.isfinite(got).all(), "output not fully written"
        err = oracle.componentwise_error(got, ref, scale)
        nrm = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        say(f"dslash dims={dims} prec={prec} parity={parity}: componentwise {err:.3e} normwise {nrm:.3e}")
        assert err <= tol


def test_dslash_32_4_full(hq):
    """Full 32^4 lattice (the bandwidth workload) against the oracle, both parities."""
    dims = (32, 32, 32, 32)
    fat, lng = fields(dims, 1002)
    for parity in (0, 1):
        src = synth.source(dims, 2128 + parity)
        ref = oracle.dslash(dims, fat, lng, src, parity)
        scale = oracle.dslash_scale(dims, fat, lng, src, parity)
        got = _dslash_gpu(hq, dims, fat, lng, src, parity, 0)
        err = oracle.componentwise_error(got, ref, scale)
        say(f"dslash 32^4 f64 parity={parity}: componentwise {err:.3e}")
        assert err <= TOL_F64


def test_free_field_on_gpu(hq):
    """The GPU Dslash reproduces the closed-form plane-wave result."""
    from oracle import freefield, lattice
    dims = (4, 6, 8, 10)
    c1, c3 = 0.7, -0.25
    fat, lng = synth.unit_links(dims, c1, c3)
    k = [1, 2, 3, 4]
    chi = np.array([1.0, 0.5j, -0.25 + 0.1j])
    psi = freefield.plane_wave(dims, k, chi)
    want = freefield.dslash_plane_wave(dims, k, chi, c1, c3)
    pe, po = lattice.split(dims, psi)
    we, wo = lattice.split(dims, want)
    assert np.abs(_dslash_gpu(hq, dims, fat, lng, po, 0, 0) - we).max() < 1e-13
    assert np.abs(_dslash_gpu(hq, dims, fat, lng, pe, 1, 0) - wo).max() < 1e-13


def test_antihermiticity_on_gpu(hq):
    dims = (8, 8, 8, 8)
    fat, lng = fields(dims)
    xe = synth.source(dims, 11)
    yo = synth.source(dims, 12)
    dx = _dslash_gpu(hq, dims, fat, lng, xe, 1, 0)
    dy = _dslash_gpu(hq, dims, fat, lng, yo, 0, 0)
    lhs, rhs = np.vdot(yo, dx), -np.vdot(dy, xe)
    assert abs(lhs - rhs) <= 1e-13 * np.linalg.norm(yo) * np.linalg.norm(dx)


@pytest.mark.parametrize("prec,tol", [(0, 1e-13), (1, 1e-5)])
def test_apply_A(hq, prec, tol):
    import torch
    dims = (6, 6, 6, 6)
    fat, lng = fields(dims)
    mass = 0.05
    x = synth.source(dims, 5)
    if prec:
        x = x.astype(np.complex64).astype(np.complex128)
    ref = oracle.apply_A(dims, mass, fat, lng, x)
    L = hq.fields.Links.pack(fat, lng, dims, prec)
    dt = hq.fields.VEC_DTYPE[prec]
    xd = torch.from_numpy(x).to(dt).cuda()
    yd, td = torch.empty_like(xd), torch.empty_like(xd)
    hq.hisq_apply_A(mass, L.fat, L.lng, xd, yd, td, dims, prec)
    got = yd.cpu().numpy().astype(np.complex128)
    rel = np.abs(got - ref).max() / np.abs(ref).max()
    say(f"apply_A prec={prec}: max rel {rel:.3e}")
    assert rel < tol


def test_dot_deterministic(hq):
    import torch
    n = 3 * 100003
    r = np.random.default_rng(3)
    x = (r.standard_normal(n) + 1j * r.standard_normal(n))
    y = (r.standard_normal(n) + 1j * r.standard_normal(n))
    xd, yd = torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()
    v1 = hq.hisq_dot(xd, yd, n, 0)
    v2 = hq.hisq_dot(xd, yd, n, 0)
    assert v1 == v2  # bitwise reproducible
    ref = np.vdot(x, y)
    assert abs(v1 - ref) < 1e-12 * np.sqrt(n) * 2
    assert hq.hisq_dot(xd, yd, 0, 0) == 0


def test_bad_arguments(hq):
    import torch
    dims = (4, 4, 4, 4)
    fat, lng = fields(dims)
    L = hq.fields.Links.pack(fat, lng, dims, 0)
    s = torch.zeros((vh(dims), 3), dtype=torch.complex128, device="cuda")
    with pytest.raises(hq.HisqError) as e:
        hq.dslash_apply(L.fat, L.lng, s, s, 0, dims, 0)
    assert e.value.code == -3
    with pytest.raises(hq.HisqError) as e:
        hq.dslash_apply(L.fat, L.lng, s, s.clone(), 0, (4, 4, 4, 5), 0)
    assert e.value.code == -2
    with pytest.raises(hq.HisqError) as e:
        hq.dslash_apply(L.fat, L.lng, s, s.clone(), 2, dims, 0)
    assert e.value.code == -1


@pytest.mark.parametrize("dims", [(6, 4, 4, 10), (16, 8, 8, 12)], ids=["ragged", "blocked-order"])
def test_all_launch_shapes_bitwise_identical(hq, dims):
    """Every launch shape of the Dslash computes the same bits (no races, no order change)."""
    import torch
    fat, lng = fields(dims)
    src = synth.source(dims, 9)
    for prec in (0, 1, 2, 3, 4, 5, 6):
        L = hq.fields.Links.pack(fat, lng, dims, prec)
        dt = hq.fields.VEC_DTYPE[prec]
        s = torch.from_numpy(src).to(dt).cuda()
        outs = []
        n = hq.hisq_dslash_shape(dims, prec, -2)
        for shape in range(n):
            hq.hisq_dslash_shape(dims, prec, shape)
            d = torch.full_like(s, float("nan"))
            hq.dslash_apply(L.fat, L.lng, s, d, 1, dims, prec)
            d2 = torch.full_like(s, float("nan"))
            hq.dslash_apply(L.fat, L.lng, s, d2, 1, dims, prec)
            torch.cuda.synchronize()
            assert torch.equal(torch.view_as_real(d), torch.view_as_real(d2))  # repeatable
            outs.append(d.cpu())
        for o in outs[1:]:
            assert torch.equal(torch.view_as_real(o), torch.view_as_real(outs[0]))
        best, us = hq.hisq_tune_dslash(L.fat, L.lng, s, torch.empty_like(s), dims, prec, reps=3)
        assert 0 <= best < n and len(us) == n and min(us) > 0
        assert hq.hisq_dslash_shape(dims, prec) == best


def test_compressed_pack_rejects_non_su3_long_links(hq):
    """Two-row packing needs +-SU(3) long links; the smeared fat field is not, and is refused."""
    dims = (4, 4, 4, 6)
    fat, lng = fields(dims)
    for prec in (hq.HISQ_F64C, hq.HISQ_F32C, hq.HISQ_I16SC):
        with pytest.raises(hq.HisqError) as e:
            hq.fields.Links.pack(fat, fat, dims, prec)
        assert e.value.code == -1
        hq.fields.Links.pack(fat, lng, dims, prec)  # Haar long links with folded signs pack


@pytest.mark.parametrize("prec,tol", [(4, TOL_F64), (5, TOL_F32), (6, TOL_I16S)], ids=["f64c", "f32c", "i16sc"])
def test_dslash_32_4_compressed(hq, prec, tol):
    """Full 32^4 lattice, two-row long links in every storage form, against the oracle."""
    dims = (32, 32, 32, 32)
    fat, lng = fields(dims, 1002)
    src = synth.source(dims, 2129)
    if prec != 4:
        src = src.astype(np.complex64).astype(np.complex128)  # the FP32 kernels see FP32 vectors
    ref = oracle.dslash(dims, fat, lng, src, 1)
    got = _dslash_gpu(hq, dims, fat, lng, src, 1, prec)
    err = oracle.componentwise_error(got, ref, oracle.dslash_scale(dims, fat, lng, src, 1))
    say(f"dslash 32^4 prec={prec} two-row long links: componentwise {err:.3e}")
    assert err <= tol


def test_read_probe_reads_every_byte_once(hq):
    """The read-rate probe's block sums add up to the sum of the buffer (every 16-byte
    word read exactly once), including a ragged tail shorter than one grid pass."""
    import torch
    n = (1 << 21) + 4 * 1000 + 2        # doubles: not a multiple of the grid's pass
    buf = torch.ones(n, dtype=torch.float64, device="cuda")
    sink = torch.zeros(8192, dtype=torch.float64, device="cuda")
    us = hq.hisq_read_probe(buf, sink, reps=2)
    assert us > 0
    assert float(sink.sum()) == float(n)
    with pytest.raises(hq.HisqError):
        hq.hisq_read_probe(buf, torch.zeros(16, dtype=torch.float64, device="cuda"))
