"""Link construction on the GPU (three-link products, path-summed one-link
matrices, phase folding; Sec. 4 of the paper) against the oracle.

Inputs are Haar SU(3) thin links, so every path product has entries of
modulus <= 1 and a sum of paths weighted by c is bounded entrywise by
sum_k |c_k| n_k (n_k paths of family k): the FP64 tolerance 1e-13 is taken
relative to that bound."""
import numpy as np
import pytest

from helpers import fields, oracle, say, synth
from oracle import links as K

pytestmark = pytest.mark.gpu

TOL = 1e-13
FAT7 = (1 / 8, 1 / 16, 1 / 64, 1 / 384, 0.0)
ODD = (0.3, -0.11, 0.037, 0.0071, -0.052)
DIMS = [(4, 4, 4, 4), (4, 6, 8, 10), (8, 8, 8, 8), (6, 4, 4, 12)]


def bound(c):
    n = K.PATH_COUNTS
    return abs(c[0]) * n["one"] + abs(c[1]) * n["3"] + abs(c[2]) * n["5"] + abs(c[3]) * n["7"] + \
        abs(c[4]) * n["lepage"]


@pytest.fixture(scope="module")
def hq():
    import paper_1411_2087_amd
    return paper_1411_2087_amd


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("dims", DIMS, ids=lambda d: "x".join(map(str, d)))
def test_three_link(hq, dims):
    import torch
    U = synth.thin_links(dims, synth.gauge_seed(7))
    out = torch.full((4, U.shape[1], 3, 3), float("nan"), dtype=torch.complex128, device="cuda")
    hq.hisq_three_link(dev(U), out, dims)
    err = np.max(np.abs(out.cpu().numpy() - K.three_link(dims, U)))
    say(f"three-link {dims}: max abs error {err:.2e}")
    assert err <= TOL


@pytest.mark.parametrize("dims", DIMS, ids=lambda d: "x".join(map(str, d)))
@pytest.mark.parametrize("coeff", [FAT7, ODD, (0.5, 0, 0, 0, 0), (0, 0, 0, 0, 1.0), (0, 1.0, 0, 0, 0)],
                         ids=["fat7", "odd", "one", "lepage", "staple3"])
def test_fat_paths(hq, dims, coeff):
    import torch
    U = synth.thin_links(dims, synth.gauge_seed(8))
    out = torch.full((4, U.shape[1], 3, 3), float("nan"), dtype=torch.complex128, device="cuda")
    ws = hq.fields.workspace("fat_paths", dims)
    hq.hisq_fat_paths(dev(U), coeff, out, dims, ws)
    err = np.max(np.abs(out.cpu().numpy() - K.fat_paths(dims, U, coeff))) / bound(coeff)
    say(f"fat paths {dims} {coeff}: max abs error / bound {err:.2e}")
    assert err <= TOL


@pytest.mark.parametrize("anti", [True, False])
@pytest.mark.parametrize("hop", [1, 3])
def test_fold(hq, hop, anti):
    dims = (4, 6, 4, 8)
    U = synth.thin_links(dims, synth.gauge_seed(9))
    d = dev(U)
    hq.hisq_fold_links(d, dims, hop, anti)
    assert np.array_equal(d.cpu().numpy(), K.fold(dims, U, hop, anti))


def test_pipeline_thin_to_dslash(hq):
    """Thin links -> GPU fat paths + three-link products -> fold -> pack -> Dslash,
    against the oracle Dslash on links built and folded by the oracle."""
    import torch
    dims = (8, 8, 8, 12)
    U = synth.thin_links(dims, synth.gauge_seed(10))
    c = (0.6, 0.05, 0.01, 0.002, -0.02)
    fat_ref = K.fold(dims, K.fat_paths(dims, U, c), 1)
    lng_ref = K.fold(dims, K.three_link(dims, U), 3)
    Ud = dev(U)
    fat = torch.empty_like(Ud)
    lng = torch.empty_like(Ud)
    hq.hisq_fat_paths(Ud, c, fat, dims, hq.fields.workspace("fat_paths", dims))
    hq.hisq_three_link(Ud, lng, dims)
    hq.hisq_fold_links(fat, dims, 1)
    hq.hisq_fold_links(lng, dims, 3)
    for prec in (hq.HISQ_F64, hq.HISQ_F64C):
        L = hq.fields.Links.pack(fat, lng, dims, prec)
        b = synth.source(dims, synth.source_seed(10))
        d = torch.full((b.shape[0], 3), float("nan"), dtype=torch.complex128, device="cuda")
        hq.dslash_apply(L.fat, L.lng, dev(b), d, 1, dims, prec)
        ref = oracle.dslash(dims, fat_ref, lng_ref, b, 1)
        err = oracle.componentwise_error(d.cpu().numpy(), ref, oracle.dslash_scale(dims, fat_ref, lng_ref, b, 1))
        say(f"pipeline {dims} prec={prec}: Dslash componentwise {err:.2e}")
        assert err <= TOL


def test_three_link_32_4(hq):
    """Full size: every matrix of the 32^4 three-link field against the oracle."""
    import torch
    dims = (32, 32, 32, 32)
    U = synth.thin_links(dims, synth.gauge_seed(11))
    out = torch.empty((4, U.shape[1], 3, 3), dtype=torch.complex128, device="cuda")
    hq.hisq_three_link(dev(U), out, dims)
    err = np.max(np.abs(out.cpu().numpy() - K.three_link(dims, U)))
    say(f"three-link 32^4: max abs error {err:.2e}")
    assert err <= TOL


def test_link_errors(hq):
    import torch
    dims = (4, 4, 4, 4)
    U = dev(synth.thin_links(dims, 1))
    with pytest.raises(hq.HisqError) as e:
        hq.hisq_three_link(U, U, dims)
    assert e.value.code == hq.HISQ_EALIAS
    with pytest.raises(hq.HisqError) as e:
        hq.hisq_fold_links(U, dims, 2)
    assert e.value.code == hq.HISQ_EINVAL
    with pytest.raises(hq.HisqError) as e:
        hq.hisq_three_link(U, torch.empty_like(U), (4, 4, 4, 5))
    assert e.value.code == hq.HISQ_EDIMS
    small = torch.empty(16, dtype=torch.uint8, device="cuda")
    with pytest.raises(hq.HisqError) as e:
        hq.hisq_fat_paths(U, FAT7, torch.empty_like(U), dims, small)
    assert e.value.code == hq.HISQ_EWORKSPACE
    with pytest.raises(hq.HisqError) as e:
        hq.hisq_fat_paths(U, (float("nan"), 0, 0, 0, 0), torch.empty_like(U), dims,
                          hq.fields.workspace("fat_paths", dims))
    assert e.value.code == hq.HISQ_EINVAL
