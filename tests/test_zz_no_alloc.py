"""hisq_dot_noalloc, the dot product on the library's static per-GPU scratch, against
hisq_dot on a caller workspace: the same kernels and grid, so the same bits, on
two calls in a row (the second on shorter vectors, so stale partials of the first
would show), in both vector precisions."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_dot_noalloc_matches_dot():
    import torch
    import paper_1411_2087_amd as hq
    r = np.random.default_rng(17)
    ws = torch.empty(hq.hisq_workspace_bytes("dot", (4, 4, 4, 4)), dtype=torch.uint8, device="cuda")
    for prec, dt in ((hq.HISQ_F64, np.complex128), (hq.HISQ_F32, np.complex64)):
        for n in (3 * 524288 + 7, 3 * 1000 + 1):
            x = (r.standard_normal(n) + 1j * r.standard_normal(n)).astype(dt)
            y = (r.standard_normal(n) + 1j * r.standard_normal(n)).astype(dt)
            xd, yd = torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()
            want = hq.hisq_dot(xd, yd, n, prec, ws)
            got = hq.hisq_dot_noalloc(xd, yd, n, prec)
            assert got == want, (prec, n, got, want)
            ref = np.vdot(x.astype(np.complex128), y.astype(np.complex128))
            assert abs(got - ref) <= 1e-12 * np.sqrt(n) * np.linalg.norm(x) * np.linalg.norm(y)
    z = torch.zeros(4, dtype=torch.complex128, device="cuda")
    assert hq.hisq_dot_noalloc(z, z, 0, hq.HISQ_F64) == 0
    with pytest.raises(hq.HisqError, match="HISQ_EINVAL"):
        hq.hisq_dot_noalloc(z, z, -1, hq.HISQ_F64)
    with pytest.raises(hq.HisqError, match="HISQ_EINVAL"):
        hq.hisq_dot_noalloc(z, z, 1 << 40, hq.HISQ_F64)
