"""The C-ABI library loads and exports every symbol include/hisq.h declares;
host-side validation paths (no GPU work) return the documented codes."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hisq.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?(?:int|size_t|char|void)\s*\*?\s*(\w+)\s*\(", src, flags=re.M)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for f in ("dslash_apply", "cg_solve", "cg_solve_multi", "hisq_pack_links", "hisq_last_error"):
        assert f in names


def test_library_exports_every_declared_symbol():
    import paper_1411_2087_amd as hq
    lib = ctypes.CDLL(hq.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, f"not exported: {missing}"
    for n in hq.EXPORTED:
        assert n in declared_functions()


def test_validation_without_gpu():
    import paper_1411_2087_amd as hq
    lib = hq._lib
    dims_bad = (ctypes.c_int * 4)(4, 4, 4, 5)
    dims_ok = (ctypes.c_int * 4)(4, 4, 4, 4)
    p1, p2 = ctypes.c_void_p(0x1000), ctypes.c_void_p(0x2000)
    assert lib.dslash_apply(p1, p1, p1, p2, 0, dims_bad, 0, None) == -2
    assert b"even" in lib.hisq_last_error()
    assert lib.dslash_apply(p1, p1, p1, p1, 0, dims_ok, 0, None) == -3
    assert lib.dslash_apply(None, p1, p1, p2, 0, dims_ok, 0, None) == -1
    assert lib.dslash_apply(p1, p1, p1, p2, 3, dims_ok, 0, None) == -1
    assert lib.dslash_apply(p1, p1, p1, p2, 0, dims_ok, 7, None) == -1
    assert lib.hisq_pack_links(p1, p1, dims_bad, 0, p1, p2, None) == -2
    assert lib.hisq_pack_links(p1, p1, dims_ok, 0, p1, p1, None) == -3
    assert lib.hisq_apply_A(0.1, p1, p1, p1, p1, p2, dims_ok, 0, None) == -3
    dims_small = (ctypes.c_int * 4)(2, 4, 4, 4)
    assert lib.dslash_apply(p1, p1, p1, p2, 0, dims_small, 0, None) == -2


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (6, 6, 6, 6), (32, 32, 32, 32), (48, 48, 48, 96)])
def test_packed_sizes(dims):
    import paper_1411_2087_amd as hq
    vh = int(np.prod(dims)) // 2
    ntiles = -(-vh // 64)
    # the fat field is the larger one for the two-row forms (their long field is smaller)
    for prec, per_matrix in ((0, 144), (1, 72), (2, 40), (3, 40), (4, 144), (5, 72), (6, 40)):
        assert hq.hisq_packed_link_bytes(dims, prec) == 2 * ntiles * 64 * 8 * per_matrix
    assert hq.hisq_packed_link_bytes((4, 4, 4, 3), 0) == 0
    assert hq.hisq_packed_link_bytes(dims, 7) == 0


def test_workspace_sizes():
    import paper_1411_2087_amd as hq
    dims = (8, 8, 8, 8)
    # plain: r, p, t (FP64); mixed: r, t (FP64) and x, r, p, t (FP32) -- A p stays in registers
    assert hq.hisq_workspace_bytes("cg", dims, 1, 0) >= 3 * 2048 * 48
    assert hq.hisq_workspace_bytes("cg", dims, 1, 1) >= 2 * 2048 * 48 + 4 * 2048 * 24
    # fat paths: three one-direction link fields
    assert hq.hisq_workspace_bytes("fat_paths", dims, 0, 0) >= 3 * 4096 * 144
    assert hq.hisq_workspace_bytes("nope", dims, 1, 0) == 0
    assert hq.hisq_workspace_bytes("cg", (4, 4, 4, 5), 1, 0) == 0
    assert hq.hisq_workspace_bytes("cg", dims, 1, 6) == hq.hisq_workspace_bytes("cg", dims, 1, 1)
    assert hq.hisq_workspace_bytes("cg", dims, 1, 7) == 0


def test_cg_option_validation_without_gpu():
    """The reliable-update trigger must be below 1; <= 0 selects the inner links' default. Rejected
    before any GPU work, as are unknown modes and (for the batched solver) half-float inner links."""
    import paper_1411_2087_amd as hq
    lib = hq._lib
    dims = (ctypes.c_int * 4)(4, 4, 4, 4)
    p = [ctypes.c_void_p(0x1000 * (i + 1)) for i in range(6)]
    st = hq.CGStats()
    for delta, mode, want in ((1.0, 1, -1), (2.5, 3, -1), (0.5, 9, -1)):
        o = hq.CGOpts(mode=mode, max_iter=0, check_every=0, use_graph=1, delta=delta)
        rc = lib.cg_solve(0.1, 1e-10, p[0], p[1], p[2], p[3], p[4], p[5], dims, ctypes.byref(o), None, 0,
                          ctypes.byref(st), None)
        assert rc == want and st.status == want, (delta, mode, rc)
        assert b"delta" in lib.hisq_last_error() or b"mode" in lib.hisq_last_error()
    # a valid trigger (or the default) passes these checks and stops at the missing workspace
    for delta in (0.0, 0.7, -1.0):
        o = hq.CGOpts(mode=3, max_iter=0, check_every=0, use_graph=1, delta=delta)
        assert lib.cg_solve(0.1, 1e-10, p[0], p[1], p[2], p[3], p[4], p[5], dims, ctypes.byref(o), None, 0,
                            ctypes.byref(st), None) == -7
    masses = (ctypes.c_double * 2)(0.01, 0.1)
    for delta, mode, want in ((1.0, 0, -1), (0.1, hq.HISQ_CG_MIXED_F16S, -1), (0.0, hq.HISQ_CG_MIXED_I16SC, -7)):
        o = hq.CGOpts(mode=mode, max_iter=0, check_every=0, use_graph=1, delta=delta)
        rc = lib.cg_solve_multi(2, masses, 1e-10, hq.HISQ_MULTI_RHS, p[0], p[1], p[2], p[3], p[4], p[5], dims,
                                ctypes.byref(o), None if want == -7 else p[0], 0 if want == -7 else 1 << 40,
                                None, None)
        assert rc == want, (delta, mode, rc)


def test_shift_and_dot_validation_without_gpu():
    """shift_tol must be below 1 (MULTI_SHIFT's shifted-phase stop); the dot product needs its
    fixed-size workspace.  Both are refused before any GPU work."""
    import paper_1411_2087_amd as hq
    lib = hq._lib
    dims = (ctypes.c_int * 4)(4, 4, 4, 4)
    p = [ctypes.c_void_p(0x1000 * (i + 1)) for i in range(6)]
    masses = (ctypes.c_double * 2)(0.01, 0.1)
    o = hq.CGOpts(mode=1, max_iter=0, check_every=0, use_graph=1, delta=0.0, shift_tol=1.0, shift_only=1)
    rc = lib.cg_solve_multi(2, masses, 1e-10, hq.HISQ_MULTI_SHIFT, p[0], p[1], p[2], p[3], p[4], p[5], dims,
                            ctypes.byref(o), p[0], 1 << 40, None, None)
    assert rc == -1 and b"shift_tol" in lib.hisq_last_error()
    o.shift_tol = 1e-4
    rc = lib.cg_solve_multi(2, masses, 1e-10, hq.HISQ_MULTI_SHIFT, p[0], p[1], p[2], p[3], p[4], p[5], dims,
                            ctypes.byref(o), None, 0, None, None)
    assert rc == -7
    need = hq.hisq_workspace_bytes("dot", (4, 4, 4, 4))
    assert need == 2 * 8 * 1024 + 256
    out = (ctypes.c_double * 2)()
    assert lib.hisq_dot(p[0], p[1], 10, 0, out, None, 0, None) == -7
    assert lib.hisq_dot(p[0], p[1], 10, 0, out, p[2], need - 1, None) == -7
    assert lib.hisq_dot(p[0], p[1], -1, 0, out, p[2], need, None) == -1


def test_dot_noalloc_validation_without_gpu():
    """The no-allocation dot product refuses bad sizes before touching a GPU."""
    import paper_1411_2087_amd as hq
    lib = hq._lib
    p = [ctypes.c_void_p(0x1000 * (i + 1)) for i in range(2)]
    out = (ctypes.c_double * 2)()
    assert lib.hisq_dot_noalloc(p[0], p[1], -1, 0, out, None) == -1
    assert lib.hisq_dot_noalloc(p[0], p[1], 1 << 38, 0, out, None) == -1 and b"2^37" in lib.hisq_last_error()
    assert lib.hisq_dot_noalloc(None, p[1], 10, 0, out, None) == -1
    assert lib.hisq_dot_noalloc(p[0], p[1], 10, 9, out, None) == -1


def test_alignment_validation_without_gpu():
    """Fields, links and workspaces are read with 16-byte loads: every entry point refuses a device pointer
    that is not 16-byte aligned, before any GPU work."""
    import paper_1411_2087_amd as hq
    lib = hq._lib
    dims = (ctypes.c_int * 4)(4, 4, 4, 4)
    p = [ctypes.c_void_p(0x10000 * (i + 1)) for i in range(8)]
    bad = ctypes.c_void_p(0x10008)
    big = 1 << 40
    out = (ctypes.c_double * 2)()
    coeff = (ctypes.c_double * 5)(1, 0, 0, 0, 0)
    st = hq.CGStats()
    o = hq.CGOpts(mode=0, max_iter=0, check_every=0, use_graph=1, delta=0.0)
    masses = (ctypes.c_double * 2)(0.01, 0.1)
    best, us = ctypes.c_int(), (ctypes.c_double * 16)()
    calls = {
        "hisq_pack_links": lambda: lib.hisq_pack_links(p[0], p[1], dims, 0, bad, p[2], None),
        "dslash_apply": lambda: lib.dslash_apply(p[0], p[1], bad, p[2], 0, dims, 0, None),
        "hisq_apply_A": lambda: lib.hisq_apply_A(0.1, p[0], p[1], p[2], p[3], bad, dims, 0, None),
        "hisq_dot": lambda: lib.hisq_dot(p[0], p[1], 10, 0, out, bad, big, None),
        "hisq_dot_noalloc": lambda: lib.hisq_dot_noalloc(bad, p[1], 10, 0, out, None),
        "hisq_tune_dslash": lambda: lib.hisq_tune_dslash(p[0], bad, p[1], p[2], dims, 0, 1, ctypes.byref(best), us,
                                                         None),
        "cg_solve": lambda: lib.cg_solve(0.1, 1e-10, p[0], p[1], None, None, bad, p[2], dims, ctypes.byref(o), p[3],
                                         big, ctypes.byref(st), None),
        "cg_solve_multi": lambda: lib.cg_solve_multi(2, masses, 1e-10, hq.HISQ_MULTI_RHS, p[0], p[1], p[2], p[3],
                                                     p[4], p[5], dims, None, bad, big, None, None),
        "hisq_dslash_multi": lambda: lib.hisq_dslash_multi(p[0], p[1], p[2], bad, 0, 8, dims, p[3], big, None),
        "hisq_tune_multi": lambda: lib.hisq_tune_multi(p[0], p[1], p[2], p[3], dims, 8, bad, big, 1,
                                                       ctypes.byref(best), us, None),
        "net_forward": lambda: lib.net_forward(p[0], p[1], 4, p[2], p[3], bad, big, 1, dims, None),
        "net_backward acts": lambda: lib.net_backward(p[0], p[1], 4, bad, big, p[2], p[3], None, 1, dims, p[4], big,
                                                      None),
        "net_backward workspace": lambda: lib.net_backward(p[0], p[1], 4, p[2], big, p[3], p[4], None, 1, dims, bad,
                                                           big, None),
        "net_transport": lambda: lib.net_transport(p[0], bad, p[1], 4, 1, dims, None),
        "net_loss": lambda: lib.net_loss(p[0], bad, 1, dims, None, None, p[1], big, None),
        "net_adam_step": lambda: lib.net_adam_step(p[0], p[1], p[2], bad, 10, 1e-3, 1, None),
        "fcg_solve": lambda: lib.fcg_solve(0.1, 1e-10, p[0], p[1], p[2], p[3], 4, p[4], p[5], dims, None, bad, big,
                                           ctypes.byref(st), None),
        "hisq_three_link": lambda: lib.hisq_three_link(bad, p[0], dims, None),
        "hisq_fat_paths": lambda: lib.hisq_fat_paths(p[0], coeff, p[1], dims, bad, big, None),
        "hisq_fold_links": lambda: lib.hisq_fold_links(bad, dims, 1, 1, None),
        "hisq_read_probe": lambda: lib.hisq_read_probe(bad, 1 << 20, p[0], 1 << 20, 1, us, None),
    }
    for name, call in calls.items():
        assert call() == -1, name
        assert b"16-byte aligned" in lib.hisq_last_error(), (name, lib.hisq_last_error())

