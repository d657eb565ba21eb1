"""CPU ORACLE -- TEST INFRASTRUCTURE ONLY.

A plain, slow, FP64 reference for the staggered (HISQ) Dslash, the even-odd
normal operator and the conjugate-gradient solves, used only by `tests/`, the
package smoke check and the benchmark's CPU-baseline leg.  It shares no code
with the GPU library (`paper_1411_2087_amd`) and never imports it.

Contents
  this module   ctypes wrapper of liboracle.so (C, FP64, OpenMP over sites):
                dslash, componentwise error scale, A = 4m^2 - D_eo D_oe, CG
  dense.py      brute-force dense D for tiny lattices, built entry by entry
  freefield.py  closed forms for unit links (plane-wave eigenvalues, FFT solve)
  net.py        gauge-covariant network: FP64 forward/backward, BF16 emulation, Adam
  fcg.py        flexible CG with a preconditioner, and multi-shift reference

Paper: Li & Gottlieb, "Staggered Dslash Performance on Intel Xeon Phi
Architecture" (Lattice 2014).  Sec. 3 defines the per-site work of the
improved staggered Dslash (16 links, 16 neighbour vectors, 1146 flops) and the
CG / multishift CG context; Sec. 4 the even-odd preconditioning and the
staggered phases folded into the links.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

# Per-site counts the paper states (Sec. 3).
FLOPS_PER_SITE = 1146          # 16 mat-vec (36 mul + 30 add) + 15 vector adds (6 adds)
INPUT_OPERANDS_PER_SITE = 384  # 16 matrices * 18 reals + 16 vectors * 6 reals
BYTES_DP_VECTOR = 48           # 3 complex doubles
BYTES_DP_MATRIX = 144          # 9 complex doubles


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    _lib = load_library(_LIB_PATH)
    return _lib


def load_library(path):
    """ctypes handle of an oracle build at `path` (the checker, or the benchmark's timing build), with the
    prototypes set; every function below takes it as `lib` (default: the checker)."""
    lib = ctypes.CDLL(path)
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int)
    lib.or_dslash.argtypes = [ip, dp, dp, dp, dp, ctypes.c_int]
    lib.or_dslash.restype = None
    lib.or_dslash_absscale.argtypes = [ip, dp, dp, dp, dp, ctypes.c_int]
    lib.or_dslash_absscale.restype = None
    lib.or_apply_A.argtypes = [ip, ctypes.c_double, dp, dp, dp, dp, dp]
    lib.or_apply_A.restype = None
    lib.or_norm2.argtypes = [ctypes.c_int64, dp]
    lib.or_norm2.restype = ctypes.c_double
    lib.or_dot.argtypes = [ctypes.c_int64, dp, dp, dp]
    lib.or_dot.restype = None
    lib.or_true_residual.argtypes = [ip, ctypes.c_double, dp, dp, dp, dp]
    lib.or_true_residual.restype = ctypes.c_double
    lib.or_cg.argtypes = [ip, ctypes.c_double, ctypes.c_double, ctypes.c_int, dp, dp, dp, dp,
                          ctypes.POINTER(ctypes.c_int), dp, dp]
    lib.or_cg.restype = ctypes.c_int
    lib.or_num_threads.argtypes = []
    lib.or_num_threads.restype = ctypes.c_int
    lib.or_set_num_threads.argtypes = [ctypes.c_int]
    lib.or_set_num_threads.restype = None
    return lib


def _L(dims):
    return (ctypes.c_int * 4)(*[int(v) for v in dims])


def _dp(a):
    if a is None:
        return None
    assert a.flags["C_CONTIGUOUS"], "oracle arrays must be C-contiguous"
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _c128(a):
    return np.ascontiguousarray(a, dtype=np.complex128)


def _check(dims, fat, lng):
    V = int(np.prod(dims))
    assert fat.shape == (4, V, 3, 3) and lng.shape == (4, V, 3, 3), (fat.shape, dims)


def dslash(dims, fat, lng, src, parity: int, lib=None):
    """(D src) on the sites of `parity`; src lives on parity 1 - parity (Sec. 3)."""
    fat, lng, src = _c128(fat), _c128(lng), _c128(src)
    _check(dims, fat, lng)
    Vh = int(np.prod(dims)) // 2
    assert src.shape == (Vh, 3)
    out = np.empty((Vh, 3), np.complex128)
    (lib or _load()).or_dslash(_L(dims), _dp(fat), _dp(lng), _dp(src), _dp(out), int(parity))
    return out


def dslash_scale(dims, fat, lng, src, parity: int):
    """Componentwise error scale a[h, c] = sum over terms of |M_cb| |psi_b|."""
    fat, lng, src = _c128(fat), _c128(lng), _c128(src)
    Vh = int(np.prod(dims)) // 2
    out = np.empty((Vh, 3), np.float64)
    _load().or_dslash_absscale(_L(dims), _dp(fat), _dp(lng), _dp(src), _dp(out), int(parity))
    return out


def apply_A(dims, mass, fat, lng, x):
    """A x = 4 m^2 x - D_eo D_oe x on the even sites (even-odd normal operator)."""
    fat, lng, x = _c128(fat), _c128(lng), _c128(x)
    y = np.empty_like(x)
    tmp = np.empty_like(x)
    _load().or_apply_A(_L(dims), float(mass), _dp(fat), _dp(lng), _dp(x), _dp(y), _dp(tmp))
    return y


def true_residual(dims, mass, fat, lng, b, x) -> float:
    """|b - A x| / |b| in FP64."""
    fat, lng, b, x = _c128(fat), _c128(lng), _c128(b), _c128(x)
    return float(_load().or_true_residual(_L(dims), float(mass), _dp(fat), _dp(lng), _dp(b), _dp(x)))


def cg(dims, mass, fat, lng, b, tol=1e-10, max_iter=100000, x0=None, history=False, lib=None):
    """Conjugate gradient on A x = b (even sites) from x0 (default 0).

    Returns (x, info) with info = {converged, iters, true_rel[, history]}.
    """
    fat, lng, b = _c128(fat), _c128(lng), _c128(b)
    x = np.zeros_like(b) if x0 is None else _c128(x0).copy()
    it = ctypes.c_int(0)
    tr = np.zeros(1)
    hist = np.zeros(max_iter + 1) if history else None
    st = (lib or _load()).or_cg(_L(dims), float(mass), float(tol), int(max_iter), _dp(fat), _dp(lng), _dp(b), _dp(x),
                       ctypes.byref(it), _dp(tr), _dp(hist))
    info = {"converged": st == 0, "iters": it.value, "true_rel": float(tr[0])}
    if history:
        info["history"] = hist[: it.value + 1]
    return x, info


def num_threads(lib=None) -> int:
    """OpenMP threads the oracle's loops use."""
    return int((lib or _load()).or_num_threads())


def set_num_threads(n: int, lib=None):
    (lib or _load()).or_set_num_threads(int(n))


def norm2(x) -> float:
    x = _c128(x)
    return float(_load().or_norm2(x.size, _dp(x)))


def dot(x, y) -> complex:
    x, y = _c128(x), _c128(y)
    out = np.zeros(2)
    _load().or_dot(x.size, _dp(x), _dp(y), _dp(out))
    return complex(out[0], out[1])


def componentwise_error(y, y_ref, scale) -> float:
    """max_i |y_i - y*_i| / a_i with a_i the oracle's componentwise scale."""
    return float(np.max(np.abs(np.asarray(y) - y_ref) / np.maximum(scale, np.finfo(np.float64).tiny)))
