"""Seeded synthetic inputs for the HISQ Dslash / even-odd CG path.

Draws and lays out random gauge links, sources and gauge transformations; it
contains none of the operator's arithmetic.  Both the CPU oracle and the GPU
library consume these arrays, so neither side generates its own inputs.

Layouts (complex128 NumPy arrays):
  links    (4, V, 3, 3)   [mu = x,y,z,t][lex][row][col], lex = x + Lx*(y + Ly*(z + Lz*t))
  vectors  (Vh, 3)        one parity, h = lex >> 1, Vh = V/2

The benchmark fields of the paper (Sec. 3, HISQ configuration generation) are
replaced by synthetic ones of the same structure: fat link
0.6*Haar SU(3) + 0.1*complex Gaussian noise, long link Haar SU(3), staggered
phases and the time boundary sign folded in (Sec. 4 describes folding the
phases into the links).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libsynth.so")
_lib = None

# Seeds of the five workloads: gauge seed 1000 + n, source seed 2000 + 64 n + rhs.
def gauge_seed(config: int) -> int:
    return 1000 + config


def source_seed(config: int, rhs: int = 0) -> int:
    return 2000 + 64 * config + rhs


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(_LIB_PATH)
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int)
    u32p = ctypes.POINTER(ctypes.c_uint32)
    lib.syn_philox4x32_10.argtypes = [u32p, u32p, u32p]
    lib.syn_links.argtypes = [ip, ctypes.c_uint64, dp, dp]
    lib.syn_unit_links.argtypes = [ip, ctypes.c_double, ctypes.c_double, dp, dp]
    lib.syn_fold.argtypes = [ip, ctypes.c_int, dp, dp]
    lib.syn_source.argtypes = [ip, ctypes.c_uint64, ctypes.c_int, dp]
    lib.syn_haar.argtypes = [ctypes.c_uint64, ctypes.c_int64, dp]
    lib.syn_gauss.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int64, dp]
    for f in (lib.syn_links, lib.syn_unit_links, lib.syn_fold, lib.syn_source, lib.syn_haar,
              lib.syn_gauss, lib.syn_philox4x32_10):
        f.restype = None
    _lib = lib
    return lib


def _dims(dims):
    d = (ctypes.c_int * 4)(*[int(v) for v in dims])
    return d


def _dp(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def check_dims(dims):
    dims = tuple(int(v) for v in dims)
    if len(dims) != 4 or any(v < 4 or v % 2 for v in dims):
        raise ValueError(f"every lattice extent must be even and >= 4, got {dims}")
    return dims


def volume(dims) -> int:
    return int(np.prod(dims))


def philox4x32_10(ctr, key):
    """Philox4x32-10 block function (Salmon et al., SC11)."""
    lib = _load()
    c = (ctypes.c_uint32 * 4)(*ctr)
    k = (ctypes.c_uint32 * 2)(*key)
    o = (ctypes.c_uint32 * 4)()
    lib.syn_philox4x32_10(c, k, o)
    return tuple(int(v) for v in o)


def links(dims, seed: int, *, fold: bool = True, antiperiodic_t: bool = True, out=None):
    """Random fat and long links (4, V, 3, 3) complex128, phases folded by default."""
    dims = check_dims(dims)
    V = volume(dims)
    fat = np.empty((4, V, 3, 3), np.complex128) if out is None else out[0]
    lng = np.empty((4, V, 3, 3), np.complex128) if out is None else out[1]
    lib = _load()
    lib.syn_links(_dims(dims), seed, _dp(fat), _dp(lng))
    if fold:
        lib.syn_fold(_dims(dims), int(antiperiodic_t), _dp(fat), _dp(lng))
    return fat, lng


def unit_links(dims, c1: float, c3: float, *, fold: bool = True, antiperiodic_t: bool = True):
    """Free-field links c1*1 (fat) and c3*1 (long), phases folded by default."""
    dims = check_dims(dims)
    V = volume(dims)
    fat = np.empty((4, V, 3, 3), np.complex128)
    lng = np.empty((4, V, 3, 3), np.complex128)
    lib = _load()
    lib.syn_unit_links(_dims(dims), float(c1), float(c3), _dp(fat), _dp(lng))
    if fold:
        lib.syn_fold(_dims(dims), int(antiperiodic_t), _dp(fat), _dp(lng))
    return fat, lng


def fold(dims, fat: np.ndarray, lng: np.ndarray, antiperiodic_t: bool = True):
    """Fold the staggered phases and time boundary sign into links, in place."""
    dims = check_dims(dims)
    _load().syn_fold(_dims(dims), int(antiperiodic_t), _dp(fat), _dp(lng))


def source(dims, seed: int, rhs: int = 0):
    """Complex Gaussian colour vectors on one parity, (Vh, 3) complex128, E|z|^2 = 1."""
    dims = check_dims(dims)
    Vh = volume(dims) // 2
    out = np.empty((Vh, 3), np.complex128)
    _load().syn_source(_dims(dims), seed, int(rhs), _dp(out))
    return out


def haar(seed: int, n: int):
    """n Haar-random SU(3) matrices, (n, 3, 3) complex128."""
    out = np.empty((n, 3, 3), np.complex128)
    _load().syn_haar(seed, int(n), _dp(out))
    return out


def gauss(seed: int, stream: int, n: int):
    """n complex Gaussians with E|z|^2 = 1."""
    out = np.empty((n,), np.complex128)
    _load().syn_gauss(seed, stream, int(n), _dp(out))
    return out


def log_masses(n: int, lo: float = 0.002, hi: float = 0.2):
    """n masses log-spaced from lo to hi inclusive (multi-RHS / multi-shift workload)."""
    if n == 1:
        return np.array([lo])
    return lo * (hi / lo) ** (np.arange(n) / (n - 1))


def thin_links(dims, seed: int):
    """Haar SU(3) thin links (4, V, 3, 3) complex128, no phases folded."""
    dims = check_dims(dims)
    return haar(seed, 4 * volume(dims)).reshape(4, volume(dims), 3, 3)
