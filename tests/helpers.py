"""Shared helpers of the GPU tests: seeded inputs, device upload, comparisons."""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

# FP tolerances (componentwise, relative to the oracle's per-component scale
# a_i = sum |M||psi| over the terms feeding component i)
TOL_F64 = 1e-13
TOL_F32 = 1e-6
TOL_F16S = 5e-3   # FP16 links carry ~2^-12 relative rounding of each entry
TOL_I16S = 5e-4   # 16-bit fixed point: steps of scale/32767
CG_TOL = 1e-10


def vh(dims):
    return int(np.prod(dims)) // 2


def fields(dims, seed=1000):
    return synth.links(dims, seed)


def say(*a):
    print(*a, flush=True)
