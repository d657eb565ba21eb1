"""Device buffers for the library's inputs: packed links, vectors, workspaces.

Torch owns the device memory; packing and every computation run in libhisq.
"""
from __future__ import annotations

import numpy as np
import torch

from . import (HISQ_F16S, HISQ_F32, HISQ_F32C, HISQ_F64, HISQ_F64C, HISQ_I16S, HISQ_I16SC, hisq_pack_links,
               hisq_packed_link_bytes, hisq_workspace_bytes)

VEC_DTYPE = {HISQ_F64: torch.complex128, HISQ_F32: torch.complex64, HISQ_F16S: torch.complex64,
             HISQ_I16S: torch.complex64, HISQ_F64C: torch.complex128, HISQ_F32C: torch.complex64,
             HISQ_I16SC: torch.complex64}


def to_device(a: np.ndarray, device="cuda"):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device)


class Links:
    """Packed fat and long links of one precision on the device."""

    def __init__(self, fat, lng, dims, prec):
        self.fat, self.lng, self.dims, self.prec = fat, lng, tuple(dims), prec

    @classmethod
    def pack(cls, fat_canon, long_canon, dims, prec, device="cuda"):
        """Pack canonical complex128 links (device tensors, or NumPy arrays uploaded here)."""
        if isinstance(fat_canon, np.ndarray):
            fat_canon = to_device(fat_canon, device)
        if isinstance(long_canon, np.ndarray):
            long_canon = to_device(long_canon, device)
        nbytes = hisq_packed_link_bytes(dims, prec)
        if nbytes == 0:
            raise ValueError(f"bad dims/precision {dims} {prec}")
        fat = torch.empty(nbytes, dtype=torch.uint8, device=fat_canon.device)
        lng = torch.empty(nbytes, dtype=torch.uint8, device=fat_canon.device)
        hisq_pack_links(fat_canon, long_canon, dims, prec, fat, lng)
        return cls(fat, lng, dims, prec)

    @property
    def nbytes(self):
        return self.fat.numel() + self.lng.numel()


def empty_vector(dims, prec=HISQ_F64, device="cuda", nrhs=None):
    Vh = int(np.prod(dims)) // 2
    shape = (Vh, 3) if nrhs is None else (nrhs, Vh, 3)
    return torch.empty(shape, dtype=VEC_DTYPE[prec], device=device)


def workspace(solver, dims, nrhs=1, mode=0, channels=0, device="cuda"):
    n = hisq_workspace_bytes(solver, dims, nrhs, mode, channels)
    if n == 0:
        raise ValueError(f"no workspace size for {solver} {dims} nrhs={nrhs} mode={mode}")
    return torch.empty(n, dtype=torch.uint8, device=device)
