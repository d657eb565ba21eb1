"""Python binding of libhisq.so: the HISQ Dslash and the even-odd CG solves on MI355X.

Argument marshalling only.  Every function keeps the name of the C-ABI entry
point it calls (declared in include/hisq.h) and takes torch tensors, whose
device pointers and the current HIP stream are handed to the library; every
step of the computation runs in the library's HIP kernels.  There is no CPU
fallback: importing this package without the built library raises.

Paper: Li & Gottlieb, "Staggered Dslash Performance on Intel Xeon Phi
Architecture" (Lattice 2014), Sec. 3 (the Dslash and the CG it drives) and
Sec. 4 (even-odd preconditioning, staggered phases in the links).
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhisq.so")

HISQ_F64, HISQ_F32, HISQ_F16S, HISQ_I16S, HISQ_F64C, HISQ_F32C, HISQ_I16SC = 0, 1, 2, 3, 4, 5, 6
HISQ_CG_PLAIN_F64, HISQ_CG_MIXED_F32, HISQ_CG_MIXED_F16S, HISQ_CG_MIXED_I16S = 0, 1, 2, 3
HISQ_CG_PLAIN_F64C, HISQ_CG_MIXED_F32C, HISQ_CG_MIXED_I16SC = 4, 5, 6
HISQ_MULTI_RHS, HISQ_MULTI_SHIFT = 0, 1
HISQ_OK, HISQ_EINVAL, HISQ_EDIMS, HISQ_EALIAS, HISQ_EHIP = 0, -1, -2, -3, -4
HISQ_ENOCONV, HISQ_EBREAKDOWN, HISQ_EWORKSPACE = -5, -6, -7
STATUS = {0: "HISQ_OK", -1: "HISQ_EINVAL", -2: "HISQ_EDIMS", -3: "HISQ_EALIAS", -4: "HISQ_EHIP",
          -5: "HISQ_ENOCONV", -6: "HISQ_EBREAKDOWN", -7: "HISQ_EWORKSPACE"}

# Algorithmic bytes per output site of one Dslash (16 links, one source read,
# one output write; Sec. 3 counts 16 matrices and 16 vectors per site), and
# the paper's flop count.
DSLASH_BYTES_PER_SITE = {HISQ_F64: 16 * 144 + 48 + 48, HISQ_F32: 16 * 72 + 24 + 24, HISQ_F16S: 16 * 40 + 24 + 24,
                         HISQ_I16S: 16 * 40 + 24 + 24, HISQ_F64C: 8 * 144 + 8 * 96 + 48 + 48,
                         HISQ_F32C: 8 * 72 + 8 * 48 + 24 + 24, HISQ_I16SC: 8 * 40 + 8 * 28 + 24 + 24}
DSLASH_FLOPS_PER_SITE = 1146


class HisqError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class CGOpts(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int), ("max_iter", ctypes.c_int), ("check_every", ctypes.c_int),
                ("use_graph", ctypes.c_int), ("delta", ctypes.c_double), ("shift_tol", ctypes.c_double),
                ("shift_only", ctypes.c_int)]


class CGStats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("reliable_updates", ctypes.c_int), ("restarts", ctypes.c_int),
                ("status", ctypes.c_int), ("true_resid", ctypes.c_double), ("time_s", ctypes.c_double),
                ("fallback_used", ctypes.c_int), ("fallback_iters", ctypes.c_int),
                ("iter_resid", ctypes.c_double), ("bytes_moved", ctypes.c_double),
                ("kernel_us", ctypes.c_double * 3)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["kernel_us"] = list(self.kernel_us)
        return d


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run python paper_1411_2087_amd/build.py (hipcc, gfx950)")
    lib = ctypes.CDLL(LIB_PATH)
    vp, ip, sz, d = ctypes.c_void_p, ctypes.POINTER(ctypes.c_int), ctypes.c_size_t, ctypes.c_double
    lib.hisq_version.restype = ctypes.c_char_p
    lib.hisq_last_error.restype = ctypes.c_char_p
    lib.hisq_packed_link_bytes.argtypes = [ip, ctypes.c_int]
    lib.hisq_packed_link_bytes.restype = sz
    lib.hisq_pack_links.argtypes = [vp, vp, ip, ctypes.c_int, vp, vp, vp]
    lib.dslash_apply.argtypes = [vp, vp, vp, vp, ctypes.c_int, ip, ctypes.c_int, vp]
    lib.hisq_apply_A.argtypes = [d, vp, vp, vp, vp, vp, ip, ctypes.c_int, vp]
    lib.hisq_dot.argtypes = [vp, vp, ctypes.c_longlong, ctypes.c_int, ctypes.POINTER(ctypes.c_double), vp, sz, vp]
    lib.hisq_dot_noalloc.argtypes = [vp, vp, ctypes.c_longlong, ctypes.c_int, ctypes.POINTER(ctypes.c_double), vp]
    lib.hisq_workspace_bytes.argtypes = [ctypes.c_char_p, ip, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    lib.hisq_workspace_bytes.restype = sz
    lib.cg_solve.argtypes = [d, d, vp, vp, vp, vp, vp, vp, ip, ctypes.POINTER(CGOpts), vp, sz,
                             ctypes.POINTER(CGStats), vp]
    lib.cg_solve_multi.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_double), d, ctypes.c_int, vp, vp, vp, vp,
                                   vp, vp, ip, ctypes.POINTER(CGOpts), vp, sz, ctypes.POINTER(CGStats), vp]
    lib.hisq_tune_dslash.argtypes = [vp, vp, vp, vp, ip, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                     ctypes.POINTER(ctypes.c_double), vp]
    lib.hisq_dslash_shape.argtypes = [ip, ctypes.c_int, ctypes.c_int]
    lib.hisq_dslash_multi.argtypes = [vp, vp, vp, vp, ctypes.c_int, ctypes.c_int, ip, vp, sz, vp]
    lib.hisq_tune_multi.argtypes = [vp, vp, vp, vp, ip, ctypes.c_int, vp, sz, ctypes.c_int,
                                    ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double), vp]
    lib.hisq_multi_shape.argtypes = [ip, ctypes.c_int, ctypes.c_int]
    lib.net_weight_count.argtypes = [ctypes.c_int]
    lib.net_weight_count.restype = sz
    lib.net_act_bytes.argtypes = [ip, ctypes.c_int, ctypes.c_int]
    lib.net_act_bytes.restype = sz
    lib.net_backward_ws_bytes.argtypes = [ip, ctypes.c_int, ctypes.c_int]
    lib.net_backward_ws_bytes.restype = sz
    lib.net_forward.argtypes = [vp, vp, ctypes.c_int, vp, vp, vp, sz, ctypes.c_int, ip, vp]
    lib.net_backward.argtypes = [vp, vp, ctypes.c_int, vp, sz, vp, vp, vp, ctypes.c_int, ip, vp, sz, vp]
    lib.net_transport.argtypes = [vp, vp, vp, ctypes.c_int, ctypes.c_int, ip, vp]
    lib.net_loss.argtypes = [vp, vp, ctypes.c_int, ip, ctypes.POINTER(ctypes.c_double), vp, vp, sz, vp]
    lib.net_adam_step.argtypes = [vp, vp, vp, vp, ctypes.c_longlong, d, ctypes.c_int, vp]
    lib.fcg_solve.argtypes = [d, d, vp, vp, vp, vp, ctypes.c_int, vp, vp, ip, ctypes.POINTER(CGOpts), vp, sz,
                              ctypes.POINTER(CGStats), vp]
    lib.hisq_three_link.argtypes = [vp, vp, ip, vp]
    lib.hisq_fat_paths.argtypes = [vp, ctypes.POINTER(ctypes.c_double), vp, ip, vp, sz, vp]
    lib.hisq_fold_links.argtypes = [vp, ip, ctypes.c_int, ctypes.c_int, vp]
    lib.hisq_read_probe.argtypes = [vp, sz, vp, sz, ctypes.c_int, ctypes.POINTER(ctypes.c_double), vp]
    for name in ("hisq_three_link", "hisq_fat_paths", "hisq_fold_links", "hisq_read_probe", "hisq_pack_links",
                 "dslash_apply", "hisq_apply_A", "hisq_dot", "hisq_dot_noalloc", "cg_solve", "cg_solve_multi",
                 "hisq_tune_dslash", "hisq_dslash_shape", "hisq_dslash_multi", "hisq_tune_multi", "hisq_multi_shape",
                 "net_forward", "net_backward", "net_transport", "net_loss", "net_adam_step", "fcg_solve"):
        getattr(lib, name).restype = ctypes.c_int
    return lib


_lib = _load()

EXPORTED = ["hisq_version", "hisq_last_error", "hisq_packed_link_bytes", "hisq_pack_links", "dslash_apply",
            "hisq_apply_A", "hisq_dot", "hisq_dot_noalloc", "hisq_workspace_bytes", "cg_solve", "cg_solve_multi",
            "hisq_tune_dslash",
            "hisq_dslash_shape", "hisq_dslash_multi", "hisq_tune_multi", "hisq_multi_shape", "net_weight_count",
            "net_act_bytes", "net_backward_ws_bytes", "net_forward", "net_backward", "net_transport", "net_loss",
            "net_adam_step",
            "fcg_solve", "hisq_three_link", "hisq_fat_paths", "hisq_fold_links", "hisq_read_probe"]


def _dims(dims):
    return (ctypes.c_int * 4)(*[int(v) for v in dims])


def _ptr(t):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError("expected a torch tensor")
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _check(rc, what):
    if rc != 0:
        raise HisqError(rc, f"{what}: {_lib.hisq_last_error().decode()}")


def hisq_version() -> str:
    return _lib.hisq_version().decode()


def hisq_last_error() -> str:
    return _lib.hisq_last_error().decode()


def hisq_packed_link_bytes(dims, prec) -> int:
    return int(_lib.hisq_packed_link_bytes(_dims(dims), int(prec)))


def hisq_pack_links(fat_canon, long_canon, dims, prec, fat_out, long_out, stream=None):
    _check(_lib.hisq_pack_links(_ptr(fat_canon), _ptr(long_canon), _dims(dims), int(prec), _ptr(fat_out),
                                _ptr(long_out), _stream(stream)), "hisq_pack_links")


def hisq_read_probe(buf, sink, reps=5, stream=None) -> float:
    """Microseconds per nontemporal streaming read of the whole of `buf` (device tensor)."""
    us = ctypes.c_double()
    _check(_lib.hisq_read_probe(_ptr(buf), buf.numel() * buf.element_size(), _ptr(sink),
                                sink.numel() * sink.element_size(), int(reps), ctypes.byref(us), _stream(stream)),
           "hisq_read_probe")
    return us.value


def hisq_three_link(thin, out, dims, stream=None):
    _check(_lib.hisq_three_link(_ptr(thin), _ptr(out), _dims(dims), _stream(stream)), "hisq_three_link")


def hisq_fat_paths(thin, coeff, out, dims, workspace, stream=None):
    c = (ctypes.c_double * 5)(*[float(v) for v in coeff])
    _check(_lib.hisq_fat_paths(_ptr(thin), c, _ptr(out), _dims(dims), _ptr(workspace),
                               workspace.numel() * workspace.element_size() if workspace is not None else 0,
                               _stream(stream)), "hisq_fat_paths")


def hisq_fold_links(links, dims, hop, antiperiodic_t=True, stream=None):
    _check(_lib.hisq_fold_links(_ptr(links), _dims(dims), int(hop), int(bool(antiperiodic_t)), _stream(stream)),
           "hisq_fold_links")


def dslash_apply(fat, lng, src, dst, parity, dims, prec, stream=None):
    _check(_lib.dslash_apply(_ptr(fat), _ptr(lng), _ptr(src), _ptr(dst), int(parity), _dims(dims), int(prec),
                             _stream(stream)), "dslash_apply")


def hisq_apply_A(mass, fat, lng, x, y, tmp, dims, prec, stream=None):
    _check(_lib.hisq_apply_A(float(mass), _ptr(fat), _ptr(lng), _ptr(x), _ptr(y), _ptr(tmp), _dims(dims), int(prec),
                             _stream(stream)), "hisq_apply_A")


def hisq_dot(x, y, n, prec, workspace=None, stream=None) -> complex:
    """<x, y> over n complex entries; `workspace` (a device tensor of at least
    hisq_workspace_bytes("dot", ...) bytes) is made here when not given."""
    if workspace is None:
        workspace = torch.empty(hisq_workspace_bytes("dot", (4, 4, 4, 4)), dtype=torch.uint8, device=x.device)
    out = (ctypes.c_double * 2)()
    _check(_lib.hisq_dot(_ptr(x), _ptr(y), int(n), int(prec), out, _ptr(workspace), _nbytes(workspace),
                         _stream(stream)), "hisq_dot")
    return complex(out[0], out[1])


def hisq_dot_noalloc(x, y, n, prec, stream=None) -> complex:
    """<x, y> over n complex entries on the library's static scratch (no allocation anywhere)."""
    out = (ctypes.c_double * 2)()
    _check(_lib.hisq_dot_noalloc(_ptr(x), _ptr(y), int(n), int(prec), out, _stream(stream)), "hisq_dot_noalloc")
    return complex(out[0], out[1])


def hisq_tune_dslash(fat, lng, src, dst, dims, prec, reps=20, stream=None):
    """Time every Dslash launch shape; returns (best_shape, [microseconds per shape])."""
    n = int(_lib.hisq_dslash_shape(_dims(dims), int(prec), -2))
    best = ctypes.c_int(-1)
    us = (ctypes.c_double * n)()
    _check(_lib.hisq_tune_dslash(_ptr(fat), _ptr(lng), _ptr(src), _ptr(dst), _dims(dims), int(prec), int(reps),
                                 ctypes.byref(best), us, _stream(stream)), "hisq_tune_dslash")
    return best.value, list(us)


def hisq_dslash_shape(dims, prec, shape=-1) -> int:
    rc = int(_lib.hisq_dslash_shape(_dims(dims), int(prec), int(shape)))
    if rc < 0:
        _check(rc, "hisq_dslash_shape")
    return rc


def hisq_dslash_multi(fat, lng, src, dst, parity, nrhs, dims, workspace, stream=None):
    _check(_lib.hisq_dslash_multi(_ptr(fat), _ptr(lng), _ptr(src), _ptr(dst), int(parity), int(nrhs), _dims(dims),
                                  _ptr(workspace), workspace.numel() * workspace.element_size(), _stream(stream)),
           "hisq_dslash_multi")


def hisq_tune_multi(fat, lng, src, dst, dims, nrhs, workspace, reps=10, stream=None):
    """Time every multi-RHS Dslash shape; returns (best_shape, [microseconds per shape, -1 if n/a])."""
    best = ctypes.c_int(-1)
    us = (ctypes.c_double * int(_lib.hisq_multi_shape(_dims(dims), int(nrhs), -2)))()
    _check(_lib.hisq_tune_multi(_ptr(fat), _ptr(lng), _ptr(src), _ptr(dst), _dims(dims), int(nrhs), _ptr(workspace),
                                workspace.numel() * workspace.element_size(), int(reps), ctypes.byref(best), us,
                                _stream(stream)), "hisq_tune_multi")
    return best.value, list(us)


def hisq_multi_shape(dims, nrhs, shape=-1) -> int:
    rc = int(_lib.hisq_multi_shape(_dims(dims), int(nrhs), int(shape)))
    if rc < 0:
        _check(rc, "hisq_multi_shape")
    return rc


def hisq_workspace_bytes(solver, dims, nrhs=1, mode=0, channels=0) -> int:
    return int(_lib.hisq_workspace_bytes(solver.encode(), _dims(dims), int(nrhs), int(mode), int(channels)))


def cg_solve(mass, tol, fat, lng, fat_lo, lng_lo, b, x, dims, opts: CGOpts | None, workspace, stream=None,
             raise_on_noconv=False) -> dict:
    st = CGStats()
    rc = _lib.cg_solve(float(mass), float(tol), _ptr(fat), _ptr(lng), _ptr(fat_lo), _ptr(lng_lo), _ptr(b), _ptr(x),
                       _dims(dims), ctypes.byref(opts) if opts is not None else None, _ptr(workspace),
                       workspace.numel() * workspace.element_size(), ctypes.byref(st), _stream(stream))
    if rc != 0 and (raise_on_noconv or rc not in (-5, -6)):
        _check(rc, "cg_solve")
    d = st.as_dict()
    d["rc"] = rc
    return d


def cg_solve_multi(nrhs, masses, tol, mode, fat, lng, fat_lo, lng_lo, b, x, dims, opts: CGOpts | None, workspace,
                   stream=None, raise_on_noconv=False) -> list:
    ms = (ctypes.c_double * nrhs)(*[float(m) for m in masses])
    st = (CGStats * nrhs)()
    rc = _lib.cg_solve_multi(int(nrhs), ms, float(tol), int(mode), _ptr(fat), _ptr(lng), _ptr(fat_lo), _ptr(lng_lo),
                             _ptr(b), _ptr(x), _dims(dims), ctypes.byref(opts) if opts is not None else None,
                             _ptr(workspace), workspace.numel() * workspace.element_size(), st, _stream(stream))
    if rc != 0 and (raise_on_noconv or rc not in (-5, -6)):
        _check(rc, "cg_solve_multi")
    out = [s.as_dict() for s in st]
    for o in out:
        o["rc"] = rc
    return out


def _nbytes(t):
    return t.numel() * t.element_size()


def net_weight_count(channels) -> int:
    return int(_lib.net_weight_count(int(channels)))


def net_act_bytes(dims, channels, batch) -> int:
    return int(_lib.net_act_bytes(_dims(dims), int(channels), int(batch)))


def net_backward_ws_bytes(dims, channels, batch) -> int:
    return int(_lib.net_backward_ws_bytes(_dims(dims), int(channels), int(batch)))


def net_forward(fat, weights, channels, inp, out, acts, batch, dims, stream=None):
    _check(_lib.net_forward(_ptr(fat), _ptr(weights), int(channels), _ptr(inp), _ptr(out), _ptr(acts), _nbytes(acts),
                            int(batch), _dims(dims), _stream(stream)), "net_forward")


def net_backward(fat, weights, channels, acts, grad_out, grad_w, grad_in, batch, dims, workspace, stream=None):
    _check(_lib.net_backward(_ptr(fat), _ptr(weights), int(channels), _ptr(acts), _nbytes(acts), _ptr(grad_out),
                             _ptr(grad_w), _ptr(grad_in), int(batch), _dims(dims), _ptr(workspace),
                             _nbytes(workspace), _stream(stream)), "net_backward")


def net_transport(fat, inp, out, channels, batch, dims, stream=None):
    _check(_lib.net_transport(_ptr(fat), _ptr(inp), _ptr(out), int(channels), int(batch), _dims(dims),
                              _stream(stream)), "net_transport")


def net_loss(y, x, batch, dims, grad_y, workspace, sync=True, stream=None):
    loss = ctypes.c_double(float("nan"))
    _check(_lib.net_loss(_ptr(y), _ptr(x), int(batch), _dims(dims), ctypes.byref(loss) if sync else None,
                         _ptr(grad_y), _ptr(workspace), _nbytes(workspace), _stream(stream)), "net_loss")
    return loss.value


def net_adam_step(weights, grad_w, m, v, n_complex, lr, step, stream=None):
    _check(_lib.net_adam_step(_ptr(weights), _ptr(grad_w), _ptr(m), _ptr(v), int(n_complex), float(lr), int(step),
                              _stream(stream)), "net_adam_step")


def fcg_solve(mass, tol, fat, lng, fat32, weights, channels, b, x, dims, opts: CGOpts | None, workspace, stream=None,
              raise_on_noconv=False) -> dict:
    st = CGStats()
    rc = _lib.fcg_solve(float(mass), float(tol), _ptr(fat), _ptr(lng), _ptr(fat32), _ptr(weights), int(channels),
                        _ptr(b), _ptr(x), _dims(dims), ctypes.byref(opts) if opts is not None else None,
                        _ptr(workspace), _nbytes(workspace), ctypes.byref(st), _stream(stream))
    if rc != 0 and (raise_on_noconv or rc not in (-5, -6)):
        _check(rc, "fcg_solve")
    d = st.as_dict()
    d["rc"] = rc
    return d


from . import fields  # noqa: E402  (device buffers for packed links and vectors)
