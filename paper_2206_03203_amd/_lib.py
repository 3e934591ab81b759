"""ctypes binding of ``include/mdp.h``: argument marshalling only.

Every function below has the name of the C entry point it calls.  Device
vectors are passed as torch tensors (their data pointers); host CSR data as
numpy arrays.  The compiled library must exist in the package directory
(``python -m paper_2206_03203_amd.build``); importing this module without it
raises ImportError — there is no fallback path.
"""

from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmdp.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2206_03203_amd.build`")

# torch brings its own HIP runtime.  Loading it first makes libmdp bind to
# that same runtime (one runtime per process); the other order would map a
# second HIP/HSA runtime whose allocations and streams torch cannot see.
import torch  # noqa: E402,F401

lib = C.CDLL(LIB_PATH)


def _hip_runtimes():
    try:
        with open("/proc/self/maps") as f:
            return sorted({ln.split()[-1] for ln in f if "libamdhip64" in ln})
    except OSError:
        return []


if len(_hip_runtimes()) > 1:
    raise ImportError("two HIP runtimes are mapped in this process (%s); import torch before "
                      "loading libmdp" % ", ".join(_hip_runtimes()))

MDP_OK, MDP_NOT_CONVERGED, MDP_PENDING, MDP_STAGNATED = 0, 1, 2, 3
MDP_EINVAL, MDP_ENONPOS_DIAG, MDP_ESINGULAR, MDP_ENAN, MDP_ENOMEM, MDP_EHIP, MDP_EBUSY = -1, -2, -3, -4, -5, -6, -7
MDP_FP64, MDP_MIXED = 0, 1
MDP_USE_X0, MDP_HOST_ONLY, MDP_NO_AUTOTUNE, MDP_GRAPHS, MDP_FALLBACK_FP64, MDP_HOST_PRODUCTS = 1, 2, 4, 8, 16, 32
MDP_BLOCK_LOWER, MDP_BLOCK_DIAG, MDP_BLOCK_UPPER = 0, 1, 2
MDP_SMOOTH_L1JACOBI, MDP_SMOOTH_GS = 0, 1
MDP_OP_A, MDP_OP_ML, MDP_OP_QOO, MDP_OP_QGG = 0, 1, 2, 3
MDP_BLOCK_OMEGA, MDP_BLOCK_GAMMA = 0, 1
MDP_MAT_A, MDP_MAT_P, MDP_MAT_R = 0, 1, 2

ERROR_NAMES = {0: "MDP_OK", 1: "MDP_NOT_CONVERGED", 2: "MDP_PENDING", 3: "MDP_STAGNATED", -1: "MDP_EINVAL",
               -2: "MDP_ENONPOS_DIAG", -3: "MDP_ESINGULAR", -4: "MDP_ENAN", -5: "MDP_ENOMEM",
               -6: "MDP_EHIP", -7: "MDP_EBUSY"}


class mdp_csr(C.Structure):
    _fields_ = [("n", C.c_int32), ("nnz", C.c_int64), ("row_ptr", C.POINTER(C.c_int32)),
                ("col", C.POINTER(C.c_int32)), ("val", C.POINTER(C.c_double))]


class mdp_options(C.Structure):
    _fields_ = [("precision", C.c_int32), ("vcycles", C.c_int32), ("pre_sweeps", C.c_int32),
                ("post_sweeps", C.c_int32), ("strength_theta", C.c_double), ("max_coarse", C.c_int32),
                ("max_dense", C.c_int32), ("max_levels", C.c_int32), ("restart", C.c_int32),
                ("max_iter", C.c_int32), ("rtol", C.c_double), ("flags", C.c_uint32),
                ("block_form", C.c_int32), ("smoother", C.c_int32)]


class mdp_stats(C.Structure):
    _fields_ = [("iters", C.c_int32), ("restarts", C.c_int32), ("converged", C.c_int32),
                ("status", C.c_int32), ("rel_res_true", C.c_double), ("rel_res_est", C.c_double),
                ("setup_ms", C.c_double), ("solve_ms", C.c_double), ("fallback", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class MdpError(RuntimeError):
    def __init__(self, code: int, where: str):
        msg = lib.mdp_last_error().decode(errors="replace")
        super().__init__(f"{where}: {ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


_vp = C.c_void_p
_ip = C.POINTER(C.c_int32)
_sig = {
    "mdp_options_default": (C.c_int, [C.POINTER(mdp_options)]),
    "mdp_setup": (C.c_int, [C.POINTER(mdp_csr), _ip, C.POINTER(mdp_options), _vp, C.POINTER(_vp)]),
    "mdp_setup_like": (C.c_int, [_vp, C.POINTER(mdp_options), _vp, C.POINTER(_vp)]),
    "mdp_setup_labeled": (C.c_int, [C.POINTER(mdp_csr), _ip, _ip, C.POINTER(mdp_options), _vp, C.POINTER(_vp)]),
    "mdp_destroy": (C.c_int, [_vp]),
    "mdp_solve": (C.c_int, [_vp, _vp, _vp, C.c_int32, C.c_int64, _vp, C.POINTER(mdp_stats)]),
    "mdp_solve_batch": (C.c_int, [C.POINTER(_vp), C.c_int32, C.POINTER(_vp), C.POINTER(_vp), _ip, _vp,
                                  C.POINTER(mdp_stats)]),
    "mdp_apply": (C.c_int, [_vp, C.c_int32, _vp, _vp, _vp]),
    "mdp_apply_noalloc": (C.c_int, [_vp, C.c_int32, _vp, _vp, _vp]),
    "mdp_info": (C.c_int, [_vp, _ip, _ip, _ip, _ip, _ip]),
    "mdp_multi_rhs_memory": (C.c_int, [_vp] + [C.POINTER(C.c_int64)] * 4),
    "mdp_residual_history": (C.c_int, [_vp, C.POINTER(C.c_double), C.c_int32, _ip]),
    "mdp_level_shape": (C.c_int, [_vp, C.c_int32, C.c_int32, C.c_int32, _ip, _ip, C.POINTER(C.c_int64)]),
    "mdp_level_export": (C.c_int, [_vp, C.c_int32, C.c_int32, C.c_int32, _ip, _ip, C.POINTER(C.c_double)]),
    "mdp_level_aggregates": (C.c_int, [_vp, C.c_int32, C.c_int32, _ip]),
    "mdp_save": (C.c_int, [_vp, C.c_char_p]),
    "mdp_load": (C.c_int, [C.c_char_p, C.POINTER(mdp_options), _vp, C.POINTER(_vp)]),
    "mdp_server_create": (C.c_int, [C.c_size_t, C.c_int32, C.POINTER(_vp)]),
    "mdp_server_register": (C.c_int, [_vp, _vp]),
    "mdp_submit": (C.c_int, [_vp, _vp, _vp, _vp, C.c_int32, C.POINTER(C.c_uint64)]),
    "mdp_poll": (C.c_int, [_vp, C.c_uint64, C.POINTER(mdp_stats)]),
    "mdp_server_destroy": (C.c_int, [_vp]),
    "mdp_server_set_grouping": (C.c_int, [_vp, C.c_int32]),
    "mdp_server_counts": (C.c_int, [_vp, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "mdp_set_allocator": (C.c_int, [_vp, _vp, _vp]),
    "mdp_tune_file": (C.c_int, [C.c_char_p]),
    "mdp_ktimer_begin": (C.c_int, [C.c_int32]),
    "mdp_ktimer_end": (C.c_int, [C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_int64), C.POINTER(C.c_double)]),
    "mdp_last_error": (C.c_char_p, []),
    "mdp_version": (C.c_char_p, []),
}
for _name, (_res, _args) in _sig.items():
    _f = getattr(lib, _name)
    _f.restype = _res
    _f.argtypes = _args

EXPORTED = tuple(_sig)


def _check(rc: int, where: str, ok=(MDP_OK,)) -> int:
    if rc not in ok:
        raise MdpError(rc, where)
    return rc


def _stream_ptr(stream) -> Optional[int]:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _dptr(t) -> int:
    return t.data_ptr()


def _rhs_pair(h: int, b, x) -> int:
    """Check that b and x are contiguous float64 device tensors of shape (n,)
    or (nrhs, n) for the system of handle h (the library cannot check the
    size of a raw device pointer); return nrhs."""
    import torch

    n = mdp_info(h)["n"]
    for name, t in (("b", b), ("x", x)):
        if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous():
            raise TypeError(f"{name} must be a contiguous float64 device tensor")
        if t.dim() not in (1, 2) or t.shape[-1] != n:
            raise ValueError(f"{name} has shape {tuple(t.shape)}; the system has {n} unknowns")
    if b.shape != x.shape:
        raise ValueError(f"b {tuple(b.shape)} and x {tuple(x.shape)} differ in shape")
    return 1 if b.dim() == 1 else b.shape[0]


def mdp_options_default(**overrides) -> mdp_options:
    o = mdp_options()
    _check(lib.mdp_options_default(C.byref(o)), "mdp_options_default")
    for k, v in overrides.items():
        if not hasattr(o, k):
            raise TypeError(f"unknown option {k}")
        setattr(o, k, v)
    return o


class _CsrHold:
    """Keeps the numpy arrays behind an mdp_csr alive during a call."""

    def __init__(self, row_ptr, col, val):
        self.row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int32)
        self.col = np.ascontiguousarray(col, dtype=np.int32)
        self.val = np.ascontiguousarray(val, dtype=np.float64)
        n = self.row_ptr.shape[0] - 1
        self.s = mdp_csr(n, int(self.row_ptr[-1]) if n >= 0 else 0,
                         self.row_ptr.ctypes.data_as(_ip), self.col.ctypes.data_as(_ip),
                         self.val.ctypes.data_as(C.POINTER(C.c_double)))


def mdp_setup(A, part, opts: Optional[mdp_options] = None, stream=None, labels=None) -> int:
    """A: scipy CSR (or (row_ptr, col, val)); part: int array (0 Omega, 1
    Gamma); labels: optional int array (dimension of each unknown's
    subdomain), which calls mdp_setup_labeled.  Returns the handle (an
    integer address)."""
    if hasattr(A, "indptr"):
        hold = _CsrHold(A.indptr, A.indices, A.data)
    else:
        hold = _CsrHold(*A)
    part = np.ascontiguousarray(part, dtype=np.int32)
    opts = opts if opts is not None else mdp_options_default()
    host_only = bool(opts.flags & MDP_HOST_ONLY)
    sp = None if host_only else _stream_ptr(stream)
    h = _vp()
    if labels is None:
        _check(lib.mdp_setup(C.byref(hold.s), part.ctypes.data_as(_ip), C.byref(opts), sp, C.byref(h)), "mdp_setup")
    else:
        lab = np.ascontiguousarray(labels, dtype=np.int32)
        if lab.shape != part.shape:
            raise ValueError("labels must have one entry per unknown")
        _check(lib.mdp_setup_labeled(C.byref(hold.s), part.ctypes.data_as(_ip), lab.ctypes.data_as(_ip),
                                     C.byref(opts), sp, C.byref(h)), "mdp_setup_labeled")
    return h.value


def mdp_setup_like(src: int, opts: mdp_options, stream=None) -> int:
    """Another handle for src's system with other options (e.g. precision)."""
    sp = None if (opts.flags & MDP_HOST_ONLY) else _stream_ptr(stream)
    h = _vp()
    _check(lib.mdp_setup_like(src, C.byref(opts), sp, C.byref(h)), "mdp_setup_like")
    return h.value


def mdp_destroy(h: int) -> None:
    _check(lib.mdp_destroy(h), "mdp_destroy")


def mdp_solve(h: int, b, x, stream=None, ok=(MDP_OK, MDP_NOT_CONVERGED, MDP_STAGNATED)):
    """b, x: CUDA float64 tensors of shape (n,) or (nrhs, n) (each row one
    right-hand side, contiguous).  Returns (code, [stats dicts])."""
    nrhs = _rhs_pair(h, b, x)
    ld = b.shape[-1]
    st = (mdp_stats * nrhs)()
    rc = lib.mdp_solve(h, _dptr(b), _dptr(x), nrhs, ld, _stream_ptr(stream), st)
    _check(rc, "mdp_solve", ok)
    return rc, [s.as_dict() for s in st]


def mdp_solve_batch(hs: Sequence[int], bs, xs, stream=None, ok=(MDP_OK, MDP_NOT_CONVERGED, MDP_STAGNATED)):
    """hs: handles; bs/xs: per-system CUDA float64 tensors (n,) or (nrhs, n)."""
    ns = len(hs)
    if len(bs) != ns or len(xs) != ns:
        raise ValueError("hs, bs and xs differ in length")
    nrhs = [_rhs_pair(h, b, x) for h, b, x in zip(hs, bs, xs)]
    harr = (_vp * ns)(*hs)
    barr = (_vp * ns)(*[_dptr(b) for b in bs])
    xarr = (_vp * ns)(*[_dptr(x) for x in xs])
    rarr = (C.c_int32 * ns)(*nrhs)
    st = (mdp_stats * max(1, sum(nrhs)))()
    rc = lib.mdp_solve_batch(harr, ns, barr, xarr, rarr, _stream_ptr(stream), st)
    _check(rc, "mdp_solve_batch", ok)
    return rc, [st[i].as_dict() for i in range(sum(nrhs))]


def mdp_apply(h: int, op: int, x, y, stream=None) -> None:
    _check(lib.mdp_apply(h, op, _dptr(x), _dptr(y), _stream_ptr(stream)), "mdp_apply")


def mdp_apply_noalloc(h: int, op: int, x, y, stream=None) -> None:
    """Enqueues only (no synchronisation): y is ready once the stream has run."""
    _check(lib.mdp_apply_noalloc(h, op, _dptr(x), _dptr(y), _stream_ptr(stream)), "mdp_apply_noalloc")


def mdp_info(h: int) -> dict:
    v = [C.c_int32() for _ in range(5)]
    _check(lib.mdp_info(h, *[C.byref(x) for x in v]), "mdp_info")
    return dict(zip(["n", "n_omega", "n_gamma", "levels_omega", "levels_gamma"], [x.value for x in v]))


def mdp_residual_history(h: int) -> np.ndarray:
    """|g_{k+1}| / ||b|| after each iteration of the handle's last one-column solve."""
    n = C.c_int32()
    _check(lib.mdp_residual_history(h, None, 0, C.byref(n)), "mdp_residual_history")
    out = np.zeros(max(n.value, 1), dtype=np.float64)
    _check(lib.mdp_residual_history(h, out.ctypes.data_as(C.POINTER(C.c_double)), n.value, None),
           "mdp_residual_history")
    return out[: n.value]


def mdp_multi_rhs_memory(h: int) -> dict:
    v = [C.c_int64() for _ in range(4)]
    _check(lib.mdp_multi_rhs_memory(h, *[C.byref(x) for x in v]), "mdp_multi_rhs_memory")
    return dict(zip(["plan_bytes", "shared_bytes", "held", "budget"], [x.value for x in v]))


def mdp_level_export(h: int, block: int, level: int, mat: int):
    """Return (row_ptr, col, val, shape) of one hierarchy matrix."""
    r, c, z = C.c_int32(), C.c_int32(), C.c_int64()
    _check(lib.mdp_level_shape(h, block, level, mat, C.byref(r), C.byref(c), C.byref(z)), "mdp_level_shape")
    ptr = np.zeros(r.value + 1, dtype=np.int32)
    col = np.zeros(max(z.value, 1), dtype=np.int32)
    val = np.zeros(max(z.value, 1), dtype=np.float64)
    _check(lib.mdp_level_export(h, block, level, mat, ptr.ctypes.data_as(_ip), col.ctypes.data_as(_ip),
                                val.ctypes.data_as(C.POINTER(C.c_double))), "mdp_level_export")
    return ptr, col[: z.value], val[: z.value], (r.value, c.value)


def mdp_level_aggregates(h: int, block: int, level: int) -> np.ndarray:
    r, c, z = C.c_int32(), C.c_int32(), C.c_int64()
    _check(lib.mdp_level_shape(h, block, level, MDP_MAT_A, C.byref(r), C.byref(c), C.byref(z)), "mdp_level_shape")
    agg = np.zeros(r.value, dtype=np.int32)
    _check(lib.mdp_level_aggregates(h, block, level, agg.ctypes.data_as(_ip)), "mdp_level_aggregates")
    return agg


def mdp_save(h: int, path: str) -> None:
    _check(lib.mdp_save(h, os.fsencode(path)), "mdp_save")


def mdp_load(path: str, opts: Optional[mdp_options] = None, stream=None) -> int:
    """Re-create a handle from a hierarchy file (see mdp_save)."""
    out = _vp()
    host_only = opts is not None and bool(opts.flags & MDP_HOST_ONLY)
    sp = None if host_only else _stream_ptr(stream)
    _check(lib.mdp_load(os.fsencode(path), C.byref(opts) if opts is not None else None, sp, C.byref(out)),
           "mdp_load")
    return out.value


def mdp_server_create(mem_budget_bytes: int = 0, max_slots: int = 64) -> int:
    s = _vp()
    _check(lib.mdp_server_create(mem_budget_bytes, max_slots, C.byref(s)), "mdp_server_create")
    return s.value


def mdp_server_register(srv: int, h: int) -> None:
    _check(lib.mdp_server_register(srv, h), "mdp_server_register")


# (server, ticket) -> (nrhs, b, x): the tensors stay referenced until the
# request has been collected, so their memory cannot be reused meanwhile.
_inflight: dict = {}


def mdp_submit(srv: int, h: int, b, x) -> int:
    """Enqueue a solve; b must be written (stream synchronised) already."""
    nrhs = _rhs_pair(h, b, x)
    t = C.c_uint64()
    _check(lib.mdp_submit(srv, h, _dptr(b), _dptr(x), nrhs, C.byref(t)), "mdp_submit")
    _inflight[(srv, t.value)] = (nrhs, b, x)
    return t.value


def mdp_poll(srv: int, ticket: int):
    """Return (code, stats list or None while pending)."""
    key = (srv, ticket)
    if key not in _inflight:
        raise ValueError(f"mdp_poll: unknown or already collected ticket {ticket}")
    st = (mdp_stats * _inflight[key][0])()
    rc = lib.mdp_poll(srv, ticket, st)
    if rc == MDP_PENDING:
        return rc, None
    del _inflight[key]
    _check(rc, "mdp_poll", ok=(MDP_OK, MDP_NOT_CONVERGED, MDP_STAGNATED))
    return rc, [s.as_dict() for s in st]


def mdp_server_set_grouping(srv: int, on: bool) -> None:
    _check(lib.mdp_server_set_grouping(srv, 1 if on else 0), "mdp_server_set_grouping")


def mdp_server_counts(srv: int) -> dict:
    c, g = C.c_int64(), C.c_int64()
    _check(lib.mdp_server_counts(srv, C.byref(c), C.byref(g)), "mdp_server_counts")
    return {"columns": c.value, "grouped": g.value}


def mdp_server_destroy(srv: int) -> None:
    _check(lib.mdp_server_destroy(srv), "mdp_server_destroy")
    for key in [k for k in _inflight if k[0] == srv]:
        del _inflight[key]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)
# Every C callback pair ever installed stays alive: blocks keep the allocator
# that made them and are freed through it even after another is installed.
_allocators = []


def mdp_set_allocator(alloc=None, free=None) -> None:
    """alloc(nbytes) -> device pointer (int, 0 on failure) and free(ptr):
    Python callables, wrapped as the C callbacks of mdp_set_allocator.  Both
    None restores hipMalloc / hipFree."""
    if (alloc is None) != (free is None):
        raise ValueError("alloc and free must both be given or both be None")
    if alloc is None:
        _check(lib.mdp_set_allocator(None, None, None), "mdp_set_allocator")
        return
    def _alloc(n, ctx):
        try:
            return alloc(n) or None
        except Exception:  # the library reports MDP_ENOMEM for NULL
            return None

    cbs = (ALLOC_FN(_alloc), FREE_FN(lambda p, ctx: free(p)))
    _allocators.append(cbs)
    _check(lib.mdp_set_allocator(C.cast(cbs[0], _vp), C.cast(cbs[1], _vp), None), "mdp_set_allocator")


def mdp_tune_file(path: Optional[str]) -> None:
    _check(lib.mdp_tune_file(path.encode() if path is not None else None), "mdp_tune_file")


def mdp_last_error() -> str:
    return lib.mdp_last_error().decode(errors="replace")


def mdp_version() -> str:
    return lib.mdp_version().decode()
