"""Kernel-class timers of the library (mdp_ktimer_begin / mdp_ktimer_end):
HIP events around every launch of a class on its launch stream, with the
algorithmic bytes of each launch."""

from __future__ import annotations

import ctypes as C

from . import _lib as L

CLASSES = {0: "outer_spmv", 1: "fine_smooth", 2: "vcycle_other", 3: "arnoldi_dot",
           4: "arnoldi_axpy", 5: "other", 6: "fine_resid"}
# classes whose launches are all of one kernel symbol (per precision)
SINGLE_KERNEL = {"outer_spmv": "system-matrix product (format chosen at setup)",
                 "fine_smooth": "post-smoothing sweep on the finest S~ level",
                 "fine_resid": "residual after the first sweep on the finest S~ level, or, where the level "
                               "restricts with R (I - A D^-1), that one restriction product",
                 "arnoldi_dot": "dcgs_reduce_kernel", "arnoldi_axpy": "dcgs_update_kernel"}


def mdp_ktimer_begin(kind: int) -> None:
    L._check(L.lib.mdp_ktimer_begin(kind), "mdp_ktimer_begin")


def mdp_ktimer_end(kind: int) -> dict:
    ms, n, b = C.c_double(), C.c_int64(), C.c_double()
    L._check(L.lib.mdp_ktimer_end(kind, C.byref(ms), C.byref(n), C.byref(b)), "mdp_ktimer_end")
    return {"ms": ms.value, "launches": n.value, "bytes": b.value}


def begin_all(names=None) -> None:
    for k, name in CLASSES.items():
        if names is None or name in names:
            mdp_ktimer_begin(k)


def end_all(names=None) -> dict:
    return {name: mdp_ktimer_end(k) for k, name in CLASSES.items() if names is None or name in names}
