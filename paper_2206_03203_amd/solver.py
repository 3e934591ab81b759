"""Object wrapper over the C ABI binding (argument marshalling only)."""

from __future__ import annotations

from typing import Optional

import numpy as np

from . import _lib as L


class Solver:
    """One system A (eq. (4)) set up for repeated solves on the GPU.

    ``precision`` is "fp64" or "mixed" (FP32 preconditioner, FP64 outer).
    Extra keyword arguments set fields of mdp_options."""

    def __init__(self, A, part, precision: str = "fp64", stream=None, labels=None, **opts):
        prec = {"fp64": L.MDP_FP64, "mixed": L.MDP_MIXED}[precision]
        self.options = L.mdp_options_default(precision=prec, **opts)
        self.handle = L.mdp_setup(A, part, self.options, stream, labels=labels)
        self.info = L.mdp_info(self.handle)
        self.n = self.info["n"]
        self.precision = precision

    def solve(self, b, x=None, stream=None):
        """b: CUDA float64 tensor (n,) or (nrhs, n).  Returns (x, stats list).
        With four or more right-hand sides, mdp_solve takes them four at a time
        with shared matrix reads while its memory budget allows."""
        import torch
        if x is None:
            x = torch.zeros_like(b)
        rc, st = L.mdp_solve(self.handle, b, x, stream)
        return x, st

    def apply(self, op: int, x, y=None, stream=None):
        import torch
        if y is None:
            y = torch.empty_like(x)
        L.mdp_apply(self.handle, op, x, y, stream)
        return y

    def close(self):
        if self.handle:
            L.mdp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def use_torch_allocator(on: bool = True) -> None:
    """Route the library's device allocations made from now on through
    PyTorch's caching allocator (on the calling thread's current stream), or
    back to hipMalloc.  Memory already held keeps the allocator that made it."""
    import torch
    if on:
        L.mdp_set_allocator(lambda n: torch.cuda.caching_allocator_alloc(n),
                            lambda p: torch.cuda.caching_allocator_delete(p))
    else:
        L.mdp_set_allocator(None, None)
