"""mdp_apply_noalloc, the entry point for callers that cannot allocate device
memory, against mdp_apply: the same operators through the C ABI, on two
systems in a row (the second smaller), in both precisions.  The results
must be identical (the same kernels in the same order), the call must make
no allocation through the library's allocator (counted with an installed
allocator), and the shared scratch array must not carry anything from one
call into the next."""

import ctypes

import numpy as np
import pytest
import torch

import synth
from paper_2206_03203_amd import _lib as L
from paper_2206_03203_amd import tpfa
from paper_2206_03203_amd.solver import Solver

from gpu_common import dev, say

pytestmark = pytest.mark.gpu

OPS = [L.MDP_OP_A, L.MDP_OP_ML, L.MDP_OP_QOO, L.MDP_OP_QGG]


def _len(s, op):
    return {L.MDP_OP_QOO: s.info["n_omega"], L.MDP_OP_QGG: s.info["n_gamma"]}.get(op, s.n)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_noalloc_apply_equals_apply(prec):
    big = synth.regular_3d(n=20, k_par=1e4, kappa=1e-4, seed=2)   # 11600 unknowns
    small = synth.grid_2d_four_lines(32)                         # 1152 unknowns
    solvers = []
    for sc in (big, small):
        A, b, part = tpfa.assemble(sc)
        solvers.append(Solver(A, part, precision=prec, max_coarse=50))
    calls = {"alloc": 0}

    def alloc(n):
        calls["alloc"] += 1
        return torch.cuda.caching_allocator_alloc(n)

    stream = torch.cuda.current_stream()
    try:
        refs = {}
        for k, s in enumerate(solvers):
            for op in OPS:
                x = dev(synth.random_vector(_len(s, op), 50 + 4 * k + op))
                y = torch.empty_like(x)
                L.mdp_apply(s.handle, op, x, y)
                refs[(k, op)] = (x, y)
        torch.cuda.synchronize()
        L.mdp_set_allocator(alloc, lambda p: torch.cuda.caching_allocator_delete(p))
        try:
            for rnd in range(2):  # big then small, twice: nothing carries over
                for k, s in enumerate(solvers):
                    for op in OPS:
                        x, yref = refs[(k, op)]
                        y = torch.full_like(x, np.nan)
                        torch.cuda.synchronize()
                        L.mdp_apply_noalloc(s.handle, op, x, y, stream)
                        torch.cuda.synchronize()
                        say(f"[noalloc] {prec} round {rnd} system {k} op {op} n={x.shape[0]}")
                        assert torch.equal(y, yref), (prec, k, op)
        finally:
            L.mdp_set_allocator(None, None)
        assert calls["alloc"] == 0
    finally:
        for s in solvers:
            s.close()


def test_noalloc_apply_argument_errors():
    sc = synth.grid_2d_four_lines(16)
    A, b, part = tpfa.assemble(sc)
    s = Solver(A, part, precision="mixed")
    try:
        x = dev(np.ones(s.n))
        y = torch.empty_like(x)
        rc = L.lib.mdp_apply_noalloc(s.handle, 7, x.data_ptr(), y.data_ptr(), None)
        assert rc == L.MDP_EINVAL and "unknown operator" in L.mdp_last_error()
        rc = L.lib.mdp_apply_noalloc(s.handle, L.MDP_OP_ML, None, y.data_ptr(), None)
        assert rc == L.MDP_EINVAL
    finally:
        s.close()
