"""Device memory from the caller's allocator (mdp_set_allocator): every
allocation of a handle (hierarchy, Krylov workspace, four-column plan) comes
from PyTorch's caching allocator while it is installed, is returned to it on
mdp_destroy, and the solves are bit-identical to those of a handle whose
memory came from hipMalloc."""

import numpy as np
import pytest
import torch

import synth
from oracle import assembly as oa
from paper_2206_03203_amd import _lib as L
from paper_2206_03203_amd import tpfa
from paper_2206_03203_amd.solver import Solver, use_torch_allocator

from gpu_common import dev, host, say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_torch_caching_allocator_serves_every_allocation(prec):
    sc = synth.regular_3d(n=16, seed=7)
    A, b, part = tpfa.assemble(sc)
    Ao, bo, _ = oa.assemble(sc)
    fs = [None] + [synth.host_sources(sc, 40 + k) for k in range(3)]
    _, B, _ = tpfa.assemble(sc, sources=fs)
    B4 = dev(np.ascontiguousarray(B.T))
    say(f"[allocator] {prec} n={A.shape[0]}")
    ref = Solver(A, part, precision=prec)
    x_ref, st_ref = ref.solve(dev(b))
    X_ref, _ = ref.solve(B4)
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    use_torch_allocator(True)
    try:
        s = Solver(A, part, precision=prec)
        x, st = s.solve(dev(b))
        X, _ = s.solve(B4)  # builds the four-column plan through the hook too
        torch.cuda.synchronize()
        held = torch.cuda.memory_allocated() - before
        # the hierarchy, the workspace and the four-column plan are torch's now
        # (x, X and b's copies above are a few hundred KB)
        assert held > 20 * A.shape[0] * 8, held
        assert torch.equal(x, x_ref) and torch.equal(X, X_ref)
        assert st[0]["iters"] == st_ref[0]["iters"] and st[0]["converged"] == 1
        assert np.linalg.norm(bo - Ao @ host(x)) <= 1e-8 * np.linalg.norm(bo)
        del x, X
        s.close()
        torch.cuda.synchronize()
        assert torch.cuda.memory_allocated() - before <= 0
    finally:
        use_torch_allocator(False)
        ref.close()
