"""A handle re-created from a hierarchy file (mdp_save / mdp_load) solves
exactly as the handle it was saved from, in either precision."""

import pytest
import torch

import synth
from paper_2206_03203_amd import _lib as L
from paper_2206_03203_amd import tpfa
from paper_2206_03203_amd.solver import Solver

from gpu_common import dev, say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_loaded_handle_solves_identically(tmp_path, prec):
    sc = synth.regular_3d(n=20, k_par=1e4, kappa=1e-4, seed=5)
    A, b, part = tpfa.assemble(sc)
    s = Solver(A, part, precision=prec)
    path = str(tmp_path / "h.mdph")
    say(f"[hierfile] prec={prec}")
    try:
        L.mdp_save(s.handle, path)
        h2 = L.mdp_load(path, L.mdp_options_default(precision=s.options.precision))
        try:
            bt = dev(b)
            x1, st1 = s.solve(bt)
            x2 = torch.zeros_like(bt)
            rc, st2 = L.mdp_solve(h2, bt, x2)
            assert rc == L.MDP_OK and st1[0]["iters"] == st2[0]["iters"]
            assert torch.equal(x1, x2)
        finally:
            L.mdp_destroy(h2)
    finally:
        s.close()
