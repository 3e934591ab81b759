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


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_version_1_file_restricts_residuals_to_the_same_result(tmp_path, prec):
    """A first-version file has no fused restrictions, so its V-cycles form
    each residual and restrict it; the operator is the same as with the fused
    restriction R (I - A D^-1), so one V-cycle agrees to rounding and the
    solves agree within the solver tolerance."""
    from hierfile_util import to_version_1

    sc = synth.regular_3d(n=20, k_par=1e4, kappa=1e-4, seed=5)
    A, b, part = tpfa.assemble(sc)
    s = Solver(A, part, precision=prec)
    path = tmp_path / "h.mdph"
    say(f"[hierfile] version 1 prec={prec}")
    try:
        L.mdp_save(s.handle, str(path))
        old = tmp_path / "h1.mdph"
        old.write_bytes(to_version_1(path.read_bytes()))
        h1 = L.mdp_load(str(old), L.mdp_options_default(precision=s.options.precision))
        try:
            n_o = s.info["n_omega"]
            r = dev(synth.random_vector(n_o, 17))
            q2 = torch.zeros_like(r)
            q1 = torch.zeros_like(r)
            L.mdp_apply(s.handle, L.MDP_OP_QOO, r, q2)
            L.mdp_apply(h1, L.MDP_OP_QOO, r, q1)
            torch.cuda.synchronize()
            rel = float(torch.linalg.norm(q1 - q2) / torch.linalg.norm(q2))
            say(f"  one V-cycle on S~: relative difference {rel:.2e}")
            assert rel <= (1e-11 if prec == "fp64" else 3e-5)  # the bar of the V-cycle parity tests
            bt = dev(b)
            x2, st2 = s.solve(bt)
            x1 = torch.zeros_like(bt)
            rc, st1 = L.mdp_solve(h1, bt, x1)
            assert rc == L.MDP_OK and abs(st1[0]["iters"] - st2[0]["iters"]) <= 1
            assert float(torch.linalg.norm(x1 - x2) / torch.linalg.norm(x2)) <= 1e-6
        finally:
            L.mdp_destroy(h1)
    finally:
        s.close()
