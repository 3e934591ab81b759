"""The block-diagonal and block-upper forms of Section 3.2 (B_D = D^{-1},
B_U = (U D)^{-1}, made inexact with the same Q_OO and Q_GG as M_L) on the
GPU against the oracle's MD and MU: one preconditioner application, and
whole solves (true residual of the oracle's matrix, iterations within 2,
solution within 1e-6 of the oracle's)."""

import numpy as np
import pytest
import torch

import synth
from oracle import amg, precond
from oracle import assembly as oa
from oracle import solve as osv
from paper_2206_03203_amd import _lib as L
from paper_2206_03203_amd import tpfa
from paper_2206_03203_amd.solver import Solver

from gpu_common import dev, host, relerr, say

pytestmark = pytest.mark.gpu

FORMS = {"diag": (L.MDP_BLOCK_DIAG, precond.MD), "upper": (L.MDP_BLOCK_UPPER, precond.MU)}
CASES = {
    "2d-four-lines-32": lambda: synth.grid_2d_four_lines(32),
    "3d-regular-16-Khi-klo": lambda: synth.regular_3d(n=16, k_par=1e4, kappa=1e-4, seed=1),
    "2d-random-s5": lambda: synth.random_2d(5, n_range=(40, 70)),
}
TOL = {"fp64": 1e-11, "mixed": 3e-5}


@pytest.mark.parametrize("form", list(FORMS))
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_block_form_application(form, prec):
    code, cls = FORMS[form]
    sc = synth.regular_3d(n=12, k_par=1e4, kappa=1e4, seed=3)
    A, b, part = tpfa.assemble(sc)
    Ao, bo, po = oa.assemble(sc)
    say(f"[forms] apply form={form} prec={prec}")
    s = Solver(A, part, precision=prec, block_form=code, max_coarse=50)
    M = cls(Ao, po, cycles=1, amg_opts=amg.AMGOptions(max_coarse=50))
    try:
        x = synth.random_vector(A.shape[0], 31)
        z = host(s.apply(L.MDP_OP_ML, dev(x)))
        assert relerr(z, M.apply(x)) <= TOL[prec]
    finally:
        s.close()


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("form", list(FORMS))
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_block_form_solve(name, form, prec):
    code, _ = FORMS[form]
    sc = CASES[name]()
    A, b, part = tpfa.assemble(sc)
    Ao, bo, po = oa.assemble(sc)
    res, _, _ = osv.solve(Ao, bo, po, osv.SolveOptions(form=form))
    say(f"[forms] solve case={name} form={form} prec={prec} oracle iters={res.iters}")
    s = Solver(A, part, precision=prec, block_form=code)
    try:
        x, st = s.solve(dev(b))
        xh = host(x)
        r = np.linalg.norm(bo - Ao @ xh) / np.linalg.norm(bo)
        assert st[0]["converged"] == 1 and r <= 1e-8
        assert abs(st[0]["iters"] - res.iters) <= 2
        assert relerr(xh, res.x) <= 1e-6
    finally:
        s.close()


def test_block_forms_in_one_batch_must_agree():
    sc = synth.grid_2d_four_lines(16)
    A, b, part = tpfa.assemble(sc)
    s1 = Solver(A, part, block_form=L.MDP_BLOCK_LOWER)
    s2 = Solver(A, part, block_form=L.MDP_BLOCK_UPPER)
    try:
        bt = dev(b)
        with pytest.raises(L.MdpError) as e:
            L.mdp_solve_batch([s1.handle, s2.handle], [bt, bt], [torch.zeros_like(bt), torch.zeros_like(bt)])
        assert e.value.code == L.MDP_EINVAL
        s3 = Solver(A, part, block_form=L.MDP_BLOCK_UPPER)
        xs = [torch.zeros_like(bt), torch.zeros_like(bt)]
        rc, st = L.mdp_solve_batch([s2.handle, s3.handle], [bt, bt], xs)
        assert rc == L.MDP_OK and all(q["converged"] == 1 for q in st)
        x1, _ = s2.solve(bt)
        assert relerr(host(xs[0]), host(x1)) <= 1e-6
        s3.close()
    finally:
        s1.close()
        s2.close()
