"""The library's vectorised assembly and the oracle's face-by-face assembly
agree on every scenario family (same pattern, values to rounding, same
right-hand side and partition)."""

import numpy as np
import pytest

import synth
from oracle import assembly as oa
from paper_2206_03203_amd import tpfa

CASES = [
    lambda: synth.grid_2d_four_lines(32),
    lambda: synth.grid_2d_four_lines(16, 1e-4, 1.0),
    lambda: synth.tiny_2d(12, seed=4),
    lambda: synth.tiny_3d(7, seed=1),
    lambda: synth.regular_3d(n=12, k_par=1e-4, kappa=1e4, seed=2),
    lambda: synth.random_2d(1, n_range=(20, 40)),
    lambda: synth.random_2d(7, n_range=(20, 40)),
    lambda: synth.random_3d(3, n_range=(8, 12)),
    # degenerate grids: one cell (no interior face), one fracture cell
    lambda: synth.Scenario(2, 1, np.ones(1), [], {(0, 0): 1.0, (0, 1): 0.0}),
    lambda: synth.Scenario(3, 1, np.ones(1), [], {(0, 0): 1.0, (0, 1): 0.0}),
    lambda: synth.Scenario(2, 2, np.ones(4), [synth.Fracture(0, 1, (0,), (1,), 10.0, 0.5, 1e-2)],
                           {(0, 0): 1.0, (0, 1): 0.0}),
]


@pytest.mark.parametrize("make", CASES)
def test_assembly_matches_oracle(make):
    sc = make()
    sc = sc.with_source(synth.host_sources(sc, 5))
    A, b, part = oa.assemble(sc)
    B, c, q = tpfa.assemble(sc)
    assert A.shape == B.shape and A.nnz == B.nnz
    assert np.array_equal(A.indptr, B.indptr) and np.array_equal(A.indices, B.indices)
    assert np.allclose(A.data, B.data, rtol=1e-14, atol=0)
    assert np.allclose(b, c, rtol=1e-14, atol=1e-300)
    assert np.array_equal(part, q)


def test_multiple_sources():
    sc = synth.random_2d(2, n_range=(16, 24))
    fs = [synth.host_sources(sc, k) for k in range(3)] + [None]
    B, C, q = tpfa.assemble(sc, sources=fs)
    for k, f in enumerate(fs):
        A, b, _ = oa.assemble(sc.with_source(f))
        assert np.allclose(C[:, k], b, rtol=1e-14, atol=1e-300)


@pytest.mark.parametrize("make", [
    lambda: synth.grid_2d_four_lines(16),
    lambda: synth.tiny_2d(8, seed=2),
    lambda: synth.random_2d(5, n_range=(30, 50)),
    lambda: synth.random_2d(11, n_range=(30, 50)),
    lambda: synth.tiny_3d(6, seed=1),
    lambda: synth.regular_3d(n=9, seed=4),
    lambda: synth.random_3d(2, n_range=(10, 14)),
])
def test_flux_assembly_matches_oracle(make):
    """The library's vectorised assembly of the interface-flux system and the
    oracle's loop-based one: same unknown order, same pattern, values to
    1e-15 relative, same right-hand side and partition."""
    from oracle import mixed_dim as md
    from paper_2206_03203_amd import tpfa_flux
    sc = make()
    fs = synth.host_sources(sc, 3)
    A, b, part, info = tpfa_flux.assemble_flux(sc.with_source(fs))
    Ao, bo, po, io = md.assemble_flux(sc.with_source(fs))
    for k in ("host", "fracture", "intersection", "point", "interface", "cells"):
        assert info[k] == io[k], k
    assert np.array_equal(part, po)
    assert A.shape == Ao.shape and np.array_equal(A.indptr, Ao.indptr) and np.array_equal(A.indices, Ao.indices)
    assert np.allclose(A.data, Ao.data, rtol=1e-15, atol=0)
    assert np.allclose(b, bo, rtol=1e-15, atol=1e-300)
