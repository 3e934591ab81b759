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
