"""Arnoldi steps replayed from captured HIP graphs (MDP_GRAPHS) give exactly
the results of direct launches: several solves in a row on the same
handle, with other device work in between, on torch's default (legacy)
stream and on a side stream; restarts whose last cycle is shorter than the
restart length (the last-step graph variant); two V-cycles on a system whose
finest level is solved densely (the zero-fill inside a captured step)."""

import numpy as np
import pytest
import torch

import synth
from paper_2206_03203_amd import _lib as L
from paper_2206_03203_amd import tpfa

from gpu_common import dev, say

pytestmark = pytest.mark.gpu


def _pair(A, part, **kw):
    o1 = L.mdp_options_default(**kw)
    o1.flags |= L.MDP_GRAPHS
    h1 = L.mdp_setup(A, part, o1)
    o2 = L.mdp_options_default(**kw)
    h2 = L.mdp_setup_like(h1, o2)
    return h1, h2


CASES = [
    ("3d-regular-16", lambda: synth.regular_3d(n=16, k_par=1e4, kappa=1e-4, seed=2), {}),
    ("2d-four-lines-48", lambda: synth.grid_2d_four_lines(48), {}),
    ("restart-8-max-21", lambda: synth.regular_3d(n=12, k_par=1e4, kappa=1e4, seed=1), dict(restart=8, max_iter=21)),
    ("dense-finest-2-cycles", lambda: synth.tiny_2d(8, seed=3), dict(vcycles=2)),
]


@pytest.mark.parametrize("name,make,kw", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("prec", [L.MDP_FP64, L.MDP_MIXED])
def test_graph_replay_equals_direct_launches(name, make, kw, prec):
    sc = make()
    srcs = [None] + [synth.host_sources(sc, 40 + k) for k in range(3)]
    A, B, part = tpfa.assemble(sc, sources=srcs)
    h1, h2 = _pair(A, part, precision=prec, **kw)
    say(f"[graphs] case={name} prec={prec}")
    side = torch.cuda.Stream()
    try:
        for rep in range(2):
            for k in range(B.shape[1]):
                b = dev(B[:, k].copy())
                x1, x2 = torch.zeros_like(b), torch.zeros_like(b)
                stream = side if (k + rep) % 2 else None
                if stream is not None:
                    stream.wait_stream(torch.cuda.current_stream())
                rc1, st1 = L.mdp_solve(h1, b, x1, stream)
                junk = torch.randn(1 << 16, device="cuda:0").sum()  # other work between replays
                rc2, st2 = L.mdp_solve(h2, b, x2, stream)
                torch.cuda.synchronize()
                assert float(junk) == float(junk)
                assert rc1 == rc2 and st1[0]["iters"] == st2[0]["iters"], (k, st1, st2)
                assert torch.equal(x1, x2), f"rhs {k} rep {rep}: graph replay differs"
                if "max" not in name:
                    assert st1[0]["converged"] == 1
    finally:
        L.mdp_destroy(h1)
        L.mdp_destroy(h2)


def _batch_handles(scs, graphs, prec):
    hs = []
    for sc in scs:
        A, b, part = tpfa.assemble(sc)
        o = L.mdp_options_default(precision=prec)
        if graphs:
            o.flags |= L.MDP_GRAPHS
        hs.append(L.mdp_setup(A, part, o))
    return hs


@pytest.mark.parametrize("rhs", [1, 4])
@pytest.mark.parametrize("chunked", [False, True])
@pytest.mark.parametrize("prec", [L.MDP_FP64, L.MDP_MIXED])
def test_batch_graph_replay_equals_direct_launches(rhs, chunked, prec, monkeypatch):
    """mdp_solve_batch with MDP_GRAPHS: uneven systems, one or four
    right-hand sides each (the one-block and the shared-matrix layouts),
    optionally cut into chunks that share one workspace (each chunk keeps
    its own graphs); two rounds on the legacy and on a side stream with other
    work in between; every result bit-identical to the batch without
    graphs."""
    if chunked:
        monkeypatch.setenv("MDP_BATCH_MAX_UNKNOWNS", "30000")
    scs = [synth.random_2d(s, n_range=(40, 100), max_segments=6) for s in range(5)]
    scs.append(synth.regular_3d(n=14, k_par=1e4, kappa=1e-4, seed=3))
    hg = _batch_handles(scs, True, prec)
    hd = _batch_handles(scs, False, prec)
    bs = []
    for i, sc in enumerate(scs):
        fs = [None] + [synth.host_sources(sc, 60 + 4 * i + k) for k in range(rhs - 1)]
        _, B, _ = tpfa.assemble(sc, sources=fs)
        bs.append(dev(np.ascontiguousarray(B.T)) if rhs > 1 else dev(B[:, 0].copy()))
    say(f"[graphs] batch rhs={rhs} chunked={chunked} prec={prec}")
    side = torch.cuda.Stream()
    try:
        for rep in range(2):
            stream = side if rep else None
            if stream is not None:
                stream.wait_stream(torch.cuda.current_stream())
            xg = [torch.zeros_like(b) for b in bs]
            xd = [torch.zeros_like(b) for b in bs]
            rcg, stg = L.mdp_solve_batch(hg, bs, xg, stream)
            junk = torch.randn(1 << 16, device="cuda:0").sum()
            rcd, std = L.mdp_solve_batch(hd, bs, xd, stream)
            torch.cuda.synchronize()
            assert float(junk) == float(junk)
            assert rcg == rcd == L.MDP_OK
            assert [s["iters"] for s in stg] == [s["iters"] for s in std]
            for a, b in zip(xg, xd):
                assert torch.equal(a, b), f"rep {rep}: batch graph replay differs"
    finally:
        for h in hg + hd:
            L.mdp_destroy(h)
