"""The V-cycle's dense tail (CPU): the matrix that the library forms at
upload for the part of a V-cycle from a level l* down (csrc/setup.cpp,
form_tail) equals the oracle's V-cycle started at level l* of its own
hierarchy (oracle/amg.py, Section 3.3), column against column, for one and
for two smoothing sweeps; the tail starts at the first level below the
finest with at most the size bound, above the coarsest.  The harness is
built with the address and undefined-behaviour sanitizers."""

import os
import shutil
import subprocess

import numpy as np
import pytest

import synth
from oracle import amg, precond
from oracle import assembly as oa
from paper_2206_03203_amd import _lib as L
from paper_2206_03203_amd import tpfa

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2206_03203_amd", "csrc")
MAX_N = 2000


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("needs g++")
    exe = tmp_path_factory.mktemp("tail") / "tail_check"
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           f"-I{CSRC}", f"-I{os.path.join(ROOT, 'include')}", os.path.join(ROOT, "tests", "cpp", "tail_check.cpp"),
           os.path.join(CSRC, "setup.cpp"), os.path.join(CSRC, "serialize.cpp"), "-lpthread", "-o", str(exe)]
    subprocess.run(cmd, check=True, timeout=600)
    return exe


def _read(path):
    raw = open(path, "rb").read()
    out, pos = [], 0
    while pos < len(raw):
        lvl, n = np.frombuffer(raw, dtype=np.int32, count=2, offset=pos)
        pos += 8
        T = None
        if lvl >= 0:
            T = np.frombuffer(raw, dtype=np.float64, count=int(n) * int(n), offset=pos).reshape(n, n)
            pos += 8 * int(n) * int(n)
        out.append((int(lvl), T))
    return out


CASES = {
    # both hierarchies have three levels, the middle one small enough
    "cube 24": (lambda: synth.regular_3d(n=24, k_par=1e4, kappa=1e-4, seed=2), 2),
    # two-level hierarchies: the level below the finest is the coarsest, no tail
    "2D 32x32": (lambda: synth.grid_2d_four_lines(32), 0),
    # a bigger cube: the Omega tail sits deeper than level 1
    "cube 40": (lambda: synth.regular_3d(n=40, k_par=1e-4, kappa=1e-4, seed=1), None),
}


@pytest.mark.parametrize("sweeps", [1, 2])
@pytest.mark.parametrize("case", list(CASES))
def test_tail_matches_the_oracle_vcycle_from_its_level(harness, tmp_path, sweeps, case):
    make, n_tails = CASES[case]
    sc = make()
    A, b, part = tpfa.assemble(sc)
    h = L.mdp_setup(A, part, L.mdp_options_default(flags=L.MDP_HOST_ONLY, pre_sweeps=sweeps, post_sweeps=sweeps))
    try:
        path = str(tmp_path / "sys.mdph")
        L.mdp_save(h, path)
    finally:
        L.mdp_destroy(h)
    out = str(tmp_path / "tails.bin")
    run = subprocess.run([str(harness), str(sweeps), str(sweeps), str(MAX_N), out, path], capture_output=True,
                         text=True, timeout=600)
    print(run.stdout)
    assert run.returncode == 0, run.stdout[-3000:] + run.stderr[-6000:]
    tails = _read(out)
    assert len(tails) == 2
    Ao, bo, po = oa.assemble(sc)
    M = precond.ML(Ao, po, 1, amg.AMGOptions(pre_sweeps=sweeps, post_sweeps=sweeps))
    rng = np.random.default_rng(11)
    checked = 0
    for (lvl, T), H in zip(tails, (M.H_omega, M.H_gamma)):
        sizes = [lv.A.shape[0] for lv in H.levels]
        expect = next((l for l in range(1, len(sizes) - 1) if sizes[l] <= MAX_N), -1)
        if H.coarse_dense is None:
            expect = -1
        assert lvl == expect, (sizes, lvl)
        if lvl < 0:
            continue
        n = sizes[lvl]
        assert T.shape == (n, n)
        # unit columns and random vectors through the oracle's V-cycle from level lvl
        for j in list(range(0, n, max(1, n // 7))) + [n - 1]:
            e = np.zeros(n)
            e[j] = 1.0
            ref = amg.vcycle(H, e, lvl)
            assert np.linalg.norm(T[:, j] - ref) <= 1e-11 * np.linalg.norm(ref), j
        for _ in range(3):
            v = rng.standard_normal(n)
            ref = amg.vcycle(H, v, lvl)
            assert np.linalg.norm(T @ v - ref) <= 1e-11 * np.linalg.norm(ref)
        checked += 1
    if n_tails is not None:
        assert checked == n_tails
    else:
        assert checked >= 1
