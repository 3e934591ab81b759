"""Host-side sparse layouts and the Arnoldi tile plan (csrc/formats.hpp),
checked on the CPU: a small C++ program rebuilds every eligible layout of
every matrix of a few host systems (set up host-only by the library and
saved with mdp_save) and replays each kernel's index arithmetic: indices in
range, products equal to the CSR product.  It also checks the tile plan:
exact coverage, tile lengths, pairs owning consecutive tiles, and a multiple
of the 256 compute units for long vectors.  Built with the address and
undefined-behaviour sanitizers (host code only)."""

import os
import shutil
import subprocess

import numpy as np
import pytest

import synth
from paper_2206_03203_amd import _lib as L
from paper_2206_03203_amd import tpfa

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2206_03203_amd", "csrc")


def _cases():
    return [
        synth.random_2d(0, n_range=(24, 90), max_segments=8),
        synth.random_2d(3, n_range=(60, 90)),
        synth.regular_3d(n=12, k_par=1e4, kappa=1e-4, seed=4),
        synth.regular_3d(n=20, k_par=1e-4, kappa=1e4, seed=2),
        synth.random_3d(5, n_range=(10, 16)),
        synth.Scenario(2, 20, np.ones(400), [], {(0, 0): 1.0, (0, 1): 0.0}),  # no fractures
        synth.tiny_3d(9, seed=3),
    ]


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_format_layouts_and_tiles(tmp_path):
    exe = tmp_path / "format_check"
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           f"-I{CSRC}", f"-I{os.path.join(ROOT, 'include')}", os.path.join(ROOT, "tests", "cpp", "format_check.cpp"),
           os.path.join(CSRC, "setup.cpp"), os.path.join(CSRC, "serialize.cpp"), "-lpthread", "-o", str(exe)]
    subprocess.run(cmd, check=True, timeout=600)
    files = []
    for i, sc in enumerate(_cases()):
        A, b, part = tpfa.assemble(sc)
        h = L.mdp_setup(A, part, L.mdp_options_default(flags=L.MDP_HOST_ONLY, max_coarse=50))
        try:
            path = str(tmp_path / f"sys{i}.mdph")
            L.mdp_save(h, path)
            files.append(path)
        finally:
            L.mdp_destroy(h)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0")
    run = subprocess.run([str(exe)] + files, capture_output=True, text=True, timeout=600, env=env)
    print(run.stdout)
    assert run.returncode == 0, run.stdout[-4000:] + run.stderr[-4000:]
    assert "failures: 0" in run.stdout
    lines = run.stdout.splitlines()
    # every layout was exercised: the system matrix of the 2D grids in
    # diagonals plus remainder (5 diagonals), the fine S~ of the 3D grids in
    # diagonals, sliced ELL somewhere
    assert any(ln.startswith("A ") and ln.endswith("hyb=5") for ln in lines)
    assert any(ln.startswith("S[0].A") and "dia=7" in ln for ln in lines)
    assert any("sell=1" in ln for ln in lines)
    # some levels restrict with R (I - A D^-1), each checked against R applied
    # to the residual of the first smoothing iterate
    assert any(ln.startswith("fused restrictions: ") and int(ln.split(": ")[1]) > 0 for ln in lines)
    # the fracture rows of the system matrix form its trailing run of rows
    # with remainder entries, dispatched first
    assert any(ln.startswith("A ") and "hyb split=" in ln and
               int(ln.split("split=")[1].split()[0]) < int(ln.split(" of ")[1]) for ln in lines)
