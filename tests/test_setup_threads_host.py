"""The multithreaded host setup under ThreadSanitizer (CPU): a small C++
program (tests/cpp/setup_threads.cpp) reruns the whole setup of a few saved
host systems, large enough for the worker threads to split the loops, with
four workers, and requires bit-identical results to the library's setup with
its default worker count; ThreadSanitizer fails the run on any data race."""

import os
import shutil
import subprocess

import pytest

import synth
from paper_2206_03203_amd import _lib as L
from paper_2206_03203_amd import tpfa, tpfa_flux

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2206_03203_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_setup_has_no_data_race_and_ignores_the_thread_count(tmp_path):
    exe = tmp_path / "setup_threads"
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=thread", f"-I{CSRC}", f"-I{os.path.join(ROOT, 'include')}",
           os.path.join(ROOT, "tests", "cpp", "setup_threads.cpp"), os.path.join(CSRC, "setup.cpp"),
           os.path.join(CSRC, "serialize.cpp"), "-lpthread", "-o", str(exe)]
    subprocess.run(cmd, check=True, timeout=600)
    files = []
    cases = [("pressure", synth.regular_3d(n=24, k_par=1e4, kappa=1e-4, seed=2)),
             ("pressure", synth.random_2d(7, n_range=(120, 130))),
             ("flux", synth.regular_3d(n=20, k_par=1e-4, kappa=1e4, seed=3))]
    for i, (form, sc) in enumerate(cases):
        if form == "flux":
            A, b, part, _ = tpfa_flux.assemble_flux(sc)
        else:
            A, b, part = tpfa.assemble(sc)
        assert A.shape[0] >= 8192  # the loops split only from 8192 rows on
        h = L.mdp_setup(A, part, L.mdp_options_default(flags=L.MDP_HOST_ONLY))
        try:
            path = str(tmp_path / f"sys{i}.mdph")
            L.mdp_save(h, path)
            files.append(path)
        finally:
            L.mdp_destroy(h)
    env = dict(os.environ, MDP_SETUP_THREADS="4", TSAN_OPTIONS="halt_on_error=1 exitcode=66")
    run = subprocess.run([str(exe)] + files, capture_output=True, text=True, timeout=900, env=env)
    print(run.stdout)
    assert run.returncode == 0, run.stdout[-4000:] + run.stderr[-6000:]
    assert "failures: 0" in run.stdout
    assert "ThreadSanitizer" not in run.stderr
