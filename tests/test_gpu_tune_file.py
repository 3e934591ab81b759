"""The autotuner's choices kept in a file (mdp_tune_file): a setup records
one line per tuned matrix; a later setup that loads the file uses those
formats instead of timing (results bit-identical); a file that forces other
valid formats is obeyed (seen in the algorithmic bytes the kernel timers
count for the finest smoothing sweep, or, between CSR layouts, in the
solution's rounding) and the solve still matches the oracle."""

import numpy as np
import pytest
import torch

import synth
from oracle import assembly as oa
from oracle import solve as osv
from paper_2206_03203_amd import _lib as L
from paper_2206_03203_amd import ktimer, tpfa
from paper_2206_03203_amd.solver import Solver

from gpu_common import dev, host, relerr, say

pytestmark = pytest.mark.gpu


def _fine_smooth_bytes(s, b):
    ktimer.mdp_ktimer_begin(1)
    s.solve(dev(b))
    k = ktimer.mdp_ktimer_end(1)
    return k["bytes"] / max(k["launches"], 1)


def test_tune_file_records_and_replays(tmp_path):
    sc = synth.regular_3d(n=40, k_par=1e4, kappa=1e-4, seed=1)  # fine S~ of 64000 rows: tuned
    A, b, part = tpfa.assemble(sc)
    Ao, bo, po = oa.assemble(sc)
    path = str(tmp_path / "tune.txt")
    L.mdp_tune_file(path)
    try:
        s1 = Solver(A, part, precision="fp64")
        x1, st1 = s1.solve(dev(b))
        lines = [ln.split() for ln in open(path) if ln.strip()]
        say(f"[tune] {len(lines)} recorded choices")
        assert lines and all(len(ln) == 12 for ln in lines)
        bytes_tuned = _fine_smooth_bytes(s1, b)
        s1.close()
        # replay: the same choices, the same results
        L.mdp_tune_file(path)
        s2 = Solver(A, part, precision="fp64")
        x2, st2 = s2.solve(dev(b))
        assert torch.equal(x1, x2) and st1[0]["iters"] == st2[0]["iters"]
        s2.close()
        # force, on every recorded matrix, CSR-vector with a lane count other
        # than the recorded one (4 lanes per row, or 16 where 4 was chosen)
        forced = str(tmp_path / "forced.txt")
        with open(forced, "w") as f:
            for ln in lines:
                was_csr4 = ln[6:10] == ["0", "0", "0", "0"] and ln[10] == "4"
                f.write(" ".join(ln[:6] + ["0", "0", "0", "0", "16" if was_csr4 else "4", "4"]) + "\n")
            f.write("not a choice\n")
        L.mdp_tune_file(forced)
        s3 = Solver(A, part, precision="fp64")
        bytes_forced = _fine_smooth_bytes(s3, b)
        x3, st3 = s3.solve(dev(b))
        s3.close()
        say(f"[tune] fine smoothing bytes per launch: tuned {bytes_tuned:.0f}, forced CSR {bytes_forced:.0f}")
        # the forced formats ran: diagonal storage counts other bytes than
        # CSR; between CSR layouts the lanes' summation order differs, so the
        # solution's last bits do
        assert bytes_forced != bytes_tuned or not torch.equal(x1, x3)
        ref, _, _ = osv.solve(Ao, bo, po, osv.SolveOptions(tol=1e-12))
        x3h = host(x3)
        assert st3[0]["converged"] == 1 and abs(st3[0]["iters"] - st1[0]["iters"]) <= 2
        assert np.linalg.norm(bo - Ao @ x3h) <= 1e-8 * np.linalg.norm(bo) and relerr(x3h, ref.x) <= 1e-6
    finally:
        L.mdp_tune_file(path)  # leave this process with the tuned choices, not the forced ones
        L.mdp_tune_file(None)
