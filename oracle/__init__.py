"""Plain FP64 CPU oracle — TEST INFRASTRUCTURE ONLY.

This package is the slow, obviously-correct reference that the GPU library
is checked against.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import it; the library never does, and it
imports nothing from the library.

Contents, each following the paper (Hu, Keilegavlen, Nordbotten 2022,
"Effective Preconditioners for Mixed-Dimensional Scalar Elliptic Problems"):

* ``assembly``  two-point-flux discretisation of the mixed-dimensional model
                (Section 2.1, eqs. (1)-(3)) on Cartesian grids, producing the
                2x2 host/fracture block system of eq. (4).
* ``blocks``    block split (eq. 4), exact Schur complement (eq. 6) and the
                diagonal-fracture-block approximation (eq. 7).
* ``amg``       smoothed-aggregation AMG setup and the V-cycle that defines
                Q_OmegaOmega and Q_GammaGamma (Section 3.3).
* ``precond``   the preconditioner M_L (eq. 8) applied as in Algorithm 1, and
                the exact block preconditioners of Section 3.2 for checks.
* ``fgmres``    right-preconditioned flexible GMRES (Section 3.2 uses right
                preconditioning; Section 4 fixes zero initial guess and a
                relative-residual stopping rule).
* ``solve``     the whole solve phase glued together.

Parity status is stated per function in each module header.
"""

from . import assembly, blocks, amg, precond, fgmres, solve  # noqa: F401
