"""MI355X solver for mixed-dimensional scalar elliptic systems.

Flexible GMRES preconditioned by the inexact block lower-triangular M_L of
Hu, Keilegavlen and Nordbotten (2022), eq. (8) / Algorithm 1, with
smoothed-aggregation AMG V-cycles on the approximate Schur complement of
eq. (7) and on the fracture block, in hand-written HIP for gfx950.

* ``paper_2206_03203_amd._lib``   ctypes binding of include/mdp.h (same names)
* ``paper_2206_03203_amd.solver`` a small object wrapper over the binding
* ``paper_2206_03203_amd.tpfa``   vectorised assembly of synthetic systems
* ``paper_2206_03203_amd.build``  builds libmdp.so for gfx950

The binding raises ImportError when libmdp.so has not been built; there is
no CPU fallback.
"""

__version__ = "0.1.0"
