"""ORACLE -- test infrastructure only.

A plain, slow, CPU reference for what the GPU library computes:

* `direct`: the FP64 direct N-body sum of paper eq. (nbodysum), in plain C
  with OpenMP (direct.c).
* `fmm`: the cubed sphere FMM of paper §3-§8 written step by step in NumPy
  (fmm.py): tree, barycentric Lagrange interpolation, upward pass, dual tree
  traversal, PP/PC/CP/CC interactions, downward pass.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It shares no code with the GPU library and never
imports it.
"""

from .direct import direct, build_oracle, oracle_threads  # noqa: F401
