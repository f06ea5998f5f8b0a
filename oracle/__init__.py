"""CPU oracle for constraint-aware evolutionary auto-tuning -- TEST INFRASTRUCTURE ONLY.

A plain, slow, obviously-correct implementation of what the GPU path
computes, written from the paper (Section IV and Alg. 1-3).  Only tests/,
__graft_entry__.smoke() and bench.py's cpu_baseline leg may import it; the
GPU library never does and shares no code with it.

Modules:
  expr   - constraint strings -> the oracle's own expression trees
  core   - search space, enumeration, validity, repair scans, Philox (C core in ct_oracle.c)
  steps  - DE / PSO / GA generation steps
  brute  - Python-eval brute force for tiny spaces (pins the C core)
"""
from . import core, expr, steps, brute  # noqa: F401
