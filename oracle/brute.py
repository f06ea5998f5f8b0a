"""Brute-force reference for tiny spaces -- TEST INFRASTRUCTURE ONLY.

Evaluates the constraint *strings* with Python's own eval over
itertools.product (the Cartesian space of Section IV-A, last parameter
fastest) and takes argmins by sorting complete key lists.  It shares nothing
with the C oracle beyond the inputs, so it pins the oracle's expression
walker, enumeration order and repair scans on spaces small enough to list.
"""
from __future__ import annotations

import itertools
from typing import Dict, List, Sequence, Tuple


def is_valid(constraints: Sequence[str], env: Dict[str, int]) -> bool:
    for c in constraints:
        try:
            if not eval(c, {"__builtins__": {}, "min": min, "max": max, "abs": abs}, dict(env)):
                return False
        except ZeroDivisionError:
            return False
    return True


def enumerate_space(names: Sequence[str], values: Sequence[Sequence[int]],
                    constraints: Sequence[str]) -> Tuple[List[int], List[Tuple[int, ...]]]:
    """Valid linear indices (ascending) and their value-index rows."""
    lin, rows = [], []
    for L, idx in enumerate(itertools.product(*[range(len(v)) for v in values])):
        env = {n: values[j][k] for j, (n, k) in enumerate(zip(names, idx))}
        if is_valid(constraints, env):
            lin.append(L)
            rows.append(idx)
    return lin, rows
