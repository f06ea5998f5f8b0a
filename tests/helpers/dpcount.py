"""Exact valid-set size of a many-problem space by dynamic programming (no enumeration).

The many-problem spaces have parameters p_j with values 1..r_j and two
constraints: sum_j w_j * p_j <= T and (p0 * p1) % 3 != 0.  The second one only
involves p0 and p1, so the count is the sum over the admissible (p0, p1) pairs
of the number of (p2, ..., p_{D-1}) whose weighted sum fits in what is left of
T.  That number comes from the distribution of the weighted sum, built one
parameter at a time by convolution (a count per attainable sum).
"""
import re

import numpy as np


def parse(spec):
    """(weights, T) from the linear constraint text, checking the second constraint's form."""
    lin, mod = spec.constraints
    assert mod.replace(" ", "") == "(p0*p1)%3!=0"
    lhs, T = lin.split("<=")
    terms = [t.strip() for t in lhs.split("+")]
    w = []
    for j, t in enumerate(terms):
        m = re.fullmatch(r"(\d+)\*p(\d+)", t)
        assert m and int(m.group(2)) == j
        w.append(int(m.group(1)))
    return w, int(T)


def count(spec) -> int:
    w, T = parse(spec)
    r = spec.radices
    if T < 0:
        return 0
    # dist[s] = number of (p2..p_{D-1}) with weighted sum s (s <= T; larger sums never fit)
    dist = np.zeros(T + 1, dtype=np.int64)
    dist[0] = 1
    for j in range(2, len(r)):
        nxt = np.zeros(T + 1, dtype=np.int64)
        for v in range(1, r[j] + 1):
            sh = w[j] * v
            if sh <= T:
                nxt[sh:] += dist[: T + 1 - sh]
        dist = nxt
    cum = np.cumsum(dist)                  # cum[s] = number with sum <= s
    total = 0
    for a in range(1, r[0] + 1):
        for b in range(1, r[1] + 1):
            if (a * b) % 3 != 0:
                rest = T - w[0] * a - w[1] * b
                if rest >= 0:
                    total += int(cum[rest])
    return total
