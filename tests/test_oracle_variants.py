"""Pins of the oracle's operator variants (Section IV-B last paragraph, Section IV-D) -- CPU only.

DE: at CR = 1 every trial is clip(round_half_up(base + F * difference)) for some distinct
members, with base and difference as each operator defines them (rand1, best1, rand2, best2,
current-to-best, rand-to-best), the rounding computed here from exact rationals; exponential
crossover takes one coordinate at CR = 0, all at CR = 1, and in between a circular run from
j_rand whose length follows P(L >= k) = CR^(k-1).  GA: two-point children are A[:c1] +
B[c1:c2] + A[c2:] and its mirror for two cuts; uniform children are complementary with half
of the genes from each parent; disruptive-uniform children swap exactly half (rounded down)
of the genes where the parents differ.
"""
import functools
import itertools
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import core, steps


def free_space(radices):
    names = [f"p{j}" for j in range(len(radices))]
    return core.Space(names, [list(range(r)) for r in radices], []).enumerate()


def rnd_half_up(x: Fraction) -> int:
    return math.floor(x + Fraction(1, 2))


def expected(method, xi, best, pick, F, j):
    x = lambda r: int(pick[r][j])  # noqa: E731
    b = int(best[j])
    if method == steps.DE_RAND1:
        base, diff = x(0), x(1) - x(2)
    elif method == steps.DE_BEST1:
        base, diff = b, x(1) - x(2)
    elif method == steps.DE_RAND2:
        base, diff = x(0), x(1) - x(2) + x(3) - x(4)
    elif method == steps.DE_BEST2:
        base, diff = b, x(1) - x(2) + x(3) - x(4)
    elif method == steps.DE_CURRENTTOBEST1:
        base, diff = int(xi[j]), b - int(xi[j]) + x(1) - x(2)
    else:
        base, diff = x(0), b - x(0) + x(1) - x(2)
    return base + F * diff


@pytest.mark.parametrize("method", [steps.DE_RAND1, steps.DE_BEST1, steps.DE_RAND2, steps.DE_BEST2,
                                    steps.DE_CURRENTTOBEST1, steps.DE_RANDTOBEST1])
def test_de_operator_trials_are_their_defined_mutants(method):
    sp = free_space([9, 9, 9])
    rng = np.random.default_rng(int(method))
    P = 7
    pos = rng.choice(sp.n_valid, P, replace=False)
    st = steps.DEState(pos, np.arange(P, dtype=np.float32), np.float32(0), int(pos[0]), gen=4)
    F_q16 = 32768
    F = Fraction(F_q16, 65536)
    trials = steps.de_trials(sp, st, 11, F_q16, 1 << 32, method)
    X = sp.vrows[pos]
    best = sp.vrows[pos[0]]
    k = 5 if method in (steps.DE_RAND2, steps.DE_BEST2) else 3
    for i in range(P):
        others = [r for r in range(P) if r != i]
        ok = False
        for combo in itertools.permutations(others, k):
            pick = [X[r] for r in combo]
            want = [min(max(rnd_half_up(expected(method, X[i], best, pick, F, j)), 0), 8) for j in range(3)]
            if list(trials[i]) == want:
                ok = True
                break
        assert ok, f"operator {method}: member {i}'s trial {trials[i]} is no mutant of its definition"


@functools.lru_cache(maxsize=None)
def exp_setup(P=12, D=6):
    sp = free_space([P] * D)
    # member i is (i, i, ..., i); best is member 0, so every coordinate of a best1 mutant with
    # F = 0 (the best row) differs from member i > 0
    pos = np.array([sp.pos(sp.encode(np.full((1, D), i, dtype=np.int32)))[0] for i in range(P)])
    st = steps.DEState(pos, np.arange(P, dtype=np.float32), np.float32(0), int(pos[0]), gen=2)
    return sp, st


def mutant_runs(CR_q32, seed=5):
    sp, st = exp_setup()
    tr = steps.de_trials(sp, st, seed, 0, CR_q32, steps.DE_BEST1, steps.DE_EXP)
    X = sp.vrows[st.pos]
    return [(tr[i] != X[i]) for i in range(1, len(st.pos))]


def test_exponential_crossover_extremes():
    for taken in mutant_runs(0):
        assert taken.sum() == 1                   # j_rand only
    for taken in mutant_runs(1 << 32):
        assert taken.all()


def test_exponential_crossover_is_a_circular_run_of_geometric_length():
    CR = 0.6
    lengths = []
    for seed in range(60):
        for taken in mutant_runs(round(CR * 2 ** 32), seed):
            D = len(taken)
            L = int(taken.sum())
            # the taken coordinates form one circular interval
            starts = [j for j in range(D) if taken[j] and not taken[j - 1]]
            assert L == D or len(starts) == 1
            lengths.append(L)
    D = 6
    mean = np.mean(lengths)
    want = sum(CR ** (k - 1) for k in range(1, D + 1))
    var = sum((2 * k - 1) * CR ** (k - 1) for k in range(1, D + 1)) - want ** 2
    assert abs(mean - want) <= 4 * math.sqrt(var / len(lengths)), (mean, want)


def test_two_point_children():
    rng = np.random.default_rng(3)
    D = 9
    two_cuts_seen = 0
    for k in range(300):
        A, B = rng.integers(0, 50, D), rng.integers(50, 100, D)        # differ everywhere
        o = steps.draw(7, k, 3, steps.P_GA_SEL)
        c1, c2 = steps.ga_cross_pair(A, B, 7, k, 3, o, steps.GA_TWO_POINT)
        cuts = [(a, b) for a in range(1, D) for b in range(a + 1, D)
                if np.array_equal(c1, np.concatenate([A[:a], B[a:b], A[b:]]))
                and np.array_equal(c2, np.concatenate([B[:a], A[a:b], B[b:]]))]
        assert len(cuts) == 1
        two_cuts_seen += 1
    assert two_cuts_seen == 300
    # D < 3: a single cut
    A, B = np.array([1, 2]), np.array([3, 4])
    c1, c2 = steps.ga_cross_pair(A, B, 7, 0, 0, steps.draw(7, 0, 0, steps.P_GA_SEL), steps.GA_TWO_POINT)
    assert list(c1) == [1, 4] and list(c2) == [3, 2]


def test_uniform_children_are_complementary_halves():
    rng = np.random.default_rng(4)
    D, fromB = 16, 0
    n = 400
    for k in range(n):
        A, B = rng.integers(0, 50, D), rng.integers(50, 100, D)
        o = steps.draw(9, k, 1, steps.P_GA_SEL)
        c1, c2 = steps.ga_cross_pair(A, B, 9, k, 1, o, steps.GA_UNIFORM)
        assert all({c1[j], c2[j]} == {A[j], B[j]} for j in range(D))
        fromB += int(np.sum(c1 == B))
    total = n * D
    assert abs(fromB - total / 2) <= 4 * math.sqrt(total / 4)


def test_disruptive_uniform_swaps_half_of_the_differing_genes():
    rng = np.random.default_rng(5)
    D = 12
    swapped_at = np.zeros(D)
    for k in range(500):
        A = rng.integers(0, 4, D)
        B = np.where(rng.random(D) < 0.6, rng.integers(0, 4, D), A)
        o = steps.draw(13, k, 2, steps.P_GA_SEL)
        c1, c2 = steps.ga_cross_pair(A, B, 13, k, 2, o, steps.GA_DISRUPTIVE_UNIFORM)
        diff = [j for j in range(D) if A[j] != B[j]]
        sw = [j for j in range(D) if c1[j] != A[j]]
        assert set(sw) <= set(diff) and len(sw) == len(diff) // 2
        assert all(c1[j] == B[j] and c2[j] == A[j] for j in sw)
        assert all(c1[j] == A[j] and c2[j] == B[j] for j in range(D) if j not in sw)
        for j in sw:
            swapped_at[j] += 1
    # no position is favoured: the swapped genes are a uniform half of the differing ones
    assert swapped_at.min() > 0.6 * swapped_at.mean()
