"""Pins of the oracle's step arithmetic against facts fixed by the algorithms' definitions.

Each test below targets one plausible mistake in oracle/steps.py and fails
under it:

  * pick_excluding (Alg. 1's three distinct random members): the draw is a
    bijection from [0, n - m) onto the complement of the excluded set, in
    ascending order, and uniform (chi-square);
  * DE mutation (Alg. 1, Mutate): with CR = 1 every trial equals
    clip(round_half_up(base + F * (x_r2 - x_r3))) for members base, r2, r3
    distinct from i (and from each other), where the rounding is computed
    here from exact rationals; F = 0.5 makes half-integers common, so a
    dropped "+1/2" term or a truncating rounding fails;
  * DE crossover (Alg. 1, Crossover): a coordinate takes the mutant with
    probability CR (plus the j_rand coordinate), measured against the
    binomial spread; a reversed comparison gives 1 - CR;
  * PSO update (Section IV-C): a cognitive-only step moves every coordinate
    towards the particle's own best, a social-only step towards the swarm's
    best, an inertia-only step never grows a velocity; the cognitive term
    uses the first output word of its Philox block and the social term the
    second (the counter contract);
  * GA (Section IV-D): every pair of children is the single-point crossover
    of two population members at one cut in 1..D-1, and the parents' ranks
    follow Beta(1, b) over the population sorted best first (mean 1/(b+1)),
    which fixes the sort direction; ga_children equals ga_step child by child.
"""
import math
from fractions import Fraction

import numpy as np
import pytest
from scipy import stats

import workloads as W
from oracle import core, steps


def free_space(radices):
    names = [f"p{j}" for j in range(len(radices))]
    return core.Space(names, [list(range(r)) for r in radices], []).enumerate()


@pytest.fixture(scope="module")
def gemm10():
    sp = core.Space.from_spec(W.gemm10()).enumerate()
    return sp, W.objective(sp.n_valid, 1)


# ---------------------------------------------------------------------------
# distinct random members
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n,excluded", [(7, [3]), (20, [19, 0]), (20, [5, 2, 11]), (1024, [0, 1023, 512])])
def test_pick_excluding_is_an_ordered_bijection(n, excluded):
    rest = [k for k in range(n) if k not in excluded]
    m = len(rest)
    for k in range(m):
        u = -(-(k << 32) // m)                          # smallest 32-bit draw that maps to k
        assert steps.pick_excluding(u, n, list(excluded)) == rest[k]
        assert steps.pick_excluding(u, n, list(reversed(excluded))) == rest[k]
    assert steps.pick_excluding(2 ** 32 - 1, n, list(excluded)) == rest[-1]


def test_pick_excluding_is_uniform():
    rng = np.random.default_rng(11)
    n, ex = 13, [4, 9]
    u = rng.integers(0, 2 ** 32, size=60_000, dtype=np.uint64)
    got = np.array([steps.pick_excluding(int(x), n, ex) for x in u])
    assert not np.isin(got, ex).any()
    counts = np.bincount(got, minlength=n)[[k for k in range(n) if k not in ex]]
    assert stats.chisquare(counts).pvalue > 1e-4


# ---------------------------------------------------------------------------
# DE mutation and crossover
# ---------------------------------------------------------------------------
def _round_half_up(x: Fraction) -> int:
    return math.floor(x + Fraction(1, 2))


@pytest.mark.parametrize("F_q16,use_best", [(32768, True), (65536, True), (32768, False), (45875, False)])
def test_de_mutant_is_base_plus_rounded_scaled_difference(F_q16, use_best):
    sp = free_space([9, 8, 7, 6, 5])
    obj = W.objective(sp.n_valid, 3)
    P, seed = 12, 21
    st = steps.de_init(sp, obj, P, seed)
    for _ in range(2):                                  # a later generation as well as the first
        X = sp.vrows[st.pos].astype(np.int64)
        best = sp.vrows[st.best_pos].astype(np.int64)
        trials = steps.de_trials(sp, st, seed, F_q16, 1 << 32, use_best)
        F = Fraction(F_q16, 65536)
        hi = sp.radices.astype(np.int64) - 1
        for i in range(P):
            others = [k for k in range(P) if k != i]
            found = False
            for r1 in (others if not use_best else [None]):
                base = best if use_best else X[r1]
                for r2 in others:
                    for r3 in others:
                        if r3 == r2 or r1 in (r2, r3):
                            continue
                        m = [min(max(_round_half_up(int(base[j]) + F * int(X[r2, j] - X[r3, j])), 0), int(hi[j]))
                             for j in range(sp.D)]
                        if list(trials[i]) == m:
                            found = True
                            break
                    if found:
                        break
                if found:
                    break
            assert found, f"trial {i} = {trials[i].tolist()} is no rounded F-scaled difference step"
        st = steps.de_step(sp, obj, st, seed, F_q16, 1 << 32, use_best)


def test_de_crossover_takes_the_mutant_with_probability_cr():
    sp = free_space([4] * 8)
    obj = W.objective(sp.n_valid, 5)
    P, seed, CR = 256, 9, 0.6
    st = steps.de_init(sp, obj, P, seed)
    took = tot = 0
    for _ in range(3):
        X = sp.vrows[st.pos]
        best = sp.vrows[st.best_pos]
        trials = steps.de_trials(sp, st, seed, 0, W.q32(CR), True)     # F = 0: the mutant is best
        diff = X != best[None, :]
        took += int(np.sum((trials == best[None, :]) & diff))
        tot += int(np.sum(diff))
        st = steps.de_step(sp, obj, st, seed, 0, W.q32(CR), True)
    # every coordinate takes the mutant with probability CR, j_rand (1 of D) always
    expect = CR + (1 - CR) / sp.D
    assert abs(took / tot - expect) < 4.5 * math.sqrt(expect * (1 - expect) / tot) + 1e-3, (took / tot, expect)


# ---------------------------------------------------------------------------
# PSO velocity / position update
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def pso_moved(gemm10):
    """A swarm a few generations in, so personal bests, the global best and velocities differ."""
    sp, obj = gemm10
    st = steps.pso_init(sp, obj, 64, 13)
    for _ in range(3):
        st = steps.pso_step(sp, obj, st, 13, 32768, 196608, 32768)
    assert np.any(st.PB != st.X) and np.any(st.V != 0)
    return sp, st


def test_pso_cognitive_term_moves_towards_own_best(pso_moved):
    sp, st = pso_moved
    X, V, _ = steps.pso_move(sp, st, 13, 0, 196608, 0)
    d = st.PB - st.X
    assert np.all(np.sign(V) * np.sign(d) >= 0) and np.all((d == 0) <= (V == 0))
    assert np.all(np.abs(V) <= 3 * np.abs(d) + 1)
    assert np.any(np.sign(st.PB[st.g_idx][None, :] - st.X) * np.sign(V) < 0)   # not the social direction


def test_pso_social_term_moves_towards_swarm_best(pso_moved):
    sp, st = pso_moved
    X, V, _ = steps.pso_move(sp, st, 13, 0, 0, 196608)
    d = st.PB[st.g_idx][None, :] - st.X
    assert np.all(np.sign(V) * np.sign(d) >= 0) and np.all((d == 0) <= (V == 0))
    assert np.any(np.sign(st.PB - st.X) * np.sign(V) < 0)                      # not the cognitive direction


def test_pso_inertia_alone_never_grows_a_velocity(pso_moved):
    sp, st = pso_moved
    X, V, snapped = steps.pso_move(sp, st, 13, 32768, 0, 0)
    M = int(sp.radices.max())
    assert np.all(np.abs(V) <= np.abs(st.V))
    assert np.array_equal(X, np.clip(st.X + V, 0, M * 65536 - 1))
    assert np.array_equal(snapped, np.minimum(X >> 16, sp.radices - 1))


def test_pso_draw_words_follow_the_counter_contract(pso_moved):
    """r1 (cognitive) is word 0 and r2 (social) word 1 of the block at (particle, generation,
    PSO purpose | dimension): with a unit coefficient the step is r * distance / 2^16."""
    sp, st = pso_moved
    _, V1, _ = steps.pso_move(sp, st, 13, 0, 65536, 0)
    _, V2, _ = steps.pso_move(sp, st, 13, 0, 0, 65536)
    GB = st.PB[st.g_idx]
    for i in range(0, 64, 7):
        for j in range(sp.D):
            w = core.philox(13, [i, st.gen, (steps.P_PSO_R << 24) | j, 0])
            assert V1[i, j] == ((w[0] >> 16) * int(st.PB[i, j] - st.X[i, j])) >> 16
            assert V2[i, j] == ((w[1] >> 16) * int(GB[j] - st.X[i, j])) >> 16


# ---------------------------------------------------------------------------
# GA selection and crossover
# ---------------------------------------------------------------------------
def _parents(rows_set, c0, c1):
    """(A, B, cut) with c0 = A[:cut] + B[cut:] and c1 = B[:cut] + A[cut:], A and B members."""
    D = len(c0)
    for cut in range(1, D):
        A = tuple(c0[:cut]) + tuple(c1[cut:])
        B = tuple(c1[:cut]) + tuple(c0[cut:])
        if A in rows_set and B in rows_set:
            return A, B, cut
    return None


def test_ga_children_are_single_point_crossovers_of_members(gemm10):
    sp, obj = gemm10
    st = steps.ga_init(sp, obj, 63, 4)                 # odd: the last pair keeps one child
    for _ in range(2):
        rows = sp.vrows[st.pos]
        members = {tuple(r) for r in rows.tolist()}
        kids = steps.ga_crossover(sp, st, 4, 3)
        for k in range(0, 62, 2):
            assert _parents(members, kids[k].tolist(), kids[k + 1].tolist()) is not None, k
        last = tuple(kids[62].tolist())
        assert any(any(m[:c] == last[:c] for m in members) and any(m[c:] == last[c:] for m in members)
                   for c in range(1, sp.D))
        st = steps.ga_step(sp, obj, st, 4, 5, 3)


@pytest.mark.parametrize("b", [1, 3, 5])
def test_ga_parent_ranks_follow_beta(gemm10, b):
    sp, obj = gemm10
    P = 600
    st = steps.ga_init(sp, obj, P, 7)
    rows = sp.vrows[st.pos]
    order = sorted(range(P), key=lambda i: (float(st.f[i]), int(st.pos[i])))      # best first
    rank_of = {tuple(rows[i]): r for r, i in enumerate(order)}
    kids = steps.ga_crossover(sp, st, 7, b)
    ranks = []
    for k in range(0, P, 2):
        found = _parents(set(rank_of), kids[k].tolist(), kids[k + 1].tolist())
        assert found is not None
        ranks += [rank_of[found[0]], rank_of[found[1]]]
    u = (np.array(ranks) + 0.5) / P
    mean, sd = 1.0 / (b + 1), math.sqrt(b / ((b + 1) ** 2 * (b + 2)))
    assert abs(u.mean() - mean) < 4.5 * sd / math.sqrt(len(u)) + 1e-3, (u.mean(), mean)
    assert stats.kstest(u, stats.beta(1, b).cdf).pvalue > 1e-4


def test_ga_children_equals_ga_step(gemm10):
    sp, obj = gemm10
    st = steps.ga_init(sp, obj, 96, 6)
    for _ in range(3):
        nxt = steps.ga_step(sp, obj, st, 6, 5, 3)
        kids = steps.ga_children(sp, obj, st, 6, 5, 3, np.arange(96))
        assert np.array_equal(kids, sp.vrows[nxt.pos])
        part = np.array([95, 3, 40, 41, 0])
        assert np.array_equal(steps.ga_children(sp, obj, st, 6, 5, 3, part), sp.vrows[nxt.pos[part]])
        st = nxt


def test_ga_mutation_chance_one_mutates_every_child(gemm10):
    """Chance 1 in 1: every child with a valid Hamming-1 neighbour moves to one."""
    sp, obj = gemm10
    st = steps.ga_init(sp, obj, 40, 8)
    never = steps.ga_step(sp, obj, st, 8, 1 << 40, 3)
    always = steps.ga_step(sp, obj, st, 8, 1, 3)
    a, n = sp.vrows[always.pos], sp.vrows[never.pos]
    assert np.all(np.sum(a != n, axis=1) == 1)
