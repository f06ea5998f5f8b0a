"""Pins the oracle's full enumeration of the valid set (Section IV-A).

Pins used: Python-eval brute force on small spaces, closed-form counts for
power-of-two product bounds (inclusion-exclusion over exponent sums), an
independent numpy engine for the GEMM-like spaces, a factored exact count
for the large sparse space, and the structural invariants of the bitmask
and the list.
"""
import itertools
import math

import hypothesis.strategies as st
import numpy as np
import pytest
from hypothesis import given, settings, HealthCheck

import workloads as W
from oracle import brute, core
from tests.helpers import npeval


def popcount_words(words):
    return int(np.unpackbits(words.view(np.uint8)).sum())


def test_tiny_matches_python_brute_force():
    spec = W.tiny()
    lin, rows = brute.enumerate_space(spec.names, list(spec.params.values()), spec.constraints)
    sp = core.Space.from_spec(spec).enumerate()
    assert sp.vlin.tolist() == lin
    assert sp.vrows.tolist() == [list(r) for r in rows]
    assert sp.n_valid == 100 and lin[0] == 4 and lin[-1] == 145
    assert popcount_words(sp.words) == 100


def count_sum_at_most(K, sizes):
    """#{(a_1..a_D): 0 <= a_i < n_i, sum a_i <= K} by inclusion-exclusion (stars and bars)."""
    D = len(sizes)
    tot = 0
    for m in range(D + 1):
        for S in itertools.combinations(sizes, m):
            k = K - sum(S)
            if k >= 0:
                tot += (-1) ** m * math.comb(k + D, D)
    return tot


def count_sum_between(lo, hi, sizes):
    return count_sum_at_most(hi, sizes) - (count_sum_at_most(lo - 1, sizes) if lo > 0 else 0)


def test_tiny_closed_form():
    # block_x = 2^a (a in 4..10), block_y = 2^b (b in 0..5), tile = 2^c (c in 0..3).
    # 32 <= bx*by <= 1024  <=>  5 <= a+b <= 10 ; bx*tile <= 2048 <=> a+c <= 11.
    # Shift a' = a-4 (0..6): 1 <= a'+b <= 6 and a'+c <= 7.
    alone1 = count_sum_between(1, 6, [7, 6]) * 4
    alone2 = count_sum_at_most(7, [7, 4]) * 6
    assert (alone1, alone2) == (104, 150)
    both = sum(1 for a in range(7) for b in range(6) for c in range(4) if 1 <= a + b <= 6 and a + c <= 7)
    spec = W.tiny()
    for k, cons in enumerate([[spec.constraints[0]], [spec.constraints[1]], spec.constraints]):
        sp = core.Space(spec.names, list(spec.params.values()), cons).enumerate()
        assert sp.n_valid == [alone1, alone2, both][k]
    assert both == 100


@settings(max_examples=25, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(sizes=st.lists(st.integers(1, 6), min_size=1, max_size=4), frac=st.floats(0, 1))
def test_power_of_two_product_closed_form(sizes, frac):
    # p_j = 2^(a_j), constraint prod p_j <= 2^K  <=>  sum a_j <= K
    K = int(round(frac * sum(s - 1 for s in sizes)))
    names = [f"p{j}" for j in range(len(sizes))]
    vals = [[2 ** a for a in range(s)] for s in sizes]
    sp = core.Space(names, vals, [f"{'*'.join(names)} <= {2 ** K}"]).enumerate()
    assert sp.n_valid == count_sum_at_most(K, sizes)


space_strategy = st.integers(1, 4).flatmap(lambda D: st.tuples(
    st.lists(st.lists(st.integers(-5, 12), min_size=1, max_size=5), min_size=D, max_size=D),
    st.lists(st.sampled_from([
        "p0 + p1 <= 7", "p0 * p1 % 3 != 0", "max(p0, p1) - min(p0, p1) >= 2", "p0 // (p1 - 2) > 0",
        "p0 < p1 <= 9", "abs(p0 - 3) != 1 or p1 == 0", "not (p0 % 2 == 0 and p1 % 2 == 0)",
    ]), min_size=0, max_size=3)))


@settings(max_examples=60, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(sp_def=space_strategy)
def test_random_small_spaces_match_brute_force(sp_def):
    vals, cons = sp_def
    names = [f"p{j}" for j in range(len(vals))]
    if len(vals) < 2:
        cons = [c for c in cons if "p1" not in c]
    lin, rows = brute.enumerate_space(names, vals, cons)
    sp = core.Space(names, vals, cons).enumerate()
    assert sp.vlin.tolist() == lin
    assert popcount_words(sp.words) == len(lin)


@pytest.mark.parametrize("name,count", [("gemm10", 3629), ("gemm13", 206786)])
def test_gemm_counts_match_independent_numpy_engine(name, count):
    spec = W.space(name)
    ok = npeval.valid_mask(spec.names, list(spec.params.values()), spec.constraints)
    sp = core.Space.from_spec(spec).enumerate()
    assert np.array_equal(sp.vlin, np.flatnonzero(ok).astype(np.uint64))
    assert sp.n_valid == count
    assert popcount_words(sp.words) == count
    assert np.all(np.diff(sp.vlin.astype(np.int64)) > 0)


def sparse16_factored_count():
    """Exact |V| of the sparse 16-parameter space without enumerating it.

    The constraints touching h0..h8 involve, among the outer parameters,
    only c and e, so |V| = sum over valid outer prefixes (a..g) of
    inner(c, e), where inner counts valid (h0..h8) for that c, e.
    """
    spec = W.sparse16()
    outer = ["a", "b", "c", "d", "e", "f", "g"]
    inner = [f"h{k}" for k in range(9)]
    outer_cons = [c for c in spec.constraints if not any(h in c for h in inner)]
    inner_cons = [c for c in spec.constraints if any(h in c for h in inner)]
    env_g = {"__builtins__": {}, "min": min, "max": max, "abs": abs}
    inner_count = {}
    for cv in spec.params["c"]:
        for ev in spec.params["e"]:
            n = 0
            for hv in itertools.product(*[spec.params[h] for h in inner]):
                env = dict(zip(inner, hv), c=cv, e=ev)
                n += all(eval(c, env_g, env) for c in inner_cons)
            inner_count[(cv, ev)] = n
    tot = 0
    for ov in itertools.product(*[spec.params[o] for o in outer]):
        env = dict(zip(outer, ov))
        if all(eval(c, env_g, env) for c in outer_cons):
            tot += inner_count[(env["c"], env["e"])]
    return tot


def test_sparse16_factored_count_is_pinned_golden():
    import json, os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "sparse16_space.json")))
    assert sparse16_factored_count() == g["n_valid"] == 4657116


def test_sparse16_sampled_words_match_python():
    """Random bitmask words of the 4.35e9-configuration space against Python eval, bit by bit."""
    spec = W.sparse16()
    sp = core.Space.from_spec(spec)
    rng = np.random.default_rng(5)
    n_words = (sp.n_cartesian + 63) // 64
    env_g = {"__builtins__": {}, "min": min, "max": max, "abs": abs}
    checked_set = 0
    import json, os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "sparse16_space.json")))
    dense_words = [x // 64 for x in g["sample_lin"][::25]]          # words known to hold solutions
    for w in rng.integers(0, n_words, size=30).tolist() + [n_words - 1] + dense_words:
        word = int(sp.mask_words(w, w + 1)[0])
        for b in range(64):
            L = w * 64 + b
            if L >= sp.n_cartesian:
                assert not (word >> b) & 1
                continue
            row = sp.decode(np.array([L], dtype=np.uint64))[0]
            env = {n: spec.params[n][row[j]] for j, n in enumerate(spec.names)}
            expect = all(eval(c, env_g, env) for c in spec.constraints)
            assert bool((word >> b) & 1) == expect
            checked_set += expect
    assert checked_set >= len(dense_words)


def test_many_problem_counts_match_dynamic_programming():
    """The oracle's enumeration of many-problem spaces equals an exact DP count that never enumerates
    (linear bound by convolution of per-parameter sum distributions, the modulo pair by direct sum)."""
    from tests.helpers import dpcount
    done = 0
    for pr in W.batched(64, seed=3):
        if pr.spec.n_cartesian > 4_000_000:
            continue
        osp = core.Space.from_spec(pr.spec).enumerate()
        assert osp.n_valid == dpcount.count(pr.spec), pr.spec.name
        done += 1
    assert done >= 5
    # a hand-checkable case: p0, p1 in 1..3, p2 in 1..2, p0 + p1 + p2 <= 5, (p0*p1)%3 != 0
    spec = W.SpaceSpec("hand", {"p0": [1, 2, 3], "p1": [1, 2, 3], "p2": [1, 2]},
                       ["1*p0+1*p1+1*p2 <= 5", "(p0*p1)%3 != 0"])
    # admissible (p0, p1): (1,1) (1,2) (2,1) (2,2); p2 choices with sum <= 5: 2, 2, 2, 1
    assert dpcount.count(spec) == 7 == core.Space.from_spec(spec).enumerate().n_valid
