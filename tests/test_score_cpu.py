"""The performance-score harness (Eq. 2) on the CPU: the calculated random-search baseline against
brute force, the budget rule, and the score's fixed points (0 for the baseline, 1 for the optimum
at once).  Also the Table III stand-ins' shapes, counted by the oracle."""
import itertools
import math

import numpy as np
import pytest

import workloads as W
from oracle import core as ocore
from paper_2606_28372_amd import score as S


@pytest.mark.parametrize("N", [1, 2, 5, 8])
def test_baseline_is_the_mean_minimum_over_all_subsets(N):
    rng = np.random.default_rng(N)
    v = np.sort(rng.lognormal(0.0, 0.5, N))
    v[N // 2:] = np.round(v[N // 2:], 1)                # some equal values
    v = np.sort(v)
    for n in range(1, N + 1):
        subsets = list(itertools.combinations(range(N), n))
        brute = sum(min(v[list(c)]) for c in subsets) / len(subsets)
        assert S.baseline(v, n) == pytest.approx(brute, rel=1e-12, abs=1e-12)


def test_baseline_end_points_and_monotone():
    v = np.sort(np.random.default_rng(3).lognormal(0.0, 0.5, 2000))
    assert S.baseline(v, 1) == pytest.approx(v.mean(), rel=1e-12)
    assert S.baseline(v, len(v)) == pytest.approx(v[0], rel=1e-12)
    b = [S.baseline(v, n) for n in range(1, 200)]
    assert all(x >= y for x, y in zip(b, b[1:]))
    with pytest.raises(ValueError):
        S.baseline(v, 0)


def test_baseline_against_sampling():
    """Random search itself: the mean best of 20,000 draws of n distinct values."""
    rng = np.random.default_rng(5)
    v = np.sort(rng.lognormal(0.0, 0.5, 500))
    for n in (3, 40):
        m = np.mean([v[rng.choice(500, n, replace=False)].min() for _ in range(20000)])
        assert S.baseline(v, n) == pytest.approx(m, rel=0.01)


def test_budget_is_the_first_time_the_baseline_reaches_95_percent():
    v = np.sort(np.random.default_rng(6).lognormal(0.0, 0.5, 5000))
    nb = S.budget(v)
    target = np.median(v) - 0.95 * (np.median(v) - v[0])
    assert S.baseline(v, nb) <= target < S.baseline(v, nb - 1)
    assert S.budget(v, 0.5) < nb < S.budget(v, 0.99)


def test_score_fixed_points():
    v = np.sort(np.random.default_rng(7).lognormal(0.0, 0.5, 3000))
    nb = S.budget(v)
    times = S.sample_times(nb, 20)
    # a run that holds the optimum from its first evaluation scores 1
    assert np.allclose(S.score_curve([np.full(nb, v[0])], times, v), 1.0)
    # a run whose best after n evaluations is the baseline B(n) scores 0
    base = np.array([S.baseline(v, n) for n in range(1, nb + 1)])
    assert np.allclose(S.score_curve([base], times, v), 0.0, atol=1e-12)
    # +inf (no valid configuration yet) counts as the worst value: below the baseline
    assert np.all(S.score_curve([np.full(nb, np.inf)], times, v) < 0)
    # the score of a group is that of its mean best: two runs above and below the baseline
    lo, hi = base - 0.01, base + 0.01
    assert np.allclose(S.score_curve([lo, hi], times, v), 0.0, atol=1e-12)


def test_best_at_running_minimum():
    ev = np.array([5.0, 6.0, np.inf, 4.0, 7.0, 2.0])
    assert S.best_at(ev, 0, 9.0) == 9.0          # before the first evaluation
    assert S.best_at(ev, 1, 9.0) == 5.0
    assert S.best_at(ev, 3, 9.0) == 5.0          # an invalid evaluation changes nothing
    assert S.best_at(ev, 4, 9.0) == 4.0
    assert S.best_at(ev, 1000, 9.0) == 2.0       # a finished run keeps its last best
    assert S.best_at(np.array([np.inf, np.inf]), 2, 9.0) == 9.0   # nothing valid: the worst value
    v = np.sort(np.random.default_rng(8).lognormal(0.0, 0.5, 100))
    ev = np.random.default_rng(9).choice(v, 40)
    times = np.arange(1, 41)
    want = [(S.baseline(v, t) - S.best_at(ev, t, v[-1])) / (S.baseline(v, t) - v[0]) for t in times]
    assert np.allclose(S.score_curve([ev], times, v), want, rtol=1e-12)


def test_charged_evaluations():
    obj = np.array([3.0, 1.0, 2.0, 5.0])
    N = S.NONE
    pos = np.array([2, N, 0, 2, 3, N, 0, 1])
    # every evaluation costs a unit; an invalid one is +inf
    assert np.array_equal(S.charged(pos, obj, "every"), [2.0, np.inf, 3.0, 2.0, 5.0, np.inf, 3.0, 1.0])
    # only first evaluations of valid configurations cost, in the order they happen
    assert np.array_equal(S.charged(pos, obj, "unique"), [2.0, 3.0, 5.0, 1.0])
    with pytest.raises(ValueError):
        S.charged(pos, obj, "free")


def test_runtime_model_structure():
    """The synthetic runtimes: positive, deterministic, and smooth (neighbouring values of one
    parameter differ less than random pairs)."""
    spec = W.bat_convolution()
    osp = ocore.Space.from_spec(spec).enumerate()
    f = W.runtime_model(spec, osp.vrows, 7)
    assert f.dtype == np.float32 and len(f) == osp.n_valid and (f > 0).all()
    assert np.array_equal(f, W.runtime_model(spec, osp.vrows, 7))
    lf = np.log(f.astype(np.float64))
    index = {tuple(r): k for k, r in enumerate(osp.vrows.tolist())}
    near = []
    for k, r in enumerate(osp.vrows.tolist()[:500]):
        r2 = list(r)
        r2[1] += 1
        if tuple(r2) in index:
            near.append(abs(lf[k] - lf[index[tuple(r2)]]))
    rng = np.random.default_rng(0)
    far = np.abs(lf[rng.integers(0, len(lf), 2000)] - lf[rng.integers(0, len(lf), 2000)])
    assert len(near) > 50 and np.mean(near) < 0.6 * np.mean(far)


@pytest.mark.parametrize("name,cart,valid", [
    ("bat_dedispersion", 22272, 10780), ("bat_convolution", 10240, 4338),
    ("bat_hotspot", 22200000, 344576), ("bat_gemm", 663552, 114768)])
def test_table_iii_stand_in_shapes(name, cart, valid):
    """Table III: Cartesian size, dimensions, constraint count and values per parameter exact;
    density within 2 points of the table's."""
    spec = W.space(name)
    table = {"bat_dedispersion": (8, 3, 29, 49.973), "bat_convolution": (10, 4, 16, 42.598),
             "bat_hotspot": (11, 5, 37, 1.576), "bat_gemm": (17, 8, 4, 17.622)}[name]
    assert spec.n_cartesian == cart and len(spec.params) == table[0] and len(spec.constraints) == table[1]
    assert max(spec.radices) == table[2] and min(spec.radices) == 1
    sp = ocore.Space.from_spec(spec).enumerate()
    assert sp.n_valid == valid
    assert abs(100.0 * valid / cart - table[3]) < 2.0


def test_table_iv_populations():
    assert W.table_iv(W.ALGO_DE, 8, 0).pop_size == 128          # popsize 16 per parameter
    assert W.table_iv(W.ALGO_PSO, 8, 0).pop_size == 30
    assert W.table_iv(W.ALGO_FF, 8, 0).pop_size == 20
    assert W.table_iv(W.ALGO_GA, 8, 0, unaware=1).unaware == 1
