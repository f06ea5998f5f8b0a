"""Pins of the oracle's non-constraint-aware variants (Sections IV-B and IV-C, last sentences).

Random initial populations are uniform over the Cartesian space (chi-square per parameter);
evaluation gives (NONE, +inf) exactly for invalid configurations; on a space without
constraints -- where repair is the identity and nothing is penalised -- one non-aware step
from the same state equals the constraint-aware step for DE, PSO, Firefly and (without
mutation) GA; the non-aware GA mutation changes exactly one parameter to another value.
"""
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


def test_random_rows_are_uniform_per_parameter():
    sp = free_space([5, 3, 7, 2])
    rows = steps.random_rows(sp, 3000, 17, 0)
    for j, r in enumerate(sp.radices):
        counts = np.bincount(rows[:, j], minlength=int(r))
        assert len(counts) == r and stats.chisquare(counts).pvalue > 1e-4
    X = steps.random_coords(sp, 500, 17)
    assert X.min() >= 0 and X.max() < 7 * 65536
    assert stats.kstest(X.ravel() / (7 * 65536.0), "uniform").pvalue > 1e-4


def test_evaluation_penalises_exactly_the_invalid(gemm10):
    sp, obj = gemm10
    rows = steps.random_rows(sp, 400, 5, 0)
    rows[:40] = sp.vrows[np.random.default_rng(1).choice(sp.n_valid, 40)]
    pos, f = steps.evaluate(sp, obj, rows)
    valid = sp.valid_rows(rows)
    assert np.all((pos == steps.NONE) == ~valid) and np.all(np.isinf(f) == ~valid)
    assert np.array_equal(f[valid], obj[pos[valid]]) and valid.sum() >= 40


def aware_from_rows(sp, obj, rows):
    pos = sp.pos(sp.encode(rows))
    f = obj[pos].astype(np.float32)
    b = min(zip(f.tolist(), pos.tolist()))
    return pos, f, b


@pytest.mark.parametrize("method", [steps.DE_BEST1, steps.DE_RAND2, steps.DE_CURRENTTOBEST1])
def test_unaware_de_equals_aware_without_constraints(method):
    sp = free_space([6, 5, 7, 4])
    obj = W.objective(sp.n_valid, 3)
    rng = np.random.default_rng(2)
    rows = sp.vrows[rng.choice(sp.n_valid, 24, replace=False)]
    pos, f, b = aware_from_rows(sp, obj, rows)
    a = steps.DEState(pos.copy(), f.copy(), np.float32(b[0]), int(b[1]), gen=3)
    u = steps.UState(rows.copy(), pos.copy(), f.copy(), np.float32(b[0]), int(b[1]), gen=3)
    a2 = steps.de_step(sp, obj, a, 9, 45875, 2576980378, method)
    u2 = steps.ude_step(sp, obj, u, 9, 45875, 2576980378, method)
    assert np.array_equal(a2.pos, u2.pos) and np.array_equal(a2.f, u2.f) and a2.best_pos == u2.best_pos
    assert np.array_equal(sp.vrows[u2.pos], u2.rows)


def test_unaware_ga_equals_aware_without_constraints_or_mutation():
    sp = free_space([6, 5, 7, 4])
    obj = W.objective(sp.n_valid, 4)
    rows = sp.vrows[np.random.default_rng(3).choice(sp.n_valid, 30, replace=False)]
    pos, f, b = aware_from_rows(sp, obj, rows)
    never = 1 << 40                          # threshold 2^32 // never = 0: no child mutates
    a2 = steps.ga_step(sp, obj, steps.GAState(pos, f, np.float32(b[0]), int(b[1]), 2), 5, never, 3)
    u2 = steps.uga_step(sp, obj, steps.UState(rows, pos, f, np.float32(b[0]), int(b[1]), 2), 5, never, 3)
    assert np.array_equal(a2.pos, u2.pos) and a2.best_pos == u2.best_pos


def test_unaware_pso_and_firefly_equal_aware_without_constraints():
    sp = free_space([6, 5, 7, 4])
    obj = W.objective(sp.n_valid, 5)
    st = steps.pso_init(sp, obj, 20, 6)
    for _ in range(3):
        a, u = steps.pso_step(sp, obj, st, 6, 32768, 196608, 32768), steps.upso_step(sp, obj, st, 6, 32768, 196608, 32768)
        for k in ("X", "V", "PB", "f_pb", "pb_pos"):
            assert np.array_equal(getattr(a, k), getattr(u, k)), k
        st = a
    ff = steps.ff_init(sp, obj, 20, 7)
    for _ in range(3):
        a, u = steps.ff_step(sp, obj, ff, 7, 65536, 65536, 13107), steps.uff_step(sp, obj, ff, 7, 65536, 65536, 13107)
        assert np.array_equal(a.X, u.X) and np.array_equal(a.pos, u.pos) and a.best_pos == u.best_pos
        ff = a


def test_unaware_ga_mutation_changes_one_parameter():
    sp = free_space([5, 1, 7, 4, 3])
    obj = W.objective(sp.n_valid, 6)
    row = np.array([[2, 0, 3, 1, 2]], dtype=np.int32)
    P = 400
    rows = np.repeat(row, P, axis=0)
    pos, f = steps.evaluate(sp, obj, rows)
    st = steps.UState(rows, pos, f, np.float32(f[0]), int(pos[0]), 1)
    out = steps.uga_step(sp, obj, st, 11, 1, 3)          # every child mutates; parents identical
    changed = (out.rows != row).sum(axis=1)
    where = np.argmax(out.rows != row, axis=1)
    # parameter 1 has one value: a draw that picks it leaves the child unchanged
    assert set(changed.tolist()) <= {0, 1} and np.all(where[changed == 1] != 1)
    assert np.all(out.rows[changed == 0][:, 1] == 0) and (changed == 0).sum() > 0
    picked = np.bincount(where[changed == 1], minlength=5)[[0, 2, 3, 4]]
    assert stats.chisquare(picked).pvalue > 1e-4


def test_unaware_steps_on_a_constrained_space(gemm10):
    sp, obj = gemm10
    for opt in (W.OptParams(W.ALGO_DE, 64, 3, unaware=1), W.OptParams(W.ALGO_GA, 64, 3, unaware=1),
                W.OptParams(W.ALGO_PSO, 32, 3, unaware=1), W.OptParams(W.ALGO_FF, 16, 3, unaware=1)):
        st = steps.init_run(sp, obj, opt)
        best = np.inf
        for _ in range(4):
            st = steps.step_run(sp, obj, st, opt)
            f, pos = (st.f_pb, st.pb_pos) if opt.algo == W.ALGO_PSO else (st.f, st.pos)
            fin = np.isfinite(f)
            assert np.all((pos == steps.NONE) == ~fin)
            assert np.array_equal(f[fin], obj[pos[fin]])
            bf = float(st.best_f)
            assert bf <= best
            best = bf
