"""Pins the oracle's DE / PSO / GA generation steps (Alg. 1, Sections IV-B..IV-D).

Pins used: special cases whose outcome is fixed by the algorithm's
definition (CR = 0 changes exactly one coordinate; F = 0 with best1bin and
CR = 1 proposes the incumbent best everywhere, so nothing is accepted and the
population is reinitialised; PSO with zero coefficients never moves; GA on
an all-identical population without mutation reproduces it), the beta
selection table against scipy's Beta CDF, and the invariants of each
algorithm (population inside the valid set, DE duplicate-free and per-slot
monotone, best values monotone), plus determinism of the pure step.
"""
import numpy as np
import pytest
from scipy import stats

import workloads as W
from oracle import core, steps


@pytest.fixture(scope="module")
def tiny():
    sp = core.Space.from_spec(W.tiny()).enumerate()
    return sp, W.objective(sp.n_valid, 0)


@pytest.fixture(scope="module")
def gemm10():
    sp = core.Space.from_spec(W.gemm10()).enumerate()
    return sp, W.objective(sp.n_valid, 1)


def free_space():
    """No constraints: every configuration is valid, so repair never changes a trial."""
    return core.Space(["a", "b", "c", "d"], [list(range(7)), list(range(5)), list(range(9)), list(range(3))], []).enumerate()


def test_init_is_stratified_and_distinct(gemm10):
    sp, _ = gemm10
    P = 64
    pos = steps.init_positions(sp, P, 5, 0)
    n = sp.n_valid
    for i, p in enumerate(pos):
        assert (i * n) // P <= p < ((i + 1) * n) // P
    assert len(set(pos.tolist())) == P


def test_de_cr_zero_changes_only_jrand():
    sp = free_space()
    obj = W.objective(sp.n_valid, 9)
    st = steps.de_init(sp, obj, 16, 3)
    X0 = sp.vrows[st.pos].copy()
    # run one step with CR = 0 and rand1bin and inspect the trials through acceptance:
    # every accepted member differs from its predecessor in at most one parameter
    st1 = steps.de_step(sp, obj, st, 3, F_q16=65536, CR_q32=0, use_best=False)
    X1 = sp.vrows[st1.pos]
    changed = np.flatnonzero(st1.pos != st.pos)
    assert len(changed) > 0
    for i in changed:
        assert np.sum(X1[i] != X0[i]) == 1


def test_de_f0_cr1_best1bin_proposes_best_and_reinitialises(tiny):
    sp, obj = tiny
    st = steps.de_init(sp, obj, 20, 0)
    st1 = steps.de_step(sp, obj, st, 0, F_q16=0, CR_q32=1 << 32, use_best=True)
    # every trial equals best, which is already in X: nothing accepted, so reinit with tag 1
    assert st1.reinits == 1
    assert np.array_equal(st1.pos, steps.init_positions(sp, 20, 0, 1))
    assert (float(st1.best_f), st1.best_pos) <= (float(st.best_f), st.best_pos)


def test_de_invariants_and_determinism(gemm10):
    sp, obj = gemm10
    P, seed = 40, 7
    st = steps.de_init(sp, obj, P, seed)
    prev = st
    for g in range(4):
        nxt = steps.de_step(sp, obj, prev, seed, 45875, 2576980378)
        assert len(set(nxt.pos.tolist())) == P                       # duplicate-free
        assert np.all(nxt.pos < sp.n_valid)                          # X subset of V
        if nxt.reinits == prev.reinits:
            assert np.all(nxt.f <= prev.f)                           # per-slot monotone
        assert (float(nxt.best_f), nxt.best_pos) <= (float(prev.best_f), prev.best_pos)
        assert obj[nxt.best_pos] == nxt.best_f
        prev = nxt
    again = steps.de_step(sp, obj, st, seed, 45875, 2576980378)
    first = steps.de_step(sp, obj, st, seed, 45875, 2576980378)
    assert np.array_equal(again.pos, first.pos)


def test_pso_zero_coefficients_static(gemm10):
    sp, obj = gemm10
    st = steps.pso_init(sp, obj, 32, 4)
    s1 = steps.pso_step(sp, obj, st, 4, 0, 0, 0)
    assert np.array_equal(s1.X, st.X)
    assert np.array_equal(s1.f_pb, st.f_pb)
    # centres snap back to their own value index
    assert np.array_equal(np.minimum(st.X >> 16, sp.radices - 1), sp.vrows[st.pb_pos])


def test_pso_invariants(gemm10):
    sp, obj = gemm10
    st = steps.pso_init(sp, obj, 48, 5)
    M = int(sp.radices.max())
    for g in range(3):
        nxt = steps.pso_step(sp, obj, st, 5, 32768, 196608, 32768)
        assert np.all(nxt.f_pb <= st.f_pb)
        assert float(nxt.best_f) <= float(st.best_f)
        assert np.all((nxt.X >= 0) & (nxt.X < M * 65536))
        assert np.all(obj[nxt.pb_pos] == nxt.f_pb)
        st = nxt


def test_pso_unconstrained_evaluates_the_snapped_point():
    sp = free_space()
    obj = W.objective(sp.n_valid, 2)
    st = steps.pso_init(sp, obj, 12, 1)
    nxt = steps.pso_step(sp, obj, st, 1, 32768, 196608, 32768)
    snapped = np.minimum(nxt.X >> 16, sp.radices - 1)
    improved = nxt.f_pb < st.f_pb
    assert np.array_equal(sp.vrows[nxt.pb_pos[improved]], snapped[improved])


@pytest.mark.parametrize("P,b", [(20, 3), (1024, 3), (7, 1), (4096, 3), (33, 5)])
def test_beta_table_matches_scipy(P, b):
    t = steps.beta_rank_table(P, b)
    assert t[-1] == 1 << 32 and all(x <= y for x, y in zip(t, t[1:]))   # tail ranks may round to zero mass
    cdf = stats.beta(1, b).cdf((np.arange(P) + 1) / P)
    assert np.max(np.abs(np.array(t, dtype=np.float64) / 2.0 ** 32 - cdf)) < 1e-9
    assert steps.rank_from_draw(t, 0) == 0 and steps.rank_from_draw(t, 2 ** 32 - 1) == P - 1


def test_ga_identical_population_without_mutation_is_constant(gemm10):
    sp, obj = gemm10
    P = 16
    st = steps.ga_init(sp, obj, P, 3)
    st.pos[:] = st.pos[5]
    st.f[:] = obj[st.pos[5]]
    nxt = steps.ga_step(sp, obj, st, 3, mutation_chance=1 << 40, beta_b=3)
    assert np.all(nxt.pos == st.pos[5])


def test_ga_invariants(gemm10):
    sp, obj = gemm10
    st = steps.ga_init(sp, obj, 30, 8)
    for g in range(3):
        nxt = steps.ga_step(sp, obj, st, 8, 5, 3)
        assert np.all(nxt.pos < sp.n_valid) and len(nxt.pos) == 30
        assert (float(nxt.best_f), nxt.best_pos) <= (float(st.best_f), st.best_pos)
        st = nxt
