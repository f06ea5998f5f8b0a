"""Pins of the oracle's Firefly step (Section IV-C, last paragraph; Table IV) -- CPU only.

The fixed-point exponential is checked against math.exp within its stated
bound; the move is checked at settings where its outcome follows from the
firefly rule itself: no attraction and no noise leave every firefly in place,
full attraction (beta = 1) puts firefly i on the last brighter firefly in index
order, no attraction across large distances, and beta against
B0 exp(-gamma r^2) with r in the paper's [0,1]^N coordinates.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import core
from oracle import steps as ost

ALPHA_Q16 = 13107       # 0.2
ONE = 65536


@pytest.fixture(scope="module")
def gemm10():
    return core.Space.from_spec(W.gemm10()).enumerate()


def test_exp_within_bound_and_monotone():
    rng = np.random.default_rng(0)
    xs = sorted(set([0, 1, 2, 3, (1 << 21) - 1] + [1 << b for b in range(21)] +
                    rng.integers(0, 1 << 21, 3000).tolist()))
    prev = None
    for x in xs:
        e = ost.ff_exp_q32(x)
        exact = math.exp(-x / 65536.0) * 2 ** 32
        assert abs(e - exact) <= 21, (x, e, exact)
        if prev is not None:
            assert e <= prev
        prev = e
    assert ost.ff_exp_q32(0) == 1 << 32
    assert ost.ff_exp_q32(1 << 21) == 0 and ost.ff_exp_q32(1 << 30) == 0
    t = ost.ff_exp_table()
    assert len(t) == 21 and all(abs(t[b] - math.exp(-2.0 ** (b - 16)) * 2 ** 32) <= 0.5 + 1e-3 for b in range(21))


def state(space, X, f):
    X = np.asarray(X, dtype=np.int64)
    f = np.asarray(f, dtype=np.float32)
    return ost.FFState(X, f, np.zeros(len(f), dtype=np.int64), np.float32(f.min()), 0, gen=3)


def random_state(space, P, seed):
    rng = np.random.default_rng(seed)
    M = int(space.radices.max())
    X = rng.integers(0, M * 65536, size=(P, space.D))
    f = rng.permutation(P).astype(np.float32) + 1.0
    return state(space, X, f)


def test_no_attraction_no_noise_is_static(gemm10):
    st = random_state(gemm10, 12, 1)
    assert np.array_equal(ost.ff_move(gemm10, st, 5, 0, ONE, 0), st.X)


def test_full_attraction_lands_on_last_brighter(gemm10):
    """gamma = 0 gives beta = B0 = 1, so every move lands exactly on the other firefly: after the
    moves towards the brighter ones in ascending index, firefly i sits on the last brighter one."""
    st = random_state(gemm10, 15, 2)
    Xn = ost.ff_move(gemm10, st, 5, ONE, 0, 0)
    for i in range(15):
        brighter = [j for j in range(15) if st.f[j] < st.f[i]]
        want = st.X[brighter[-1]] if brighter else st.X[i]
        assert np.array_equal(Xn[i], want), i
    # the brightest firefly never moves
    b = int(np.argmin(st.f))
    assert np.array_equal(Xn[b], st.X[b])


def test_far_fireflies_do_not_attract(gemm10):
    """gamma = 16 and fireflies at opposite corners in every dimension: gamma r^2 >= 32, e^-32 < 2^-32."""
    M = int(gemm10.radices.max())
    lo, hi = 0, M * 65536 - 1
    X = [[lo] * gemm10.D, [hi] * gemm10.D, [hi] * gemm10.D]
    st = state(gemm10, X, [3.0, 1.0, 2.0])
    Xn = ost.ff_move(gemm10, st, 5, ONE, 16 * ONE, 0)
    assert np.array_equal(Xn[0], X[0])          # both brighter fireflies are at the far corner
    assert np.array_equal(Xn[2], X[2])          # its brighter peer sits on it: beta = 1, no displacement
    assert np.array_equal(Xn[1], X[1])


@pytest.mark.parametrize("gamma", [ONE, 3 * ONE // 2, ONE // 4])
def test_beta_follows_the_distance_in_unit_coordinates(gemm10, gamma):
    """One move of the dimmer of two fireflies: x' - x = beta (x_j - x) with
    beta = B0 exp(-gamma r^2), r^2 = sum ((x_j - x)/(M 2^16))^2 (the [0,1]^N mapping)."""
    rng = np.random.default_rng(int(gamma))
    M = int(gemm10.radices.max())
    for _ in range(40):
        X = rng.integers(0, M * 65536, size=(2, gemm10.D))
        st = state(gemm10, X, [2.0, 1.0])
        Xn = ost.ff_move(gemm10, st, 5, ONE, gamma, 0)
        dx = (X[1] - X[0]).astype(np.float64)
        r2 = float(np.sum((dx / (M * 65536.0)) ** 2))
        beta = math.exp(-(gamma / 65536.0) * r2)
        moved = (Xn[0] - X[0]).astype(np.float64)
        assert np.all(np.abs(moved - beta * dx) <= 1 + np.abs(dx) * 2.0 ** -13)
        assert np.array_equal(Xn[1], X[1])


def test_noise_only_moves_within_alpha(gemm10):
    """B0 = 0: each move adds alpha (u - 1/2) M per dimension, |step| <= alpha M / 2 index units;
    fireflies with a brighter peer move, the brightest stays, and steps average out near zero."""
    M = int(gemm10.radices.max())
    P = 16
    X = np.full((P, gemm10.D), (M * 65536) // 2, dtype=np.int64)
    f = np.arange(P, dtype=np.float32) + 1.0
    st = state(gemm10, X, f)
    Xn = ost.ff_move(gemm10, st, 9, 0, ONE, ALPHA_Q16)
    step_max = ALPHA_Q16 * M * 32768 / 65536 + 1
    for i in range(P):
        d = Xn[i] - X[i]
        assert np.all(np.abs(d) <= i * step_max)             # i fireflies are brighter than firefly i
        assert (i == 0) == bool(np.all(d == 0))
    total = (Xn - X).astype(np.float64).sum()
    n_steps = gemm10.D * P * (P - 1) / 2
    assert abs(total) <= 4 * math.sqrt(n_steps) * step_max / math.sqrt(3)


def test_step_invariants_on_gemm10(gemm10):
    obj = W.objective(gemm10.n_valid, 1)
    st = ost.ff_init(gemm10, obj, 20, 4)
    M = int(gemm10.radices.max())
    best = [(float(st.best_f), st.best_pos)]
    for _ in range(6):
        st = ost.ff_step(gemm10, obj, st, 4, ONE, ONE, ALPHA_Q16)
        assert np.all((st.X >= 0) & (st.X < M * 65536))
        assert np.all(st.pos < gemm10.n_valid)
        assert np.array_equal(st.f, obj[st.pos])
        best.append((float(st.best_f), st.best_pos))
        assert best[-1] == min(best[-2], min(zip(st.f.tolist(), st.pos.tolist())))
    assert st.gen == 6
