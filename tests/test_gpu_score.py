"""The Eq. 2 harness on the GPU: the best-so-far trajectories it scores are the oracle's (aware
and non-aware runs with Table IV's hyperparameters on a Table III stand-in), and a small run of
the whole harness gives finite scores with the budget of the calculated baseline."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import steps as ost
from paper_2606_28372_amd import score as S
from tests.gpu_common import gpu_space, oracle_space, say, torch

pytestmark = pytest.mark.gpu


def oracle_evaluations(osp, obj, o, gens):
    """The same evaluation sequence from the oracle's states: the positions each step evaluated,
    and a DE reinitialisation's new population after its trials."""
    st = ost.init_run(osp, obj, o)
    out, re = [st.evaluated], 0
    for _ in range(gens):
        st = ost.step_run(osp, obj, st, o)
        out.append(st.evaluated)
        if getattr(st, "reinits", 0) > re:
            out.append(st.pos)
            re = st.reinits
    return np.concatenate([np.asarray(x, dtype=np.int64) for x in out])


@pytest.mark.parametrize("algo", [W.ALGO_DE, W.ALGO_PSO, W.ALGO_FF, W.ALGO_GA])
def test_trajectories_are_the_oracles(algo):
    t = torch()
    name = "bat_convolution"
    osp = oracle_space(name)
    obj = W.objective(osp.n_valid, 7)
    sp = gpu_space(W.space(name))
    opts = [W.table_iv(algo, osp.D, 100, u) for u in (0, 1)]
    say(f"[gpu_score] {W.ALGO_NAMES[algo]} trajectories")
    got = S.trajectories(sp, opts, t.tensor(obj, device="cuda"), 6)
    for o, ev in zip(opts, got):
        want = oracle_evaluations(osp, obj, o, 6)
        assert np.array_equal(ev, want), f"{W.ALGO_NAMES[algo]} unaware={o.unaware}"
        if o.unaware:
            assert (ev == S.NONE).any()                 # invalid evaluations are recorded


def test_de_reinitialisation_counts_its_evaluations():
    """A DE run forced to reinitialise every generation (rand1 with F = 0, CR = 1: every trial is
    a member): each generation evaluates 2P configurations, the trials all repeats."""
    t = torch()
    osp = oracle_space("bat_dedispersion")
    obj = W.objective(osp.n_valid, 7)
    sp = gpu_space(W.space("bat_dedispersion"))
    o = W.OptParams(W.ALGO_DE, 16, 5, F_q16=0, CR_q32=1 << 32, de_method=0)
    (ev,) = S.trajectories(sp, [o], t.tensor(obj, device="cuda"), 3)
    assert len(ev) == 16 * 7
    assert set(ev[16:32].tolist()) <= set(ev[:16].tolist())
    assert np.array_equal(ev, oracle_evaluations(osp, obj, o, 3))


def test_small_harness_run():
    say("[gpu_score] harness on the convolution stand-in, 3 runs per variant")
    r = S.run_space("bat_convolution", [W.ALGO_DE, W.ALGO_GA], runs=3, n_samples=10, objective="table")
    v = np.sort(W.objective(r["n_valid"], 7).astype(np.float64))
    assert r["budget_evals"] == S.budget(v)
    assert set(r["variants"]) == {"DE", "DE-unaware", "GA", "GA-unaware"}
    for k, x in r["variants"].items():
        assert math.isfinite(x["score"]) and x["score"] <= 1.0, k
    agg = S.aggregate([r])
    assert agg["GA"] == r["variants"]["GA"]["score"]
