"""GPU parity of the non-constraint-aware DE / PSO / GA / Firefly (bit-exact against the oracle).

The variants of Sections IV-B and IV-C's last sentences: a random sample over the whole Cartesian
space, no repair, +inf for an invalid configuration.  Every generation's full state is compared
(member rows as well for DE and GA, whose members may be invalid).  The 20-parameter space has
about 3% valid configurations, so most members there are invalid; the tiny space makes DE's
reinitialisation and equal-trial rule fire.
"""
import numpy as np
import pytest

import workloads as W
from oracle import steps as ost
from tests.gpu_common import gpu_space, oracle_space, parse_snapshot, say, torch
from tests.test_gpu_steps import compare, make_pop

pytestmark = pytest.mark.gpu


def compare_u(pop, st, opt, D, where):
    compare(pop, st, opt, D, where)
    g = parse_snapshot(pop.snapshot(), opt.algo, opt.pop_size, D)
    assert g["unaware"], where
    if opt.algo in (W.ALGO_DE, W.ALGO_GA):
        bad = np.argwhere(g["rows"] != st.rows)
        assert len(bad) == 0, f"{where}: member rows differ at {bad[:3].tolist()}"


def run_u(space_name, opt, gens, obj_seed):
    t = torch()
    osp = oracle_space(space_name)
    obj = W.objective(osp.n_valid, obj_seed)
    sp = gpu_space(W.space(space_name))
    pop = make_pop(sp, opt, t.tensor(obj, device="cuda"))
    st = ost.init_run(osp, obj, opt)
    name = f"{space_name}/unaware {W.ALGO_NAMES[opt.algo]}/P{opt.pop_size}"
    compare_u(pop, st, opt, osp.D, f"{name} init")
    for gnum in range(gens):
        say(f"[gpu_unaware] {name} generation {gnum}")
        pop.step(1)
        st = ost.step_run(osp, obj, st, opt)
        compare_u(pop, st, opt, osp.D, f"{name} gen {gnum + 1}")
    return pop, st


def U(algo, P, seed, **kw):
    return W.OptParams(algo, P, seed, unaware=1, **kw)


@pytest.mark.parametrize("algo", [W.ALGO_DE, W.ALGO_PSO, W.ALGO_GA, W.ALGO_FF])
def test_gemm10_unaware(algo):
    run_u("gemm10", U(algo, 256, 21), 4, 1)


@pytest.mark.parametrize("algo", [W.ALGO_DE, W.ALGO_PSO, W.ALGO_GA, W.ALGO_FF])
def test_wide20_unaware_mostly_invalid(algo):
    run_u("wide20", U(algo, 128, 22), 3, 2)


def test_tiny_unaware_de_long_run():
    """30 generations of population 20 on the 168-configuration space: equal trials, trials
    already in the population and reinitialisations all occur."""
    _, st = run_u("tiny", U(W.ALGO_DE, 20, 23), 30, 0)
    assert st.gen == 30 and st.reinits > 0


def test_unaware_operators_and_crossovers():
    run_u("gemm10", U(W.ALGO_DE, 64, 24, de_method=2, de_crossover=1), 3, 1)       # rand2exp
    run_u("gemm10", U(W.ALGO_DE, 64, 25, de_method=4), 3, 1)                       # current-to-best
    run_u("gemm10", U(W.ALGO_GA, 64, 26, ga_crossover=1), 3, 1)                    # two-point
    run_u("gemm10", U(W.ALGO_GA, 65, 27, ga_crossover=3, mutation_chance=1), 3, 1)  # disruptive uniform


def test_unaware_populations_past_the_block():
    """DE with 2,000 members (two chunks of the pairwise selection, two members a thread) and
    GA with 1,500 (the multi-key rank sort over member indices)."""
    run_u("gemm10", U(W.ALGO_DE, 2000, 28), 2, 1)
    run_u("gemm10", U(W.ALGO_GA, 1500, 29), 2, 1)


def test_mixed_batch_aware_and_unaware():
    """Aware and non-aware runs of every algorithm stepped together in one captured graph."""
    from paper_2606_28372_amd import Batch
    t = torch()
    osp = oracle_space("gemm10")
    obj = W.objective(osp.n_valid, 1)
    sp = gpu_space(W.gemm10())
    obj_t = t.tensor(obj, device="cuda")
    opts = [W.OptParams(a, 96, 30 + a, unaware=u) for a in range(4) for u in (0, 1)]
    pops = [make_pop(sp, o, obj_t) for o in opts]
    sts = [ost.init_run(osp, obj, o) for o in opts]
    b = Batch(pops)
    for gnum in range(3):
        say(f"[gpu_unaware] mixed batch generation {gnum}")
        b.step(1)
        for k, o in enumerate(opts):
            sts[k] = ost.step_run(osp, obj, sts[k], o)
            where = f"mixed {W.ALGO_NAMES[o.algo]} unaware={o.unaware} gen {gnum + 1}"
            (compare_u if o.unaware else compare)(pops[k], sts[k], o, osp.D, where)
    b.close()


def test_unaware_snapshot_restore():
    t = torch()
    osp = oracle_space("wide20")
    obj_t = t.tensor(W.objective(osp.n_valid, 2), device="cuda")
    sp = gpu_space(W.wide20())
    for algo in range(4):
        pop = make_pop(sp, U(algo, 64, 31), obj_t)
        pop.step(2)
        snap = pop.snapshot()
        pop.step(3)
        a = pop.snapshot()
        pop.restore(snap)
        pop.step(3)
        assert pop.snapshot() == a, W.ALGO_NAMES[algo]


def test_unaware_errors():
    from paper_2606_28372_amd import CtError, Pop
    t = torch()
    sp = gpu_space(W.tiny())
    obj_t = t.ones(sp.n_valid, device="cuda")
    # more members than valid configurations is fine without the stratified valid sample
    Pop(sp, W.ALGO_GA, 300, 0, obj_t, unaware=1).close()
    with pytest.raises(CtError):
        Pop(sp, W.ALGO_DE, 8193, 0, obj_t, unaware=1)
    with pytest.raises(CtError):
        Pop(sp, W.ALGO_DE, 20, 0, obj_t, unaware=2)
    # an aware snapshot does not restore into a non-aware run
    a = Pop(sp, W.ALGO_GA, 20, 0, obj_t)
    u = Pop(sp, W.ALGO_GA, 20, 0, obj_t, unaware=1)
    with pytest.raises(CtError):
        u.restore(a.snapshot())
