"""GPU parity of the operator variants against the oracle (bit-exact, generation by generation).

DE: every mutation operator (rand1, best1, rand2, best2, current-to-best1, rand-to-best1) with
binomial and with exponential crossover; GA: single-point, two-point, uniform and disruptive-
uniform crossover; all on the 10-parameter GEMM space, one pair also on the 20-parameter
space, and a mixed batch of variants stepped batched and graph-replayed.
"""
import pytest

import workloads as W
from tests.gpu_common import gpu_space, oracle_space, say, torch
from tests.test_gpu_steps import compare, oracle_init, oracle_step, run

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("cross", [0, 1])
@pytest.mark.parametrize("method", [0, 1, 2, 3, 4, 5])
def test_de_operators(method, cross):
    run("gemm10", W.OptParams(W.ALGO_DE, 96, 20 + method, de_method=method, de_crossover=cross), 4, 1)


@pytest.mark.parametrize("cross", [1, 2, 3])
def test_ga_crossovers(cross):
    run("gemm10", W.OptParams(W.ALGO_GA, 96, 30 + cross, ga_crossover=cross), 4, 1)


def test_wide_variants():
    run("wide20", W.OptParams(W.ALGO_DE, 64, 41, de_method=2, de_crossover=1), 3, 2)
    run("wide20", W.OptParams(W.ALGO_GA, 64, 42, ga_crossover=3), 3, 2)


def test_variants_in_a_mixed_batch():
    from paper_2606_28372_amd import Batch, CT_STEP_BATCHED, CT_STEP_GRAPH, Pop, step_many
    t = torch()
    specs = [W.OptParams(W.ALGO_DE, 64, 51, de_method=4, de_crossover=1),
             W.OptParams(W.ALGO_GA, 65, 52, ga_crossover=2), W.OptParams(W.ALGO_DE, 40, 53, de_method=3),
             W.OptParams(W.ALGO_GA, 48, 54, ga_crossover=1), W.OptParams(W.ALGO_FF, 20, 55)]
    sp = gpu_space(W.gemm10())
    obj_t = t.tensor(W.objective(sp.n_valid, 1), device="cuda")
    plain = [Pop.from_opt(sp, o, obj_t) for o in specs]
    batched = [Pop.from_opt(sp, o, obj_t) for o in specs]
    graph = [Pop.from_opt(sp, o, obj_t) for o in specs]
    b1, b2 = Batch(batched), Batch(graph)
    step_many(plain, 3)
    b1.step(3, CT_STEP_BATCHED)
    b2.step(3, CT_STEP_GRAPH)
    t.cuda.synchronize()
    osp = oracle_space("gemm10")
    obj = W.objective(osp.n_valid, 1)
    for k, opt in enumerate(specs):
        assert plain[k].snapshot() == batched[k].snapshot() == graph[k].snapshot(), f"run {k}"
        st = oracle_init(osp, obj, opt)
        for _ in range(3):
            st = oracle_step(osp, obj, st, opt)
        compare(graph[k], st, opt, osp.D, f"mixed batch run {k}")
    b1.close()
    b2.close()


def test_operator_parameter_errors():
    from paper_2606_28372_amd import CtError, Pop
    t = torch()
    sp = gpu_space(W.tiny())
    obj_t = t.ones(sp.n_valid, device="cuda")
    with pytest.raises(CtError):
        Pop(sp, W.ALGO_DE, 5, 0, obj_t, de_method=2)        # rand2 needs six members
    with pytest.raises(CtError):
        Pop(sp, W.ALGO_DE, 20, 0, obj_t, de_method=6)
    with pytest.raises(CtError):
        Pop(sp, W.ALGO_DE, 20, 0, obj_t, de_crossover=2)
    with pytest.raises(CtError):
        Pop(sp, W.ALGO_GA, 20, 0, obj_t, ga_crossover=4)
