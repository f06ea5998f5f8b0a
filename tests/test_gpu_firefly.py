"""GPU parity of the constraint-aware Firefly step against the oracle (bit-exact).

Table IV's setting (population 20, 100 iterations, B0 1, gamma 1, alpha 0.2)
on the tiny and 10-parameter GEMM spaces, generation by generation (positions,
brightness, evaluated configurations, best); other coefficients and larger
populations over a few generations; Firefly runs in a mixed batch (plain,
batched and graph-replayed stepping equal, and equal to the oracle); snapshot
and restore.
"""
import numpy as np
import pytest

import workloads as W
from tests.gpu_common import gpu_space, oracle_space, say, torch
from tests.test_gpu_steps import compare, make_pop, oracle_init, oracle_step, run

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name", ["tiny", "gemm10"])
def test_table_iv_firefly_run(name):
    run(name, W.OptParams(W.ALGO_FF, 20, 3), 100, 1)


def test_firefly_other_coefficients_and_sizes():
    run("gemm10", W.OptParams(W.ALGO_FF, 48, 4, ff_B0_q16=32768, ff_gamma_q16=131072, ff_alpha_q16=3277), 5, 1)
    run("gemm13", W.OptParams(W.ALGO_FF, 64, 5), 3, 1)
    run("wide20", W.OptParams(W.ALGO_FF, 32, 6, ff_gamma_q16=1 << 20, ff_alpha_q16=1 << 16), 3, 2)
    run("tiny", W.OptParams(W.ALGO_FF, 100, 7, ff_B0_q16=0, ff_alpha_q16=0), 3, 0)       # no move: static swarm


def test_firefly_in_a_mixed_batch():
    from paper_2606_28372_amd import Batch, CT_STEP_BATCHED, CT_STEP_GRAPH, Pop, step_many
    t = torch()
    specs = [("tiny", W.OptParams(W.ALGO_FF, 20, 11)), ("gemm10", W.OptParams(W.ALGO_DE, 64, 12)),
             ("gemm10", W.OptParams(W.ALGO_FF, 40, 13)), ("gemm10", W.OptParams(W.ALGO_GA, 33, 14)),
             ("tiny", W.OptParams(W.ALGO_PSO, 30, 15)), ("gemm13", W.OptParams(W.ALGO_FF, 20, 16))]
    spaces = {}
    for name in ("tiny", "gemm10", "gemm13"):
        sp = gpu_space(W.space(name))
        spaces[name] = (sp, t.tensor(W.objective(sp.n_valid, 3), device="cuda"))

    def make():
        return [Pop.from_opt(spaces[n][0], o, spaces[n][1]) for n, o in specs]
    plain, batched, graph = make(), make(), make()
    b1, b2 = Batch(batched), Batch(graph)
    for stage in range(2):
        say(f"[gpu_firefly] mixed batch stage {stage}")
        step_many(plain, 3)
        b1.step(3, CT_STEP_BATCHED)
        b2.step(3, CT_STEP_GRAPH)
        t.cuda.synchronize()
        for k, (a, b, c) in enumerate(zip(plain, batched, graph)):
            assert a.snapshot() == b.snapshot() == c.snapshot(), f"run {k} stage {stage}"
    for k, (name, opt) in enumerate(specs):
        osp = oracle_space(name)
        obj = W.objective(osp.n_valid, 3)
        st = oracle_init(osp, obj, opt)
        for _ in range(6):
            st = oracle_step(osp, obj, st, opt)
        compare(graph[k], st, opt, osp.D, f"mixed batch run {k} ({W.ALGO_NAMES[opt.algo]}) after 6 generations")
    b1.close()
    b2.close()


def test_firefly_snapshot_restore():
    t = torch()
    sp = gpu_space(W.gemm10())
    obj_t = t.tensor(W.objective(sp.n_valid, 1), device="cuda")
    pop = make_pop(sp, W.OptParams(W.ALGO_FF, 24, 8), obj_t)
    pop.step(3)
    snap = pop.snapshot()
    pop.step(4)
    a = pop.snapshot()
    pop.restore(snap)
    pop.step(4)
    assert pop.snapshot() == a
    bad = bytearray(snap)
    # the first coordinate of firefly 0 sits after the header (32 bytes), pos[P] and f[P]
    off = 32 + 24 * 8
    bad[off:off + 4] = np.int32(-1).tobytes()
    from paper_2606_28372_amd import CtError
    with pytest.raises(CtError):
        pop.restore(bytes(bad))
    assert pop.snapshot() == a
