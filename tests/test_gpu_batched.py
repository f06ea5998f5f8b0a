"""Batched stepping is bit-identical to stepping each run alone.

A mixed group of runs (DE, PSO and GA over spaces with different parameter
counts, row widths and valid-set sizes) is advanced (a) one run at a time,
(b) with one launch per phase for the whole group, and (c) by replaying a
captured hipGraph of one generation; every run's full state must be equal
after every stage, and one run is also checked against the oracle.
"""
import numpy as np
import pytest

import workloads as W
from oracle import steps as ost
from tests.gpu_common import gpu_space, oracle_space, say, torch  # noqa: F401
from tests.test_gpu_steps import compare, oracle_init, oracle_step

pytestmark = pytest.mark.gpu


SPECS = [("tiny", W.OptParams(W.ALGO_DE, 20, 1)), ("gemm10", W.OptParams(W.ALGO_PSO, 200, 2)),
         ("gemm10", W.OptParams(W.ALGO_GA, 129, 3)), ("gemm13", W.OptParams(W.ALGO_DE, 512, 4)),
         ("tiny", W.OptParams(W.ALGO_GA, 33, 5)), ("gemm13", W.OptParams(W.ALGO_PSO, 300, 6)),
         ("gemm13", W.OptParams(W.ALGO_GA, 1024, 7)), ("gemm10", W.OptParams(W.ALGO_DE, 64, 8))]
OBJ_SEED = {"tiny": 10, "gemm10": 11, "gemm13": 12}


def make_runs(t, spaces):
    from paper_2606_28372_amd import Pop
    runs = []
    for name, opt in SPECS:
        sp, obj = spaces[name]
        runs.append(Pop.from_opt(sp, opt, obj))
    return runs


@pytest.fixture(scope="module")
def spaces():
    t = torch()
    out = {}
    for k, name in enumerate(["tiny", "gemm10", "gemm13"]):
        sp = gpu_space(W.space(name))
        out[name] = (sp, t.tensor(W.objective(sp.n_valid, OBJ_SEED[name]), device="cuda"))
    return out


def test_batched_and_graph_equal_plain(spaces):
    from paper_2606_28372_amd import Batch, CT_STEP_BATCHED, CT_STEP_GRAPH, step_many
    t = torch()
    plain, batched, graph = make_runs(t, spaces), make_runs(t, spaces), make_runs(t, spaces)
    b1, b2 = Batch(batched), Batch(graph)
    for stage in range(3):
        say(f"[gpu_batched] stage {stage}")
        step_many(plain, 4)
        b1.step(4, CT_STEP_BATCHED)
        b2.step(4, CT_STEP_GRAPH)
        t.cuda.synchronize()
        for k, (a, b, c) in enumerate(zip(plain, batched, graph)):
            sa = a.snapshot()
            assert sa == b.snapshot(), f"run {k}: batched differs at stage {stage}"
            assert sa == c.snapshot(), f"run {k}: graph replay differs at stage {stage}"
    b1.close()
    b2.close()


def test_batched_run_matches_oracle(spaces):
    from paper_2606_28372_amd import Batch, CT_STEP_GRAPH
    t = torch()
    runs = make_runs(t, spaces)
    b = Batch(runs)
    b.step(3, CT_STEP_GRAPH)
    t.cuda.synchronize()
    osp = oracle_space("gemm13")
    obj = W.objective(osp.n_valid, 12)
    for k in (3, 5, 6):
        name, opt = SPECS[k]
        osp = oracle_space(name)
        obj = W.objective(osp.n_valid, OBJ_SEED[name])
        st = oracle_init(osp, obj, opt)
        for _ in range(3):
            st = oracle_step(osp, obj, st, opt)
        compare(runs[k], st, opt, len(W.space(name).params), f"run {k} ({name}) after 3 graph generations")
    b.close()


def test_step_flags_equal(spaces):
    from paper_2606_28372_amd import CT_STEP_BATCHED, CT_STEP_GRAPH, step_many
    t = torch()
    a, b, c = make_runs(t, spaces), make_runs(t, spaces), make_runs(t, spaces)
    step_many(a, 3)
    step_many(b, 3, CT_STEP_BATCHED)
    step_many(c, 3, CT_STEP_GRAPH)
    for x, y, z in zip(a, b, c):
        assert x.snapshot() == y.snapshot() == z.snapshot()


def test_many_problem_batch():
    """24 problems of the many-problem distribution (uneven spaces, dimensions, populations,
    algorithms): graph replay equals plain stepping; the smallest space of each algorithm also
    matches the oracle."""
    from oracle import core as ocore
    from paper_2606_28372_amd import Batch, CT_STEP_GRAPH, Pop, step_many
    t = torch()
    probs = W.batched(24, seed=5)
    spaces, objs, a, b, opts = [], [], [], [], []
    for pr in probs:
        sp = gpu_space(pr.spec)
        obj = t.tensor(W.objective(sp.n_valid, pr.obj_seed), device="cuda")
        opt = W.fit_pop(pr.opt, sp.n_valid)
        spaces.append(sp)
        objs.append(obj)
        opts.append(opt)
        a.append(Pop.from_opt(sp, opt, obj))
        b.append(Pop.from_opt(sp, opt, obj))
    say(f"[gpu_batched] many-problem batch: valid sizes {[s.n_valid for s in spaces]}")
    bt = Batch(b)
    for stage in range(2):
        step_many(a, 3)
        bt.step(3, CT_STEP_GRAPH)
        t.cuda.synchronize()
        for k in range(len(probs)):
            assert a[k].snapshot() == b[k].snapshot(), f"problem {k} differs at stage {stage}"
    bt.close()
    for algo in (W.ALGO_DE, W.ALGO_PSO, W.ALGO_GA):
        mine = [k for k in range(len(probs)) if opts[k].algo == algo]
        k = min(mine, key=lambda q: spaces[q].n_cartesian)
        pr, opt = probs[k], opts[k]
        say(f"[gpu_batched] oracle check of problem {k} ({W.ALGO_NAMES[algo]}, {spaces[k].n_cartesian} configurations)")
        osp = ocore.Space.from_spec(pr.spec).enumerate()
        obj = W.objective(osp.n_valid, pr.obj_seed)
        st = oracle_init(osp, obj, opt)
        for _ in range(6):
            st = oracle_step(osp, obj, st, opt)
        compare(b[k], st, opt, len(pr.spec.params), f"problem {k} after 6 generations")


def test_autotuned_batch_equals_plain(spaces):
    """The autotuner's generation advances the runs exactly like a plain generation, whatever
    partitioning it picks; a later batch of the same shape reuses the choice."""
    from paper_2606_28372_amd import Batch, CT_STEP_GRAPH, step_many
    t = torch()
    plain, tuned = make_runs(t, spaces), make_runs(t, spaces)
    b = Batch(tuned)
    b.autotune(11, sample_every=5, force=True)    # sweeps at 0, 5 and 10; a timed block of each stream setting between
    tn = b.tuning()
    say(f"[gpu_batched] tuning {tn}")
    assert tn["tuned"] and tn["items"] in (2048, 4096, 8192, 16384, 32768) and tn["min_boxes"] in (8, 16, 32, 64)
    assert tn["grid_waves"] in (4096, 8192, 16384, 32768) and tn["mode"] in (0, 1, 2)
    step_many(plain, 11)
    t.cuda.synchronize()
    for x, y in zip(plain, tuned):
        assert x.snapshot() == y.snapshot()
    b.step(3, CT_STEP_GRAPH)
    step_many(plain, 3)
    t.cuda.synchronize()
    for x, y in zip(plain, tuned):
        assert x.snapshot() == y.snapshot()
    again = Batch(make_runs(t, spaces))
    assert again.tuning() == tn
    again.close()
    b.close()


@pytest.mark.parametrize("tune", [(64, 1, 64, 0), (2048, 8, 4096, 1), (8192, 64, 8192, 1), (8192, 1024, 512, 0),
                                  (64, 1, 64, 2), (4096, 16, 8192, 2), (8192, 64, 512, 2), (8192, 16, 16384, 2),
                                  (32768, 64, 32768, 2), (2048, 8, 100, 2), (4096, 32, 1000, 0)])
def test_set_tuning_equals_plain(spaces, tune):
    """Any installed scan partitioning (few or many items per launch, small or large boxes per
    part, small or large grids, grids of a multiple of 8 blocks (waves numbered XCD by XCD) or not
    (plain numbering); scan classes one after another, on side streams or fused per row width)
    gives the plain results, both launched directly and replayed from a graph."""
    from paper_2606_28372_amd import Batch, CT_STEP_BATCHED, CT_STEP_GRAPH, step_many
    t = torch()
    plain, tuned = make_runs(t, spaces), make_runs(t, spaces)
    b = Batch(tuned)
    b.set_tuning(*tune)
    got = b.tuning()
    assert (got["items"], got["min_boxes"], got["grid_waves"], got["mode"]) == tune and got["tuned"]
    say(f"[gpu_batched] set_tuning {tune}")
    b.step(3, CT_STEP_BATCHED)
    b.step(3, CT_STEP_GRAPH)
    step_many(plain, 6)
    t.cuda.synchronize()
    for k, (x, y) in enumerate(zip(plain, tuned)):
        assert x.snapshot() == y.snapshot(), f"run {k} differs under {tune}"
    b.close()


def test_set_tuning_rejects_out_of_range(spaces):
    from paper_2606_28372_amd import Batch, CtError
    t = torch()
    b = Batch(make_runs(t, spaces))
    before = b.tuning()
    for bad in [(63, 16, 4096, 0), (32769, 16, 4096, 0), (4096, 0, 4096, 0), (4096, 16, 32, 0), (4096, 16, 4096, 3)]:
        with pytest.raises(CtError):
            b.set_tuning(*bad)
    assert b.tuning() == before
    b.close()


def test_large_batch_equals_plain(spaces):
    """A batch of more than 16,384 individuals takes the narrow proposal groups (4 lanes per
    individual); one run at a time takes the wide ones (16 lanes): both give the same state."""
    from paper_2606_28372_amd import Batch, CT_STEP_BATCHED, Pop, step_many
    t = torch()
    sp, obj = spaces["gemm10"]
    opts = [W.OptParams(a, 1024, 40 + k) for k, a in enumerate([W.ALGO_DE, W.ALGO_PSO, W.ALGO_GA] * 6)]
    plain = [Pop.from_opt(sp, o, obj) for o in opts]
    big = [Pop.from_opt(sp, o, obj) for o in opts]
    assert sum(o.pop_size for o in opts) > 16384
    b = Batch(big)
    say("[gpu_batched] 18 runs x 1024 individuals")
    b.step(3, CT_STEP_BATCHED)
    step_many(plain, 3)
    t.cuda.synchronize()
    for k, (x, y) in enumerate(zip(plain, big)):
        assert x.snapshot() == y.snapshot(), f"run {k} differs"
    b.close()
    for p in plain + big:
        p.close()


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_wide_rows_batch_equals_plain(mode):
    """DE, PSO and GA over a 20-parameter space (32-byte rows) in one batch: the fused launch runs
    the index-distance, Alg. 2 and Alg. 3 scans of the widest rows in one kernel."""
    from paper_2606_28372_amd import Batch, CT_STEP_BATCHED, Pop, step_many
    t = torch()
    sp = gpu_space(W.space("wide20"))
    obj = t.tensor(W.objective(sp.n_valid, 13), device="cuda")
    opts = [W.OptParams(a, 200, 50 + a) for a in (W.ALGO_DE, W.ALGO_PSO, W.ALGO_GA)]
    plain = [Pop.from_opt(sp, o, obj) for o in opts]
    grouped = [Pop.from_opt(sp, o, obj) for o in opts]
    b = Batch(grouped)
    b.set_tuning(2048, 8, 4096, mode)
    say(f"[gpu_batched] wide20 mode {mode}")
    b.step(3, CT_STEP_BATCHED)
    step_many(plain, 3)
    t.cuda.synchronize()
    for k, (x, y) in enumerate(zip(plain, grouped)):
        assert x.snapshot() == y.snapshot(), f"run {k} differs"
    b.close()


def test_sparse16_partitions_agree():
    """On the 4.66M-row space (1,137 chunks) one part per candidate walks every chunk; the other
    partitionings cut candidates into many strided parts, or into whole eighths of up to 32,768
    items on a 32,768-wave grid: same results."""
    from paper_2606_28372_amd import Batch, CT_STEP_BATCHED, Pop
    t = torch()
    sp = gpu_space(W.space("sparse16"))
    obj = t.tensor(W.objective(sp.n_valid, 14), device="cuda")
    opts = [W.OptParams(W.ALGO_GA, 256, 60), W.OptParams(W.ALGO_DE, 256, 61), W.OptParams(W.ALGO_PSO, 256, 62)]
    runs = [[Pop.from_opt(sp, o, obj) for o in opts] for _ in range(3)]
    batches = [Batch(r) for r in runs]
    batches[0].set_tuning(64, 1, 4096, 2)          # fewer items than candidates: one part each
    batches[1].set_tuning(8192, 1, 8192, 0)        # many small parts
    batches[2].set_tuning(32768, 64, 32768, 2)     # the largest item target, parts in eighths
    say("[gpu_batched] sparse16 partitions")
    for b in batches:
        b.step(2, CT_STEP_BATCHED)
    t.cuda.synchronize()
    for other in runs[1:]:
        for k, (x, y) in enumerate(zip(runs[0], other)):
            assert x.snapshot() == y.snapshot(), f"run {k} differs"
    for b in batches:
        b.close()


def test_lanes_equal_plain():
    """A group of 64 runs or more steps as two lanes, each on a stream of its own: direct and
    graph-replayed generations (also from a side stream), autotuning and an installed tuning all
    leave every run where plain stepping does."""
    from paper_2606_28372_amd import Batch, CT_STEP_BATCHED, CT_STEP_GRAPH, Pop, step_many
    t = torch()
    probs = W.batched(72, seed=11)
    spaces, objs, a, b = [], [], [], []
    for pr in probs:
        sp = gpu_space(pr.spec)
        obj = t.tensor(W.objective(sp.n_valid, pr.obj_seed), device="cuda")
        opt = W.fit_pop(pr.opt, sp.n_valid)
        spaces.append(sp)
        objs.append(obj)
        a.append(Pop.from_opt(sp, opt, obj))
        b.append(Pop.from_opt(sp, opt, obj))
    bt = Batch(b)

    def check(stage):
        t.cuda.synchronize()
        for k in range(len(probs)):
            assert a[k].snapshot() == b[k].snapshot(), f"problem {k} differs after {stage}"

    say("[gpu_batched] lanes: direct generations")
    step_many(a, 2)
    bt.step(2, CT_STEP_BATCHED)
    check("direct generations")
    say("[gpu_batched] lanes: graph replays from a side stream")
    step_many(a, 3)
    side = t.cuda.Stream()
    side.wait_stream(t.cuda.current_stream())
    with t.cuda.stream(side):
        bt.step(3, CT_STEP_GRAPH)
    side.synchronize()
    check("graph replays")
    say("[gpu_batched] lanes: autotune")
    step_many(a, 2)
    bt.autotune(2, 1, force=True)
    check("autotuning")
    assert bt.tuning()["tuned"]
    bt.set_tuning(4096, 16, 8192, 2)
    assert bt.tuning()["items"] == 4096 and bt.tuning()["grid_waves"] == 8192
    step_many(a, 2)
    bt.step(2, CT_STEP_GRAPH)
    check("an installed tuning")
    bt.close()


def test_explicit_lanes_equal_plain(spaces):
    """ct_batch_create_lanes: three lanes over a small mixed group step like plain stepping; zero
    or more than eight lanes are refused."""
    from paper_2606_28372_amd import Batch, CT_STEP_GRAPH, CtError, step_many
    t = torch()
    a, b = make_runs(t, spaces), make_runs(t, spaces)
    bt = Batch(b, lanes=3)
    for stage in range(2):
        step_many(a, 2)
        bt.step(2, CT_STEP_GRAPH)
        t.cuda.synchronize()
        for k in range(len(a)):
            assert a[k].snapshot() == b[k].snapshot(), f"run {k} differs at stage {stage}"
    bt.close()
    for bad in (0, 9):
        with pytest.raises(CtError):
            Batch(b, lanes=bad)


def test_wide_batch_plans_in_slices():
    """300 runs in one lane: the wave that plans each repair pass takes the runs' sets 256 at a
    time (four per lane), carrying candidate and item offsets from one slice to the next; every
    run still ends where plain stepping leaves it."""
    import dataclasses
    from paper_2606_28372_amd import Batch, CT_STEP_BATCHED, CT_STEP_GRAPH, Pop, step_many
    t = torch()
    probs = W.batched(6, seed=13, max_pop=48)
    spaces, objs = [], []
    for pr in probs:
        sp = gpu_space(pr.spec)
        spaces.append(sp)
        objs.append(t.tensor(W.objective(sp.n_valid, pr.obj_seed), device="cuda"))
    a, b = [], []
    for j in range(300):
        k = j % len(probs)
        opt = dataclasses.replace(W.fit_pop(probs[k].opt, spaces[k].n_valid), seed=probs[k].opt.seed + 7919 * j)
        a.append(Pop.from_opt(spaces[k], opt, objs[k]))
        b.append(Pop.from_opt(spaces[k], opt, objs[k]))
    bt = Batch(b, lanes=1)
    say(f"[gpu_batched] wide batch: {len(b)} runs in one lane")
    for stage, mode in enumerate((CT_STEP_BATCHED, CT_STEP_GRAPH)):
        step_many(a, 3)
        bt.step(3, mode)
        t.cuda.synchronize()
        for k in range(len(a)):
            assert a[k].snapshot() == b[k].snapshot(), f"run {k} differs at stage {stage}"
    bt.close()
