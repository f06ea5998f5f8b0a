"""Late-generation GPU parity against the oracle, and served runs against the oracle.

A run is advanced on the GPU to a late generation g (converged populations:
DE claim ties and reinitialisations, tier-3 fallback repairs, large PSO
velocities), its snapshot is parsed into the oracle's state, and both step once
from there: the step is a pure function of (state, g, seed), so the GPU's next
snapshot must equal the oracle's next state bit for bit.  Served runs (one per
algorithm, drawn from the many-problem distribution) are compared with the
oracle's run of the same problem.
"""
import dataclasses

import numpy as np
import pytest

import workloads as W
from oracle import core as ocore
from oracle import steps as ost
from tests.gpu_common import gpu_space, oracle_space, parse_snapshot, say, torch
from tests.test_gpu_steps import compare, make_pop, oracle_init, oracle_step, ord_to_f32

pytestmark = pytest.mark.gpu


def state_from_snapshot(blob, opt, D):
    g = parse_snapshot(blob, opt.algo, opt.pop_size, D)
    if opt.algo == W.ALGO_PSO:
        return ost.PSOState(g["X"], g["V"], g["PB"], g["f_pb"], g["pb_pos"], int(g["g_idx"]), g["gen"])
    best_f = np.float32(ord_to_f32(g["best_ord"]))
    if opt.algo == W.ALGO_FF:
        return ost.FFState(g["X"], g["f"], g["pos"], best_f, int(g["best_pos"]), g["gen"])
    if opt.algo == W.ALGO_DE:
        return ost.DEState(g["pos"], g["f"], best_f, int(g["best_pos"]), g["gen"], g["reinits"])
    return ost.GAState(g["pos"], g["f"], best_f, int(g["best_pos"]), g["gen"])


@pytest.mark.parametrize("algo", [W.ALGO_DE, W.ALGO_PSO, W.ALGO_GA])
def test_gemm13_late_generations(algo):
    """Population 1024 on the 16M-configuration GEMM space (the bench's runs), one step from
    generations 100, 250 and 499 of 500."""
    t = torch()
    osp = oracle_space("gemm13")
    opt = W.OptParams(algo, 1024, 1)
    obj = W.objective(osp.n_valid, 1)
    sp = gpu_space(W.gemm13())
    pop = make_pop(sp, opt, t.tensor(obj, device="cuda"))
    at = 0
    for g in (100, 250, 499):
        pop.step(g - at)
        at = g
        st = state_from_snapshot(pop.snapshot(), opt, osp.D)
        assert st.gen == g
        say(f"[gpu_late] gemm13 {W.ALGO_NAMES[algo]} step from generation {g}")
        pop.step(1)
        at += 1
        nxt = oracle_step(osp, obj, st, opt)
        compare(pop, nxt, opt, osp.D, f"gemm13 {W.ALGO_NAMES[algo]} gen {g} -> {g + 1}")
    if algo == W.ALGO_DE:
        say(f"[gpu_late] DE reinitialisations by generation 500: {parse_snapshot(pop.snapshot(), algo, 1024, osp.D)['reinits']}")


def test_sparse16_ga_late_generations():
    """Population 4096 GA on the 4.35G-configuration sparse space: from generations 10, 100, 500 and
    999, 64 sampled children of the next generation against the oracle's, plus the best."""
    t = torch()
    osp = oracle_space("sparse16")
    opt = W.OptParams(W.ALGO_GA, 4096, 2)
    obj = W.objective(osp.n_valid, 2)
    sp = gpu_space(W.sparse16())
    pop = make_pop(sp, opt, t.tensor(obj, device="cuda"))
    rng = np.random.default_rng(99)
    table = ost.beta_rank_table(opt.pop_size, opt.beta_b)
    at = 0
    for g in (10, 100, 500, 999):
        pop.step(g - at)
        st = state_from_snapshot(pop.snapshot(), opt, osp.D)
        assert st.gen == g
        sample = np.sort(rng.choice(opt.pop_size, 64, replace=False))
        say(f"[gpu_late] sparse16 GA step from generation {g}")
        pop.step(1)
        at = g + 1
        after = parse_snapshot(pop.snapshot(), opt.algo, opt.pop_size, osp.D)
        kids = ost.ga_children(osp, obj, st, opt.seed, opt.mutation_chance, opt.beta_b, sample, table)
        assert np.array_equal(after["pos"][sample], osp.pos(osp.encode(kids))), f"generation {g}"
        assert np.array_equal(after["f"], obj[after["pos"]])
        # best-ever: the lexicographic minimum of the old best and the whole new population
        best = min([(float(st.best_f), st.best_pos)] + list(zip(after["f"].tolist(), after["pos"].tolist())))
        assert after["best_pos"] == best[1] and np.float32(ord_to_f32(after["best_ord"])) == np.float32(best[0])


def test_served_runs_match_the_oracle():
    """Three served runs, one per algorithm, each against the oracle's run of the same problem."""
    from paper_2606_28372_amd import Server
    chosen = {}
    for pr in W.batched(400, seed=21, max_pop=64):
        if pr.spec.n_cartesian <= 3_000_000 and pr.opt.algo not in chosen:
            chosen[pr.opt.algo] = pr
        if len(chosen) == 3:
            break
    assert len(chosen) == 3
    reqs = [(chosen[a], 12 + 3 * a) for a in (W.ALGO_DE, W.ALGO_PSO, W.ALGO_GA)]
    by_id = {}
    srv = Server(lambda rid, nv: W.objective(nv, by_id[rid].obj_seed), hbm_budget=4 << 30, max_active=16,
                 keep_snapshots=True)
    ids = []
    for pr, gens in reqs:
        rid = srv.submit(pr.spec, pr.opt, gens)
        by_id[rid] = pr
        ids.append(rid)
        srv.step()                     # the next run arrives while the earlier ones are on the GPU
    while srv.step():
        pass
    res = {r["id"]: r for r in srv.poll()}
    for rid, (pr, gens) in zip(ids, reqs):
        r = res[rid]
        assert r["status"] == 0 and r["generations"] == gens
        osp = ocore.Space.from_spec(pr.spec).enumerate()
        assert r["n_valid"] == osp.n_valid
        opt = W.fit_pop(pr.opt, osp.n_valid)
        obj = W.objective(osp.n_valid, pr.obj_seed)
        say(f"[gpu_late] served {W.ALGO_NAMES[opt.algo]} run: D={osp.D} |V|={osp.n_valid} P={opt.pop_size} "
            f"{gens} generations vs the oracle")
        st = oracle_init(osp, obj, opt)
        for _ in range(gens):
            st = oracle_step(osp, obj, st, opt)
        got = state_from_snapshot(srv.snapshot(rid), opt, osp.D)
        for k in ("pos", "f", "X", "V", "PB", "f_pb", "pb_pos"):
            if hasattr(st, k) and not isinstance(getattr(type(st), k, None), property):
                assert np.array_equal(getattr(got, k), getattr(st, k)), f"served {W.ALGO_NAMES[opt.algo]}: {k}"
        assert got.gen == st.gen and got.best_pos == st.best_pos
        assert r["best_pos"] == st.best_pos
    srv.close()
