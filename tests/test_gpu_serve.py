"""Serving loop on the GPU: runs that arrive while others are on the device are
admitted by footprint into the running batch, and each run's final state is
bit-identical to the same run stepped alone (which the step tests pin to the
oracle).  Also: the byte budget is never exceeded, runs that cannot run end with
the right status, and the charged footprint equals what the library allocates.
"""
import dataclasses

import numpy as np
import pytest

import workloads as W
from tests.gpu_common import gpu_space, say, torch

pytestmark = pytest.mark.gpu


def requests(n, seed, max_pop=96, gens=(6, 20)):
    rng = np.random.default_rng(seed + 100)
    out = []
    for pr in W.batched(n, seed=seed):
        opt = dataclasses.replace(pr.opt, pop_size=min(pr.opt.pop_size, max_pop))
        out.append((pr, opt, int(rng.integers(gens[0], gens[1] + 1))))
    return out


def objective_of(reqs, ids):
    by_id = {rid: reqs[k][0] for k, rid in enumerate(ids)}
    return lambda run_id, n_valid: W.objective(n_valid, by_id[run_id].obj_seed)


def run_alone(pr, opt, gens):
    from paper_2606_28372_amd import Pop
    t = torch()
    sp = gpu_space(pr.spec)
    obj = t.tensor(W.objective(sp.n_valid, pr.obj_seed), device="cuda")
    pop = Pop.from_opt(sp, opt, obj)
    fp = (sp.footprint(), pop.footprint(), sp.n_valid)
    pop.step(gens)
    snap = pop.snapshot()
    pop.close()
    sp.close()
    return snap, fp


def serve(reqs, budget, max_active=64, waves=3, steps_between=2):
    """Submit the requests in `waves` groups with a few server steps between them, then drain."""
    from paper_2606_28372_amd import Server
    ids = []
    holder = {}
    srv = Server(lambda rid, nv: holder["f"](rid, nv), hbm_budget=budget, max_active=max_active,
                 keep_snapshots=True)
    per = (len(reqs) + waves - 1) // waves
    max_active_seen = 0
    for w in range(waves):
        for pr, opt, gens in reqs[w * per:(w + 1) * per]:
            ids.append(srv.submit(pr.spec, opt, gens))
        holder["f"] = objective_of(reqs, ids)
        for _ in range(steps_between):
            srv.step()
            max_active_seen = max(max_active_seen, srv.stats()["active"])
    while srv.step():
        max_active_seen = max(max_active_seen, srv.stats()["active"])
    results = {r["id"]: r for r in srv.poll()}
    snaps = {rid: srv.snapshot(rid) for rid in ids if results[rid]["status"] == 0}
    stats = srv.stats()
    ms, act = srv.step_times()
    srv.close()
    return ids, results, snaps, stats, max_active_seen, (ms, act)


def test_serving_alone_equals_mix():
    reqs = requests(12, seed=7)
    ids, results, snaps, stats, max_seen, (ms, act) = serve(reqs, budget=8 << 30)
    say(f"[gpu_serve] stats {stats}, max active {max_seen}, {len(ms)} step intervals")
    assert stats["completed"] == len(reqs) and stats["rejected"] == 0
    assert max_seen > 1, "runs never overlapped"
    assert len(ms) > 0 and np.all(ms > 0) and np.all(act > 0)
    for k, (pr, opt, gens) in enumerate(reqs):
        r = results[ids[k]]
        assert r["status"] == 0 and r["generations"] == gens
        assert r["t_submit"] <= r["t_admit"] <= r["t_done"]
        alone, (sb, pb, nv) = run_alone(pr, opt, gens)
        assert snaps[ids[k]] == alone, f"request {k} ({W.ALGO_NAMES[opt.algo]}) differs from its run alone"
        assert r["footprint"] == sb + pb + 4 * nv, f"request {k}: charged footprint differs from allocation"


def test_serving_budget_is_respected():
    reqs = requests(10, seed=11, max_pop=64, gens=(4, 10))
    # room for roughly the three largest runs at once
    sizes = []
    for pr, opt, gens in reqs:
        _, (sb, pb, nv) = run_alone(pr, opt, 1)
        sizes.append(sb + pb + 4 * nv)
    budget = sum(sorted(sizes)[-3:]) + (2 << 20)
    ids, results, snaps, stats, max_seen, _ = serve(reqs, budget=budget, waves=1, steps_between=1)
    say(f"[gpu_serve] budget {budget}, peak {stats['peak_bytes']}, max active {max_seen}")
    assert stats["completed"] == len(reqs)
    assert stats["peak_bytes"] <= budget
    assert max_seen < len(reqs), "the budget never held a run back"
    for k, (pr, opt, gens) in enumerate(reqs):
        alone, _ = run_alone(pr, opt, gens)
        assert snaps[ids[k]] == alone


def test_serving_rejections_and_callback_errors():
    from paper_2606_28372_amd import CtError, Server
    tiny = W.space("tiny")
    empty = W.SpaceSpec("empty", {"a": [1, 2, 3], "b": [1, 2]}, ["a > 5"])
    three = W.SpaceSpec("three", {"a": [1, 2, 3], "b": [1]}, [])
    calls = []

    def obj(run_id, n_valid):
        calls.append(run_id)
        if run_id == bad_id:
            raise ValueError("objective table unavailable")
        return W.objective(n_valid, 0)

    srv = Server(obj, hbm_budget=1 << 30, max_active=8)
    too_few = srv.submit(three, W.OptParams(W.ALGO_DE, 10, 0), 3)         # DE needs 4 valid configurations
    capped = srv.submit(tiny, W.OptParams(W.ALGO_GA, 150, 0), 2)          # P cut to |V| = 100
    no_valid = srv.submit(empty, W.OptParams(W.ALGO_GA, 2, 0), 3)
    bad_id = srv.submit(tiny, W.OptParams(W.ALGO_PSO, 10, 0), 3)
    good = srv.submit(tiny, W.OptParams(W.ALGO_GA, 10, 0), 3)
    with pytest.raises(ValueError):
        srv.step()
    while srv.step():
        pass
    res = {r["id"]: r for r in srv.poll()}
    assert res[too_few]["status"] == -1 and res[no_valid]["status"] == -4 and res[bad_id]["status"] == -1
    assert res[capped]["status"] == 0 and res[capped]["pop_size"] == 100
    assert res[good]["status"] == 0 and res[good]["generations"] == 3
    with pytest.raises(CtError):
        srv.snapshot(good)                                                    # snapshots not kept
    srv.close()
    small = Server(lambda rid, nv: W.objective(nv, 0), hbm_budget=4096, max_active=2)
    rid = small.submit(tiny, W.OptParams(W.ALGO_DE, 20, 0), 2)
    while small.step():
        pass
    assert small.poll()[0]["status"] == -2                                    # can never fit
    small.close()
