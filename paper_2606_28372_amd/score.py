"""Performance score over time against a calculated random-search baseline (Eq. 2, Section V-A).

A measurement harness around the library, not a step of the optimiser path: it runs many
optimiser runs per space through `Batch` (every generation on the GPU), reads the configurations
each generation evaluated (`ct_pop_evaluated`), and scores the runs' mean best-so-far curve
against the expected curve of random search over the valid configurations.

The paper defines the aggregate (Eq. 2: the mean over search spaces and sampling times of the
per-space score) and the budget (the time the baseline needs to cover 95% of the distance from
the space's median to its optimum); the per-space score comes from the methodology it cites.
Readings taken here:

* time is counted in evaluations of configurations, in the order the runs evaluate them
  (individual order within a generation; a DE generation that reinitialises evaluates its
  trials, then the new population).  Two cost models: "unique" (the default) charges one unit
  for each valid configuration the run has not evaluated before, and nothing for a repeat (a
  tuner's cache) or an invalid configuration (rejected by the constraint check before it would
  run); "every" charges one unit for every evaluation, invalid ones included;
* the baseline B(n) is the expected best of n evaluations of random search without replacement
  over the valid configurations (an exact expectation over the sorted objective values);
* the budget is the smallest n with B(n) <= median - 0.95 (median - optimum);
* the score at time t is (B(t) - F(t)) / (B(t) - optimum), F(t) the mean over runs of the best
  objective found by time t; a run with no valid configuration yet counts the worst valid value
  (0 means "as good as the baseline", 1 "the optimum at once", below 0 worse than random search);
* the sampling times are t_k = budget k / |T|, k = 1..|T|;
* an optimiser stops at Table IV's iteration limit (DE, with none, at the budget or after
  10 budget / pop_size generations) and keeps its best for the rest of the budget;
* objectives: the structured synthetic runtime model (`workloads.runtime_model`) by default, the
  structureless log-normal table on request.

Run as `python -m paper_2606_28372_amd.score [--runs 100] [--spaces ...] [--cost unique|every]
[--objective model|table] [--out file.json]`.
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time
from typing import Dict, List, Optional, Sequence

import numpy as np


# ---------------------------------------------------------------------------
# The calculated baseline
# ---------------------------------------------------------------------------

def baseline(sorted_values: np.ndarray, n: int) -> float:
    """Expected minimum of n values drawn without replacement from `sorted_values` (ascending).

    With N values, the minimum has rank >= k with probability S_k = C(N-k+1, n) / C(N, n), so
    E[min] = sum_k v_k (S_k - S_{k+1}); S_{k+1} / S_k = (N-k+1-n) / (N-k+1).
    """
    v = np.asarray(sorted_values, dtype=np.float64)
    N = len(v)
    if not 1 <= n <= N:
        raise ValueError("baseline: need 1 <= n <= number of values")
    k = np.arange(1, N, dtype=np.float64)               # ratio S_{k+1} / S_k for k = 1..N-1
    ratio = np.clip((N - k + 1 - n) / (N - k + 1), 0.0, 1.0)
    S = np.concatenate([[1.0], np.cumprod(ratio), [0.0]])
    return float(np.dot(v, S[:-1] - S[1:]))


def budget(sorted_values: np.ndarray, fraction: float = 0.95) -> int:
    """Smallest n whose baseline covers `fraction` of the distance from the median to the optimum."""
    v = np.asarray(sorted_values, dtype=np.float64)
    target = float(np.median(v)) - fraction * (float(np.median(v)) - float(v[0]))
    lo, hi = 1, len(v)
    while lo < hi:
        mid = (lo + hi) // 2
        if baseline(v, mid) <= target:
            hi = mid
        else:
            lo = mid + 1
    return lo


def sample_times(n_budget: int, n_samples: int) -> np.ndarray:
    return np.array([max(1, (n_budget * k) // n_samples) for k in range(1, n_samples + 1)], dtype=np.int64)


def best_at(evaluations: np.ndarray, t: int, worst: float) -> float:
    """Best objective of one run after t evaluations (objectives in evaluation order, +inf for
    an invalid configuration); a run that stopped earlier keeps its last best; while nothing
    valid has been found, the worst valid value."""
    e = np.asarray(evaluations, dtype=np.float64)
    if len(e) == 0 or t < 1:
        return worst
    b = float(np.min(e[: min(t, len(e))]))
    return worst if math.isinf(b) else b


def score_curve(runs: Sequence[np.ndarray], times: np.ndarray, sorted_values: np.ndarray) -> np.ndarray:
    """Per-time scores (B(t) - F(t)) / (B(t) - optimum) of a group of runs (each the objectives
    of its evaluations, in order)."""
    v = np.asarray(sorted_values, dtype=np.float64)
    opt, worst = float(v[0]), float(v[-1])
    # running minima, with the worst valid value standing for "nothing valid yet"
    best = [np.minimum(np.minimum.accumulate(np.asarray(r, dtype=np.float64)), worst) for r in runs]
    out = np.zeros(len(times))
    for a, t in enumerate(times):
        B = baseline(v, int(t))
        F = float(np.mean([b[min(int(t), len(b)) - 1] if len(b) and t >= 1 else worst for b in best]))
        out[a] = (B - F) / (B - opt) if B > opt else 0.0
    return out


# ---------------------------------------------------------------------------
# Runs on the GPU
# ---------------------------------------------------------------------------

NONE = 0xFFFFFFFF


def trajectories(sp, opts, obj_t, gens: int, stop=None) -> List[np.ndarray]:
    """Valid-list positions every run evaluates, in order (NONE for an invalid configuration),
    over its initial population and up to `gens` generations; the runs are stepped together, one
    captured graph per generation.  `stop(evaluated_lists)`, when given, is asked every 8
    generations and ends the stepping once it returns True."""
    from . import CT_STEP_GRAPH, Batch, Pop

    pops = [Pop.from_opt(sp, o, obj_t) for o in opts]
    ev: List[List[np.ndarray]] = [[p.evaluated().astype(np.int64)] for p in pops]
    reinits = [0] * len(pops)
    b = Batch(pops)
    for g in range(gens):
        if stop is not None and g % 8 == 0 and stop(ev):
            break
        b.step(1, CT_STEP_GRAPH)
        for k, p in enumerate(pops):
            ev[k].append(p.evaluated().astype(np.int64))
            if p.algo == 0:
                r = p.read()
                if r["reinits"] > reinits[k]:              # the new population was evaluated too
                    ev[k].append(r["pos"].astype(np.int64))
                    reinits[k] = r["reinits"]
    b.close()
    for p in pops:
        p.close()
    return [np.concatenate(e) for e in ev]


def charged(positions: np.ndarray, obj: np.ndarray, cost: str = "unique") -> np.ndarray:
    """Objective values of the evaluations that cost a unit of time, in order: every evaluation
    (+inf for an invalid one), or each valid configuration's first evaluation only."""
    pos = np.asarray(positions, dtype=np.int64)
    if cost == "every":
        out = np.full(len(pos), np.inf)
        ok = pos != NONE
        out[ok] = obj[pos[ok]]
        return out
    if cost != "unique":
        raise ValueError("cost is 'unique' or 'every'")
    pos = pos[pos != NONE]
    _, first = np.unique(pos, return_index=True)
    return np.asarray(obj, dtype=np.float64)[pos[np.sort(first)]]


def run_space(name: str, algos: Sequence[int], runs: int, seed: int = 100, n_samples: int = 50,
              obj_seed: int = 7, cost: str = "unique", objective: str = "model", log=None) -> Dict[str, object]:
    """Score every algorithm, constraint-aware and not, on one space: `runs` runs each."""
    import torch

    import workloads as W
    from . import Space

    spec = W.space(name)
    sp = Space.from_spec(spec)
    D = len(spec.params)
    if objective == "model":
        _, rows = sp.valid_list()
        obj = W.runtime_model(spec, rows.cpu().numpy()[:, :D], obj_seed)
    else:
        obj = W.objective(sp.n_valid, obj_seed)
    obj_t = torch.tensor(obj, device="cuda")
    obj64 = obj.astype(np.float64)
    v = np.sort(obj64)
    nb = budget(v)
    times = sample_times(nb, n_samples)
    out: Dict[str, object] = {"space": name, "n_cartesian": spec.n_cartesian, "n_valid": sp.n_valid,
                              "budget_evals": nb, "cost": cost, "objective": objective, "variants": {}}
    for algo in algos:
        for unaware in (0, 1):
            t0 = time.perf_counter()
            opts = [W.table_iv(algo, D, seed + r, unaware) for r in range(runs)]
            P = opts[0].pop_size
            maxiter = W.TABLE_IV_MAXITER[algo]
            gens = maxiter if maxiter is not None else 10 * (-(-nb // P))

            def spent(ev):
                return all(len(charged(np.concatenate(e), obj64, cost)) >= nb for e in ev)

            traj = trajectories(sp, opts, obj_t, gens, stop=spent)
            vals = [charged(t, obj64, cost) for t in traj]
            s = score_curve(vals, times, v)
            key = f"{W.ALGO_NAMES[algo]}{'-unaware' if unaware else ''}"
            out["variants"][key] = {
                "score": float(np.mean(s)), "pop_size": P,
                "generations": int(max(len(t) for t in traj) // P - 1),
                "charged_evals_mean": float(np.mean([min(len(x), nb) for x in vals])),
                "final_mean_best": float(np.mean([best_at(x, nb, v[-1]) for x in vals])),
                "seconds": time.perf_counter() - t0}
            if log:
                x = out["variants"][key]
                log(f"[score] {name} {key}: score {x['score']:+.3f} (P {P}, {x['generations']} generations, "
                    f"{x['charged_evals_mean']:.0f} of {nb} charged evaluations)")
    sp.close()
    return out


def aggregate(results: List[Dict[str, object]]) -> Dict[str, float]:
    """Eq. 2: per variant, the mean over spaces of the per-space (time-averaged) score."""
    keys = results[0]["variants"].keys()
    return {k: float(np.mean([r["variants"][k]["score"] for r in results])) for k in keys}


def main(argv: Optional[Sequence[str]] = None) -> int:
    import workloads as W
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--runs", type=int, default=100)
    ap.add_argument("--spaces", nargs="*", default=list(W.BAT_SPACES))
    ap.add_argument("--samples", type=int, default=50)
    ap.add_argument("--cost", choices=("unique", "every"), default="unique")
    ap.add_argument("--objective", choices=("model", "table"), default="model")
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    say = lambda *x: (print(*x, flush=True))  # noqa: E731
    res = [run_space(s, [W.ALGO_DE, W.ALGO_PSO, W.ALGO_FF, W.ALGO_GA], a.runs, n_samples=a.samples,
                     cost=a.cost, objective=a.objective, log=say)
           for s in a.spaces]
    agg = aggregate(res)
    doc = {"spaces": res, "aggregate": agg,
           "gain": {k: agg[k] - agg[k + "-unaware"] for k in agg if not k.endswith("-unaware")}}
    line = json.dumps(doc)
    if a.out:
        with open(a.out, "w") as f:
            f.write(line + "\n")
    print(json.dumps({"aggregate": agg, "gain": doc["gain"]}))
    return 0


if __name__ == "__main__":
    sys.exit(main())
