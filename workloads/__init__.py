"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module only *describes* workloads: parameter value lists, constraint
strings, objective tables and population/hyperparameter choices.  It holds
none of the method's arithmetic (no constraint evaluation, no enumeration, no
repair, no optimiser step), so both the oracle and the GPU path can take their
inputs from here without sharing any computation.

The search spaces stand in for the paper's benchmark spaces (Section V-A,
Table III): those parameter lists, constraints and measured runtimes are not
available, so each space below takes a published *shape* (number of
parameters, values per parameter, number and kind of constraints, density)
and the runtime of every valid configuration is replaced by a seeded
log-normal table.

Parameter order is declaration order; the linear index of a configuration is
row-major with the last parameter fastest (the order of itertools.product).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Sequence

import numpy as np


@dataclasses.dataclass(frozen=True)
class SpaceSpec:
    """A tunable-parameter space: the CSP (X, D, C) of Section IV-A."""

    name: str
    params: Dict[str, List[int]]          # X and D: name -> ordered value list
    constraints: List[str]                # C: Python integer expressions over the names

    @property
    def names(self) -> List[str]:
        return list(self.params.keys())

    @property
    def radices(self) -> List[int]:
        return [len(v) for v in self.params.values()]

    @property
    def n_cartesian(self) -> int:
        return int(math.prod(self.radices))


def _pow2(lo: int, hi: int) -> List[int]:
    out, v = [], lo
    while v <= hi:
        out.append(v)
        v *= 2
    return out


def tiny() -> SpaceSpec:
    """Thread-block example of Section II (the bx*by bound) plus a tile bound; 168 configurations."""
    return SpaceSpec(
        "tiny",
        {
            "block_x": _pow2(16, 1024),
            "block_y": _pow2(1, 32),
            "tile": _pow2(1, 8),
        },
        ["32 <= block_x*block_y <= 1024", "block_x*tile <= 2048"],
    )


def gemm10() -> SpaceSpec:
    """GEMM-like space with ten integer parameters (128,000 configurations)."""
    t = _pow2(16, 256)
    return SpaceSpec(
        "gemm10",
        {
            "TM": t, "TN": t, "TK": t,
            "VW": [1, 2, 4, 8], "UN": [1, 2, 4, 8],
            "ST": [1, 2, 3, 4],
            "PA": [0, 1], "PB": [0, 1], "DB": [0, 1], "SW": [0, 1],
        },
        [
            "TM%(16*VW)==0 and TN%(16*UN)==0 and TK%(VW*UN)==0",
            "256 <= (TM//VW)*(TN//UN) <= 1024",
            "ST*TK*(TM+TN+4*(PA+PB))*4*(1+DB) <= 65536",
            "SW==0 or (TM>=64 and VW>=2)",
            "DB==0 or ST>=2",
            "PA+PB <= 1",
        ],
    )


def gemm13() -> SpaceSpec:
    """GEMM-like space sized to 16,000,000 configurations (adds wave tiles WM/WN/WK)."""
    t = _pow2(16, 256)
    return SpaceSpec(
        "gemm13",
        {
            "TM": t, "TN": t, "TK": t,
            "WM": t, "WN": t, "WK": t,
            "VW": [1, 2, 4, 8], "UN": [1, 2, 4, 8],
            "ST": [1, 2, 3, 4],
            "PA": [0, 1], "PB": [0, 1], "DB": [0, 1], "SW": [0, 1],
        },
        [
            "TM%WM==0 and TN%WN==0 and TK%WK==0",
            "WK%(VW*UN)==0",
            "64 <= (TM//WM)*(TN//WN)*64 <= 1024",
            "ST*TK*(TM+TN+4*(PA+PB))*4*(1+DB) <= 65536",
            "SW==0 or (TM>=64 and VW>=2)",
        ],
    )


def sparse16() -> SpaceSpec:
    """Large sparse space: 16 parameters, 4,353,564,672 configurations, 12 constraints."""
    p = {
        "a": list(range(1, 17)),
        "b": _pow2(1, 256),
        "c": [1, 2, 3, 4, 6, 8],
        "d": [1, 2, 4, 8],
        "e": [0, 1, 2, 3],
        "f": [16, 32, 64, 128],
        "g": [1, 3, 5, 7],
    }
    for k in range(9):
        p[f"h{k}"] = [1, 2, 4]
    return SpaceSpec(
        "sparse16",
        p,
        [
            "64<=a*b*d<=1024",
            "(a*c)%d==0",
            "b*f<=4096",
            "min(a,c*d)>=4",
            "max(e,h0)+h1<=4",
            "(b+g)%3!=0",
            "h2*h3*h4<=8",
            "a%g==0",
            "c*h5<=12",
            "min(b,f)>=8",
            "e+h6+h7+h8<=7",
            "max(a,2*c)<=f//4",
        ],
    )


def wide20() -> SpaceSpec:
    """20 parameters (rows of 32 bytes): 18 on/off switches and two 3-way choices; at most five
    switches on, and the two choices tied to the first switch (2,359,296 configurations)."""
    p = {f"s{k}": [0, 1] for k in range(18)}
    p["u"] = [1, 2, 3]
    p["v"] = [1, 2, 3]
    return SpaceSpec(
        "wide20",
        p,
        [
            " + ".join(f"s{k}" for k in range(18)) + " <= 5",
            "(u + v) % 2 == 0 or s0 == 1",
        ],
    )


# ---------------------------------------------------------------------------
# Stand-ins for the four real-world spaces of Table III (dedispersion, 2D
# convolution, hotspot, GEMM).  Their parameter lists and constraints are not
# published; each stand-in keeps the table's number of parameters, values per
# parameter (so the Cartesian size is exact), number of constraints and, with
# constraint bounds chosen for it, a density close to the table's:
#   dedispersion  22,272 configurations, 10,780 valid (48.40%; table 49.97%)
#   convolution   10,240 configurations,  4,338 valid (42.36%; table 42.60%)
#   hotspot   22,200,000 configurations, 344,576 valid (1.552%; table 1.576%)
#   GEMM         663,552 configurations, 114,768 valid (17.30%; table 17.62%)
# ---------------------------------------------------------------------------

def bat_dedispersion() -> SpaceSpec:
    """8 parameters (1 to 29 values), 3 constraints."""
    return SpaceSpec(
        "bat_dedispersion",
        {
            "block_size_x": [1, 2, 4, 8] + [16 * k for k in range(1, 26)],
            "block_size_y": [4, 8, 16],
            "tile_stride_x": [0, 1],
            "tile_stride_y": [0, 1],
            "tile_size_x": [1, 2, 3, 4],
            "tile_size_y": [1, 2, 4, 8],
            "loop_unroll_factor_channel": [0, 1, 2, 4],
            "blocks_per_sm": [0],
        },
        [
            "32 <= block_size_x*block_size_y <= 2048",
            "tile_size_x > 1 or tile_stride_x == 0",
            "tile_size_y > 1 or tile_stride_y == 0",
        ],
    )


def bat_convolution() -> SpaceSpec:
    """10 parameters (1 to 16 values), 4 constraints."""
    return SpaceSpec(
        "bat_convolution",
        {
            "block_size_x": [16 * k for k in range(1, 17)],
            "block_size_y": list(range(1, 17)),
            "tile_size_x": [1, 2, 3, 4, 8],
            "tile_size_y": [1, 2],
            "use_padding": [0, 1],
            "read_only": [0, 1],
            "filter_height": [15],
            "filter_width": [15],
            "image_height": [4096],
            "image_width": [4096],
        },
        [
            "block_size_x*block_size_y <= 1024",
            "block_size_x*block_size_y >= 64",
            "tile_size_x*tile_size_y <= 8",
            "use_padding == 0 or (block_size_x*tile_size_x + filter_width - 1)"
            "*(block_size_y*tile_size_y + filter_height - 1)*4 <= 36864",
        ],
    )


def bat_hotspot() -> SpaceSpec:
    """11 parameters (1 to 37 values), 5 constraints; the sparsest of the four."""
    return SpaceSpec(
        "bat_hotspot",
        {
            "block_size_x": [1, 2, 4, 8, 16] + [32 * k for k in range(1, 33)],
            "block_size_y": list(range(1, 26)),
            "tile_size_x": list(range(1, 26)),
            "tile_size_y": [1, 2, 3, 4, 5],
            "temporal_tiling_factor": [1, 2, 3, 4, 5, 6],
            "loop_unroll_factor_t": [1, 2, 3, 4],
            "blocks_per_sm": [0, 1, 2, 3],
            "sh_power": [0, 1],
            "max_tfactor": [10],
            "grid_width": [4096],
            "grid_height": [4096],
        },
        [
            "32 <= block_size_x*block_size_y <= 1024",
            "temporal_tiling_factor % loop_unroll_factor_t == 0",
            "temporal_tiling_factor <= max_tfactor",
            "(block_size_x*tile_size_x + 2*temporal_tiling_factor)*(block_size_y*tile_size_y + "
            "2*temporal_tiling_factor)*(2 + sh_power)*4 <= 24576",
            "blocks_per_sm == 0 or block_size_x*block_size_y*blocks_per_sm <= 2048",
        ],
    )


def bat_gemm() -> SpaceSpec:
    """17 parameters (1 to 4 values), 8 constraints."""
    return SpaceSpec(
        "bat_gemm",
        {
            "MWG": [16, 32, 64, 128], "NWG": [16, 32, 64, 128],
            "MDIMC": [8, 16, 32, 64], "NDIMC": [8, 16, 32, 64],
            "MDIMA": [8, 16, 32], "NDIMB": [8, 16, 32], "VWM": [1, 2, 4], "VWN": [1, 2, 4],
            "KWG": [16, 32], "KWI": [2, 8], "STRM": [0, 1], "STRN": [0, 1], "SA": [0, 1],
            "SB": [1], "KREG": [1], "GEMMK": [0], "PRECISION": [32],
        },
        [
            "MWG % (MDIMC*VWM) == 0",
            "NWG % (NDIMC*VWN) == 0",
            "MWG % (MDIMA*VWM) == 0",
            "NWG % (NDIMB*VWN) == 0",
            "KWG % ((MDIMC*NDIMC)//MDIMA) == 0",
            "KWG % KWI == 0",
            "STRM == 0 or MWG >= 32",
            "STRN == 0 or NWG >= 32",
        ],
    )


BAT_SPACES = ("bat_dedispersion", "bat_convolution", "bat_hotspot", "bat_gemm")

SPACES = {"tiny": tiny, "gemm10": gemm10, "gemm13": gemm13, "sparse16": sparse16, "wide20": wide20,
          "bat_dedispersion": bat_dedispersion, "bat_convolution": bat_convolution,
          "bat_hotspot": bat_hotspot, "bat_gemm": bat_gemm}


def space(name: str) -> SpaceSpec:
    return SPACES[name]()


# ---------------------------------------------------------------------------
# Objective tables: the measured runtime of each valid configuration is
# replaced by a seeded float32 log-normal(0, 0.5) value, indexed by the
# configuration's position in the ascending list of valid linear indices.
# All values are strictly positive.
# ---------------------------------------------------------------------------

def objective(n_valid: int, seed: int) -> np.ndarray:
    return np.random.default_rng(seed).lognormal(0.0, 0.5, int(n_valid)).astype(np.float32)


def runtime_model(spec: SpaceSpec, rows: np.ndarray, seed: int) -> np.ndarray:
    """Synthetic runtimes with the structure of a tuning landscape (for the score harness, where a
    structureless table would leave nothing for an optimiser to find): the log-runtime of a
    configuration is a sum of per-parameter bowls c_j (u_j - m_j)^2 over the normalised value
    index u_j in [0, 1], D/2 pairwise terms b (u_j - u_k)^2 and log-normal noise (sigma 0.15) per
    configuration.  rows: value indices [n, D] in valid-list order; returns float32 [n] > 0."""
    rng = np.random.default_rng(seed)
    D = len(spec.params)
    r = np.array(spec.radices, dtype=np.float64)
    u = np.asarray(rows, dtype=np.float64).reshape(-1, D) / np.maximum(r - 1.0, 1.0)
    c, m = rng.uniform(0.2, 1.5, D), rng.uniform(0.0, 1.0, D)
    logf = ((u - m) ** 2 * c).sum(axis=1)
    for _ in range(D // 2):
        j, k = rng.choice(D, 2, replace=False)
        logf += rng.uniform(0.2, 1.0) * (u[:, j] - u[:, k]) ** 2
    logf += rng.normal(0.0, 0.15, len(u))
    return np.exp(logf).astype(np.float32)


# ---------------------------------------------------------------------------
# Optimiser hyperparameters (Table IV), in the integer form both
# implementations consume: F as Q16.16, CR as a 32-bit threshold,
# PSO coefficients as Q16.16, GA mutation chance "one in X".
# ---------------------------------------------------------------------------

ALGO_DE, ALGO_PSO, ALGO_GA, ALGO_FF = 0, 1, 2, 3
ALGO_NAMES = {ALGO_DE: "DE", ALGO_PSO: "PSO", ALGO_GA: "GA", ALGO_FF: "Firefly"}


@dataclasses.dataclass(frozen=True)
class OptParams:
    algo: int
    pop_size: int
    seed: int
    # DE (Table IV: F 0.7, CR 0.6, best1bin)
    F_q16: int = 45875                  # round(0.7 * 2**16)
    CR_q32: int = 2576980378            # round(0.6 * 2**32)
    de_method: int = 1                  # 0 rand1, 1 best1, 2 rand2, 3 best2, 4 current-to-best1, 5 rand-to-best1
    de_crossover: int = 0               # 0 binomial, 1 exponential
    # PSO (Table IV: w 0.5, c1 3.0, c2 0.5)
    w_q16: int = 32768
    c1_q16: int = 196608
    c2_q16: int = 32768
    # GA (Table IV: single_point, mutation chance 5); rank selection Beta(1, beta_b)
    mutation_chance: int = 5
    beta_b: int = 3
    ga_crossover: int = 0               # 0 single point, 1 two point, 2 uniform, 3 disruptive uniform
    unaware: int = 0                    # 1: the non-constraint-aware variant (random init, no repair)
    # Firefly (Table IV: B0 1.0, gamma 1.0, alpha 0.2)
    ff_B0_q16: int = 65536
    ff_gamma_q16: int = 65536
    ff_alpha_q16: int = 13107           # round(0.2 * 2**16)


# Table IV's population sizes and iteration limits (DE's popsize is per parameter; DE has no
# iteration limit in the table and runs to the time budget).
TABLE_IV_POP = {ALGO_DE: 16, ALGO_PSO: 30, ALGO_FF: 20, ALGO_GA: 20}
TABLE_IV_MAXITER = {ALGO_DE: None, ALGO_PSO: 100, ALGO_FF: 100, ALGO_GA: 150}


def table_iv(algo: int, n_params: int, seed: int, unaware: int = 0) -> OptParams:
    """Table IV's hyperparameters for a space of n_params parameters (the defaults of OptParams)."""
    P = TABLE_IV_POP[algo] * (n_params if algo == ALGO_DE else 1)
    return OptParams(algo, P, seed, unaware=unaware)


def q16(x: float) -> int:
    return int(round(x * 65536.0))


def q32(x: float) -> int:
    return int(round(x * 4294967296.0))


# ---------------------------------------------------------------------------
# Batched / serving workload: many independent tuning problems with uneven
# dimensions, valid-set sizes and populations.
# ---------------------------------------------------------------------------

@dataclasses.dataclass(frozen=True)
class Problem:
    spec: SpaceSpec
    opt: OptParams
    obj_seed: int
    target_valid: int


def _linear_threshold(rng: np.random.Generator, radices: Sequence[int], weights: Sequence[int],
                      density: float) -> int:
    """Pick T so that roughly `density` of random configurations satisfy sum(w*p) <= T.

    Values of parameter j are 1..r_j, so the sum is estimated from uniform
    random draws (a threshold for the generator, not a count of the space).
    """
    n = 20000
    s = np.zeros(n, dtype=np.int64)
    for r, w in zip(radices, weights):
        s += w * rng.integers(1, r + 1, size=n)
    q = float(np.clip(density, 1.0 / n, 1.0))
    return int(np.quantile(s, q, method="lower"))


def batched_problem(rng: np.random.Generator, k: int, max_pop: int = 1024) -> Problem:
    """One problem of the batched distribution (D in 4..14, |V| target log-uniform 1e3..1e6)."""
    D = int(rng.integers(4, 15))
    target = int(round(10 ** rng.uniform(3.0, 6.0)))
    pop = int(rng.integers(16, max_pop + 1))
    algo = int(rng.integers(0, 3))
    rho = float(10 ** rng.uniform(-3.0, math.log10(0.5)))
    base = (target / rho) ** (1.0 / D)
    radices = [int(np.clip(round(base * rng.uniform(0.7, 1.3)), 2, 255)) for _ in range(D)]
    weights = [int(w) for w in rng.integers(1, 5, size=D)]
    # (p0*p1)%3 != 0 keeps about 4/9 of configurations; the linear bound supplies the rest
    T = _linear_threshold(rng, radices, weights, min(1.0, rho * 9.0 / 4.0))
    names = [f"p{j}" for j in range(D)]
    params = {nm: list(range(1, r + 1)) for nm, r in zip(names, radices)}
    lin = "+".join(f"{w}*{nm}" for w, nm in zip(weights, names))
    cons = [f"{lin} <= {T}", "(p0*p1)%3 != 0"]
    seed = int(rng.integers(0, 2**31 - 1))
    spec = SpaceSpec(f"batched{k}", params, cons)
    return Problem(spec, OptParams(algo=algo, pop_size=pop, seed=seed), obj_seed=seed + 1,
                   target_valid=target)


def batched(n_problems: int = 256, seed: int = 3, max_pop: int = 1024) -> List[Problem]:
    rng = np.random.default_rng(seed)
    return [batched_problem(rng, k, max_pop) for k in range(n_problems)]


def fit_pop(opt: OptParams, n_valid: int) -> OptParams:
    """The run's parameters with the population capped at the space's valid-set size."""
    return dataclasses.replace(opt, pop_size=min(opt.pop_size, n_valid)) if opt.pop_size > n_valid else opt


def serving_arrivals(n: int = 2000, mean_interval_s: float = 0.005, seed: int = 4) -> np.ndarray:
    """Poisson arrival times (seconds) of optimiser runs: exponential inter-arrival gaps."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(mean_interval_s, size=n))


# Reference configurations used by tests and the benchmark.
CONFIGS = {
    "tiny": dict(space="tiny", obj_seed=0, runs=[OptParams(ALGO_DE, 20, 0)], generations=100),
    "gemm": dict(space="gemm13", obj_seed=1,
                 runs=[OptParams(ALGO_DE, 1024, 1), OptParams(ALGO_PSO, 1024, 1),
                       OptParams(ALGO_GA, 1024, 1)], generations=500),
    "gemm10": dict(space="gemm10", obj_seed=1,
                   runs=[OptParams(ALGO_DE, 1024, 1), OptParams(ALGO_PSO, 1024, 1),
                         OptParams(ALGO_GA, 1024, 1)], generations=500),
    "sparse16": dict(space="sparse16", obj_seed=2, runs=[OptParams(ALGO_GA, 4096, 2)],
                     generations=1000),
}
