"""Oracle optimiser steps (DE, PSO, GA) -- TEST INFRASTRUCTURE ONLY.

Plain per-individual Python loops that follow the paper's algorithms in the
paper's order:
  - Differential Evolution: Alg. 1 (Mutate, Crossover, Repair, selection),
    Section IV-B (valid-only initial population, "u not in X", reinit);
  - Particle Swarm Optimization: Section IV-C (inertia, cognitive, social
    terms; mapping to [0,1]^N; evaluation through Alg. 2's repair, position
    unchanged);
  - Genetic Algorithm: Section IV-D (sorted population, beta-distributed rank
    selection, single-point crossover, Alg. 3 repair, then mutation to a
    random valid Hamming neighbour).

Randomness: every draw is a Philox4x32-10 output at a counter that names
its use (individual, generation, purpose, sub-index), so the step is a pure
function of (space, state, generation, seed).  Fixed-point rules (Q16.16 for
DE mutation and PSO coordinates) make every result an exact integer.

Where the paper is silent the readings are:
  DE  - synchronous generation; "u not in X" tested against the population at
        the start of the generation, later duplicates of an accepted trial are
        rejected (lowest individual index wins); reinitialise after a
        generation with no accepted trial; initial sample stratified over the
        ascending valid list (one stratum per member).
  PSO - positions in index units (the largest domain spans [0, M)), centre of
        value k at k + 1/2, snap = floor then clip to the domain; per-dimension
        r1, r2; zero initial velocity; pbest on strict improvement; gbest
        recomputed after all particles moved.
  GA  - rank selection from Beta(1, b) over normalised rank; cut point uniform
        in 1..D-1; two children per pair (the last one dropped for odd P);
        repair, then mutation with probability 1/mutation_chance.
  Firefly (Section IV-C, last paragraph: a PSO variant with PSO's sampling and
        Alg. 2 evaluation; Table IV: B0, gamma, alpha) - the standard firefly
        move (Yang, 2008): firefly i moves towards every firefly j that was
        brighter (lower objective) at the start of the generation, in
        ascending j, by beta = B0 exp(-gamma r^2) of the way plus a random
        step alpha (u - 1/2) per dimension; r is measured in PSO's [0,1]^N
        coordinates; positions in PSO's index units, clamped like PSO's;
        brightness is the objective of the Alg. 2 evaluation; the brightest
        firefly does not move.  Fixed point: exp by binary decomposition of
        the exponent (below).
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np

from . import core

P_INIT, P_DE_PICK, P_DE_CR, P_PSO_R, P_GA_SEL, P_GA_MUT = 1, 2, 3, 4, 5, 6
P_FF_NOISE, P_GA_XO = 9, 10

# DE mutation operators (Section IV-B, last paragraph) and crossovers; GA crossovers (Section IV-D)
DE_RAND1, DE_BEST1, DE_RAND2, DE_BEST2, DE_CURRENTTOBEST1, DE_RANDTOBEST1 = 0, 1, 2, 3, 4, 5
DE_BIN, DE_EXP = 0, 1
GA_SINGLE_POINT, GA_TWO_POINT, GA_UNIFORM, GA_DISRUPTIVE_UNIFORM = 0, 1, 2, 3


def uniform_below(u: int, n: int) -> int:
    """Integer in [0, n) from a 32-bit draw: floor(u * n / 2^32)."""
    return (int(u) * int(n)) >> 32


def pick_excluding(u: int, n: int, excluded: List[int]) -> int:
    """Uniform member of {0..n-1} minus `excluded` (the k-th member in ascending order)."""
    k = uniform_below(u, n - len(excluded))
    for e in sorted(excluded):
        if k >= e:
            k += 1
    return k


def draw(seed: int, c0: int, c1: int, purpose: int, sub: int = 0, extra: int = 0) -> List[int]:
    return core.philox(seed, [c0 & 0xFFFFFFFF, c1 & 0xFFFFFFFF, (purpose << 24) | sub, extra & 0xFFFFFFFF])


def init_positions(space: core.Space, P: int, seed: int, tag: int) -> np.ndarray:
    """Valid-only initial sample: member i is uniform inside stratum i of the valid list.

    Stratum i is [floor(i*|V|/P), floor((i+1)*|V|/P)); the strata are disjoint
    and non-empty for P <= |V|, so the members are distinct.
    """
    n = space.n_valid
    out = np.zeros(P, dtype=np.int64)
    for i in range(P):
        lo, hi = (i * n) // P, ((i + 1) * n) // P
        out[i] = lo + uniform_below(draw(seed, i, tag, P_INIT)[0], hi - lo)
    return out


def beta_rank_table(P: int, b: int) -> List[int]:
    """Cumulative Beta(1, b) selection thresholds over ranks, as exact 32-bit fractions.

    Rank r (0 = best) is chosen with probability CDF((r+1)/P) - CDF(r/P), where
    CDF(x) = 1 - (1 - x)^b.  Entry r is floor(CDF((r+1)/P) * 2^32); the last
    entry is 2^32.
    """
    Pb = P ** b
    return [((Pb - (P - r - 1) ** b) << 32) // Pb for r in range(P)]


def rank_from_draw(table: List[int], u: int) -> int:
    for r, t in enumerate(table):
        if u < t:
            return r
    raise AssertionError("unreachable: last threshold is 2^32")


def _lexmin(a, b):
    return a if (a[0], a[1]) <= (b[0], b[1]) else b


# ---------------------------------------------------------------------------
# Differential Evolution (Alg. 1)
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class DEState:
    pos: np.ndarray            # population as positions in the valid list
    f: np.ndarray              # float32 objective of each member
    best_f: float
    best_pos: int
    gen: int = 0
    reinits: int = 0
    evaluated: Optional[np.ndarray] = None   # positions the last step evaluated (trials after repair)


def de_init(space, obj, P, seed) -> DEState:
    pos = init_positions(space, P, seed, 0)
    f = obj[pos].astype(np.float32)
    b = min(zip(f.tolist(), pos.tolist()))
    return DEState(pos, f, np.float32(b[0]), int(b[1]), evaluated=pos.copy())


def de_picks(seed: int, i: int, g: int, P: int, k: int) -> List[int]:
    """k distinct members other than i: r1, r2, r3 from words 0-2 of the individual's first draw
    block (word 3 is j_rand), r4, r5 from words 0-1 of its second block."""
    o = draw(seed, i, g, P_DE_PICK)
    words = [o[0], o[1], o[2]]
    if k > 3:
        o2 = draw(seed, i, g, P_DE_PICK, 1)
        words += [o2[0], o2[1]]
    picks: List[int] = []
    for t in range(k):
        picks.append(pick_excluding(words[t], P, [i] + picks))
    return picks


def de_mutant_terms(method: int, i: int, r: List[int], X: np.ndarray, best_row: np.ndarray, j: int):
    """(base, scaled difference) of coordinate j: the mutant is base + F * difference (Alg. 1's
    Mutate for best1/rand1; Section IV-B's other operators)."""
    x = lambda k: int(X[k, j])  # noqa: E731
    b = int(best_row[j])
    if method == DE_RAND1:
        return x(r[0]), x(r[1]) - x(r[2])
    if method == DE_BEST1:
        return b, x(r[1]) - x(r[2])
    if method == DE_RAND2:
        return x(r[0]), x(r[1]) - x(r[2]) + x(r[3]) - x(r[4])
    if method == DE_BEST2:
        return b, x(r[1]) - x(r[2]) + x(r[3]) - x(r[4])
    if method == DE_CURRENTTOBEST1:
        return x(i), b - x(i) + x(r[1]) - x(r[2])
    if method == DE_RANDTOBEST1:
        return x(r[0]), b - x(r[0]) + x(r[1]) - x(r[2])
    raise ValueError("unknown DE method")


def de_trials(space: core.Space, st: DEState, seed: int, F_q16: int, CR_q32: int,
              use_best=True, crossover: int = DE_BIN) -> np.ndarray:
    """Alg. 1's Mutate and Crossover for every member: the trial vectors before repair.

    use_best: True / False for best1 / rand1 (Alg. 1), or one of the DE_* operators.  Binomial
    crossover takes each coordinate from the mutant with probability CR, and coordinate j_rand
    always; exponential crossover takes the circular run of coordinates starting at j_rand that
    continues while successive draws stay below CR (at most D).
    """
    method = use_best if not isinstance(use_best, bool) else (DE_BEST1 if use_best else DE_RAND1)
    P, D, g = len(st.pos), space.D, st.gen
    k = 5 if method in (DE_RAND2, DE_BEST2) else 3
    if P < k + 1:
        raise ValueError(f"DE operator {method} needs at least {k + 1} members")
    rad = space.radices
    X = space.vrows[st.pos]                              # value indices of the population
    best_row = space.vrows[st.best_pos]
    trials = np.zeros((P, D), dtype=np.int32)
    for i in range(P):
        r = de_picks(seed, i, g, P, k)
        j_rand = uniform_below(draw(seed, i, g, P_DE_PICK)[3], D)
        if crossover == DE_EXP:
            run = 1
            while run < D and draw(seed, i, g, P_DE_CR, run >> 2)[run & 3] < CR_q32:
                run += 1
        for j in range(D):
            base, diff = de_mutant_terms(method, i, r, X, best_row, j)
            # m = base + F*diff, rounded half up in Q16.16, clipped to the domain
            num = base * 65536 + F_q16 * diff + 32768
            m = min(max(num // 65536, 0), int(rad[j]) - 1)
            if crossover == DE_EXP:
                take = (j - j_rand) % D < run
            else:
                cr = draw(seed, i, g, P_DE_CR, j >> 2)[j & 3]
                take = cr < CR_q32 or j == j_rand
            trials[i, j] = m if take else X[i, j]
    return trials


def de_step(space: core.Space, obj: np.ndarray, st: DEState, seed: int, F_q16: int, CR_q32: int,
            use_best=True, crossover: int = DE_BIN) -> DEState:
    P, g = len(st.pos), st.gen
    trials = de_trials(space, st, seed, F_q16, CR_q32, use_best, crossover)
    # Repair: invalid trials move to the nearest valid configuration by index distance
    trials = space.repair(trials, core.INDEX_L1)
    upos = space.pos(space.encode(trials))
    fu = obj[upos].astype(np.float32)
    members = set(st.pos.tolist())
    pre = [bool(fu[i] <= st.f[i]) and int(upos[i]) not in members for i in range(P)]
    taken = set()
    new_pos, new_f = st.pos.copy(), st.f.copy()
    accepted = 0
    for i in range(P):
        if pre[i] and int(upos[i]) not in taken:
            taken.add(int(upos[i]))
            new_pos[i], new_f[i] = upos[i], fu[i]
            accepted += 1
    best = (float(st.best_f), st.best_pos)
    for i in range(P):
        best = _lexmin(best, (float(new_f[i]), int(new_pos[i])))
    reinits = st.reinits
    if accepted == 0:
        new_pos = init_positions(space, P, seed, g + 1)
        new_f = obj[new_pos].astype(np.float32)
        for i in range(P):
            best = _lexmin(best, (float(new_f[i]), int(new_pos[i])))
        reinits += 1
    return DEState(new_pos, new_f, np.float32(best[0]), int(best[1]), g + 1, reinits, evaluated=upos.copy())


# ---------------------------------------------------------------------------
# Particle Swarm Optimization (Section IV-C, Alg. 2)
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class PSOState:
    X: np.ndarray              # P x D positions, Q16.16 index units
    V: np.ndarray              # P x D velocities, Q16.16
    PB: np.ndarray             # P x D personal-best positions
    f_pb: np.ndarray           # personal-best objective
    pb_pos: np.ndarray         # valid-list position evaluated at the personal best
    g_idx: int                 # particle holding the global best
    gen: int = 0
    evaluated: Optional[np.ndarray] = None   # positions the last step evaluated (after Alg. 2)

    @property
    def best_f(self):
        return self.f_pb[self.g_idx]

    @property
    def best_pos(self):
        return int(self.pb_pos[self.g_idx])


def _gbest(f_pb: np.ndarray) -> int:
    return int(min(range(len(f_pb)), key=lambda i: (float(f_pb[i]), i)))


def centre_q16(k):
    return (2 * np.asarray(k, dtype=np.int64) + 1) * 32768


def pso_init(space, obj, P, seed) -> PSOState:
    pos = init_positions(space, P, seed, 0)
    X = centre_q16(space.vrows[pos])
    f = obj[pos].astype(np.float32)
    return PSOState(X.copy(), np.zeros_like(X), X.copy(), f.copy(), pos.copy(), _gbest(f), evaluated=pos.copy())


def pso_move(space: core.Space, st: PSOState, seed: int, w_q16: int, c1_q16: int, c2_q16: int):
    """Velocity and position update of every particle and the snapped configurations
    (before Alg. 2's repair): returns (X, V, snapped)."""
    P, D, g = st.X.shape[0], space.D, st.gen
    M = int(space.radices.max())
    hi = M * 65536 - 1
    X, V, PB = st.X.copy(), st.V.copy(), st.PB
    GB = st.PB[st.g_idx].copy()
    snapped = np.zeros((P, D), dtype=np.int32)
    for i in range(P):
        for j in range(D):
            o = draw(seed, i, g, P_PSO_R, j)
            r1, r2 = o[0] >> 16, o[1] >> 16
            x = int(X[i, j])
            v = ((w_q16 * int(V[i, j])) >> 16) \
                + ((((c1_q16 * r1) >> 16) * (int(PB[i, j]) - x)) >> 16) \
                + ((((c2_q16 * r2) >> 16) * (int(GB[j]) - x)) >> 16)
            x = min(max(x + v, 0), hi)
            V[i, j], X[i, j] = v, x
            snapped[i, j] = min(x >> 16, int(space.radices[j]) - 1)
    return X, V, snapped


def pso_step(space: core.Space, obj: np.ndarray, st: PSOState, seed: int, w_q16: int, c1_q16: int,
             c2_q16: int) -> PSOState:
    P, g = st.X.shape[0], st.gen
    X, V, snapped = pso_move(space, st, seed, w_q16, c1_q16, c2_q16)
    PB = st.PB.copy()
    # Evaluation goes through Alg. 2: invalid snapped points are replaced by the nearest
    # neighbour (Euclidean distance to the particle) of the first non-empty neighbour set.
    ev = space.repair(snapped, core.TIER_EUCLID, pos_q16=X)
    epos = space.pos(space.encode(ev))
    f = obj[epos].astype(np.float32)
    f_pb, pb_pos = st.f_pb.copy(), st.pb_pos.copy()
    for i in range(P):
        if f[i] < f_pb[i]:
            PB[i], f_pb[i], pb_pos[i] = X[i], f[i], epos[i]
    return PSOState(X, V, PB, f_pb, pb_pos, _gbest(f_pb), g + 1, evaluated=epos.copy())


# ---------------------------------------------------------------------------
# Genetic Algorithm (Section IV-D, Alg. 3)
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class GAState:
    pos: np.ndarray
    f: np.ndarray
    best_f: float
    best_pos: int
    gen: int = 0
    evaluated: Optional[np.ndarray] = None   # positions the last step evaluated (the children)


def ga_init(space, obj, P, seed) -> GAState:
    pos = init_positions(space, P, seed, 0)
    f = obj[pos].astype(np.float32)
    b = min(zip(f.tolist(), pos.tolist()))
    return GAState(pos, f, np.float32(b[0]), int(b[1]), evaluated=pos.copy())


def ga_cross_pair(A: np.ndarray, B: np.ndarray, seed: int, k: int, g: int, o: List[int], method: int):
    """The two children of pair k from parents A, B (Section IV-D's crossovers).

    single point: cut c in 1..D-1 (word 2), children A[:c]+B[c:] and B[:c]+A[c:];
    two point: two distinct cuts (words 2 and 3, the second drawn from the other D-2 points),
    children A[:c1]+B[c1:c2]+A[c2:] and its mirror (single point when D < 3);
    uniform: gene j from B when the top bit of draw (k, g, GA_XO | j/4, 0) word j%4 is set,
    the second child the complement;
    disruptive uniform: of the genes where A and B differ, exactly half (rounded down) are
    swapped -- the ones with the smallest keys (draw (k, g, GA_XO | j/4, 1) word j%4, ties by j).
    """
    D = len(A)
    if method == GA_SINGLE_POINT or (method == GA_TWO_POINT and D < 3):
        cut = 1 + uniform_below(o[2], D - 1)
        return np.concatenate([A[:cut], B[cut:]]), np.concatenate([B[:cut], A[cut:]])
    if method == GA_TWO_POINT:
        a = 1 + uniform_below(o[2], D - 1)
        b = 1 + pick_excluding(o[3], D - 1, [a - 1])
        c1, c2 = min(a, b), max(a, b)
        return (np.concatenate([A[:c1], B[c1:c2], A[c2:]]), np.concatenate([B[:c1], A[c1:c2], B[c2:]]))
    if method == GA_UNIFORM:
        fromB = np.array([draw(seed, k, g, P_GA_XO, j >> 2)[j & 3] >> 31 for j in range(D)], dtype=bool)
        return np.where(fromB, B, A), np.where(fromB, A, B)
    if method == GA_DISRUPTIVE_UNIFORM:
        diff = [j for j in range(D) if A[j] != B[j]]
        keys = sorted(diff, key=lambda j: (draw(seed, k, g, P_GA_XO, j >> 2, 1)[j & 3], j))
        swap = set(keys[:len(diff) // 2])
        c1 = np.array([B[j] if j in swap else A[j] for j in range(D)], dtype=A.dtype)
        c2 = np.array([A[j] if j in swap else B[j] for j in range(D)], dtype=A.dtype)
        return c1, c2
    raise ValueError("unknown GA crossover")


def ga_crossover(space: core.Space, st: GAState, seed: int, beta_b: int,
                 table: Optional[List[int]] = None, method: int = GA_SINGLE_POINT) -> np.ndarray:
    """Rank selection of two parents per pair and crossover (Section IV-D): every child before
    Alg. 3's repair and the mutation (children 2k and 2k+1 are pair k's)."""
    P, D, g = len(st.pos), space.D, st.gen
    order = sorted(range(P), key=lambda i: (float(st.f[i]), int(st.pos[i])))
    table = table or beta_rank_table(P, beta_b)
    rows = space.vrows[st.pos]
    children = np.zeros((P, D), dtype=np.int32)
    for k in range((P + 1) // 2):
        o = draw(seed, k, g, P_GA_SEL)
        A = rows[order[rank_from_draw(table, o[0])]]
        B = rows[order[rank_from_draw(table, o[1])]]
        c1, c2 = ga_cross_pair(A, B, seed, k, g, o, method)
        children[2 * k] = c1
        if 2 * k + 1 < P:
            children[2 * k + 1] = c2
    return children


def ga_step(space: core.Space, obj: np.ndarray, st: GAState, seed: int, mutation_chance: int,
            beta_b: int, table: Optional[List[int]] = None, method: int = GA_SINGLE_POINT) -> GAState:
    P, g = len(st.pos), st.gen
    children = ga_crossover(space, st, seed, beta_b, table, method)
    # Alg. 3: invalid children become a random member of the first non-empty neighbour set
    children = space.repair(children, core.TIER_RANDOM, key=seed, gen=g)
    # Mutation (after repair): with chance 1/mutation_chance, a random valid Hamming neighbour
    thresh = (1 << 32) // mutation_chance
    mut = [i for i in range(P) if draw(seed, i, g, P_GA_MUT)[0] < thresh]
    if mut:
        mutated = space.repair(children[mut], core.HAM1_RANDOM, who=np.array(mut), key=seed, gen=g)
        children[mut] = mutated
    pos = space.pos(space.encode(children))
    f = obj[pos].astype(np.float32)
    best = (float(st.best_f), st.best_pos)
    for i in range(P):
        best = _lexmin(best, (float(f[i]), int(pos[i])))
    return GAState(pos, f, np.float32(best[0]), int(best[1]), g + 1, evaluated=pos.copy())


def ga_children(space: core.Space, obj: np.ndarray, st: GAState, seed: int, mutation_chance: int, beta_b: int,
                indices, table: Optional[List[int]] = None, method: int = GA_SINGLE_POINT) -> np.ndarray:
    """Final rows of selected children of generation st.gen (same definition as ga_step).

    Lets a test check a sample of a large population without repairing all of it.
    """
    g = st.gen
    idx = np.asarray(indices, dtype=np.int64)
    kids = ga_crossover(space, st, seed, beta_b, table, method)[idx]
    kids = space.repair(kids, core.TIER_RANDOM, who=idx, key=seed, gen=g)
    thresh = (1 << 32) // mutation_chance
    mut = [n for n, i in enumerate(idx) if draw(seed, int(i), g, P_GA_MUT)[0] < thresh]
    if mut:
        kids[mut] = space.repair(kids[mut], core.HAM1_RANDOM, who=idx[mut], key=seed, gen=g)
    return kids


# ---------------------------------------------------------------------------
# Firefly Algorithm (Section IV-C, last paragraph; Table IV hyperparameters)
# ---------------------------------------------------------------------------

FF_EXP_BITS = 21            # exponents x (Q16.16) below 2^21, i.e. below 32; e^-32 < 2^-32 rounds to 0


def ff_exp_table() -> List[int]:
    """T[b] = e^(-2^(b-16)) in Q0.32, rounded half up, b = 0..20, from 60-digit decimal arithmetic."""
    import decimal
    ctx = decimal.Context(prec=60)
    out = []
    for b in range(FF_EXP_BITS):
        v = ctx.exp(ctx.minus(decimal.Decimal(2) ** (b - 16))) * (decimal.Decimal(2) ** 32)
        out.append(int((v + decimal.Decimal("0.5")).to_integral_value(rounding=decimal.ROUND_FLOOR)))
    return out


_FF_T = None


def ff_exp_q32(x_q16: int) -> int:
    """e^(-x) for x = x_q16 / 2^16 >= 0, in Q0.32 (2^32 is 1.0).

    e^-(sum of the set bits of x) is the product of e^-(2^(b-16)) over the set
    bits b; the product runs over ascending b, each step rounded half up to
    Q0.32.  Every step adds at most half a unit, the table another half per
    factor, so the result is within 21 units of 2^-32 of the exact value.
    """
    global _FF_T
    if _FF_T is None:
        _FF_T = ff_exp_table()
    x = int(x_q16)
    if x < 0:
        raise ValueError("exponent must be non-negative")
    if x >> FF_EXP_BITS:
        return 0
    a = 1 << 32
    for b in range(FF_EXP_BITS):
        if (x >> b) & 1:
            a = (a * _FF_T[b] + (1 << 31)) >> 32
    return a


@dataclasses.dataclass
class FFState:
    X: np.ndarray              # P x D positions, Q16.16 index units (PSO's mapping)
    f: np.ndarray              # brightness: objective of each firefly's last evaluation (lower = brighter)
    pos: np.ndarray            # valid-list position that evaluation used
    best_f: float
    best_pos: int
    gen: int = 0
    evaluated: Optional[np.ndarray] = None   # positions the last step evaluated (= pos)


def ff_init(space, obj, P, seed) -> FFState:
    pos = init_positions(space, P, seed, 0)
    X = centre_q16(space.vrows[pos])
    f = obj[pos].astype(np.float32)
    b = min(zip(f.tolist(), pos.tolist()))
    return FFState(X, f, pos.copy(), np.float32(b[0]), int(b[1]), evaluated=pos.copy())


def ff_move(space: core.Space, st: FFState, seed: int, B0_q16: int, gamma_q16: int, alpha_q16: int) -> np.ndarray:
    """Every firefly's new position (before Alg. 2's evaluation).

    For firefly i and each j (ascending) with f_j < f_i at the start of the
    generation: r^2 = sum_d ((X_j,d - x_d) / (M 2^16))^2 in [0,1]^N units
    (x is i's position so far), beta = B0 e^(-gamma r^2), and per dimension
    x_d += beta (X_j,d - x_d) + alpha (u - 1/2) M, with u uniform in [0, 1)
    (a Philox draw at (i, generation, FF_NOISE | d/4, j), word d%4, top 16
    bits), then x_d is clamped to [0, M 2^16 - 1] as in PSO.  Fixed point:
    r^2 in Q16.16 is floor(floor(S / 2^16) / M^2) with S the integer sum of
    squares, gamma r^2 is floor(gamma_q16 r2_q16 / 2^16), beta_q16 is
    B0_q16 e_q32 / 2^32 rounded half up, the attraction floor(beta_q16 dX / 2^16)
    and the random step floor(alpha_q16 M (u_16 - 2^15) / 2^16).
    """
    P, D, g = st.X.shape[0], space.D, st.gen
    M = int(space.radices.max())
    hi, mm = M * 65536 - 1, M * M
    Xn = st.X.copy()
    for i in range(P):
        x = [int(v) for v in st.X[i]]
        for j in range(P):
            if not (st.f[j] < st.f[i]):
                continue
            xj = [int(v) for v in st.X[j]]
            S = sum((xj[d] - x[d]) ** 2 for d in range(D))
            r2 = (S >> 16) // mm
            beta = (B0_q16 * ff_exp_q32((gamma_q16 * r2) >> 16) + (1 << 31)) >> 32
            for d in range(D):
                u = draw(seed, i, g, P_FF_NOISE, d >> 2, j)[d & 3]
                noise = (alpha_q16 * M * ((u >> 16) - 32768)) >> 16
                x[d] = min(max(x[d] + ((beta * (xj[d] - x[d])) >> 16) + noise, 0), hi)
        Xn[i] = x
    return Xn


def ff_step(space: core.Space, obj: np.ndarray, st: FFState, seed: int, B0_q16: int, gamma_q16: int,
            alpha_q16: int) -> FFState:
    P, g = st.X.shape[0], st.gen
    Xn = ff_move(space, st, seed, B0_q16, gamma_q16, alpha_q16)
    snapped = np.minimum(Xn >> 16, space.radices.astype(np.int64) - 1).astype(np.int32)
    # evaluation through Alg. 2 (as PSO): the nearest member of the first non-empty neighbour set
    ev = space.repair(snapped, core.TIER_EUCLID, pos_q16=Xn)
    epos = space.pos(space.encode(ev))
    f = obj[epos].astype(np.float32)
    best = (float(st.best_f), st.best_pos)
    for i in range(P):
        best = _lexmin(best, (float(f[i]), int(epos[i])))
    return FFState(Xn, f, epos.astype(np.int64), np.float32(best[0]), int(best[1]), g + 1,
                   evaluated=epos.astype(np.int64))


# ---------------------------------------------------------------------------
# dispatch on an optimiser description (algo 0 DE, 1 PSO, 2 GA, 3 Firefly and its hyperparameters)
# ---------------------------------------------------------------------------

def init_run(space, obj, opt):
    if getattr(opt, "unaware", 0):
        f = {0: u_init, 1: upso_init, 2: u_init, 3: uff_init}[opt.algo]
    else:
        f = {0: de_init, 1: pso_init, 2: ga_init, 3: ff_init}[opt.algo]
    return f(space, obj, opt.pop_size, opt.seed)


def step_run(space, obj, st, opt):
    if getattr(opt, "unaware", 0):
        if opt.algo == 0:
            return ude_step(space, obj, st, opt.seed, opt.F_q16, opt.CR_q32, int(opt.de_method),
                            int(getattr(opt, "de_crossover", DE_BIN)))
        if opt.algo == 1:
            return upso_step(space, obj, st, opt.seed, opt.w_q16, opt.c1_q16, opt.c2_q16)
        if opt.algo == 2:
            return uga_step(space, obj, st, opt.seed, opt.mutation_chance, opt.beta_b,
                            int(getattr(opt, "ga_crossover", GA_SINGLE_POINT)))
        return uff_step(space, obj, st, opt.seed, opt.ff_B0_q16, opt.ff_gamma_q16, opt.ff_alpha_q16)
    if opt.algo == 0:
        return de_step(space, obj, st, opt.seed, opt.F_q16, opt.CR_q32, int(opt.de_method),
                       int(getattr(opt, "de_crossover", DE_BIN)))
    if opt.algo == 1:
        return pso_step(space, obj, st, opt.seed, opt.w_q16, opt.c1_q16, opt.c2_q16)
    if opt.algo == 2:
        return ga_step(space, obj, st, opt.seed, opt.mutation_chance, opt.beta_b,
                       method=int(getattr(opt, "ga_crossover", GA_SINGLE_POINT)))
    return ff_step(space, obj, st, opt.seed, opt.ff_B0_q16, opt.ff_gamma_q16, opt.ff_alpha_q16)


# ---------------------------------------------------------------------------
# Non-constraint-aware variants (Section IV-B, last sentence; Section IV-C, last sentence):
# a random initial population over the whole Cartesian space (coordinates uniform in PSO's
# [0,1]^N for PSO and Firefly), no repair, and one static penalty for invalid configurations
# (+infinity: the objective is minimised).  DE/GA members are digit rows; a member's position
# is its place in the valid list or NONE.
# ---------------------------------------------------------------------------

NONE = 0xFFFFFFFF


def evaluate(space: core.Space, obj: np.ndarray, rows: np.ndarray):
    """(positions, objective) of configurations: NONE and +inf for the invalid ones."""
    rows = np.asarray(rows, dtype=np.int32).reshape(-1, space.D)
    ok = space.valid_rows(rows) if len(rows) else np.zeros(0, dtype=bool)
    pos = np.full(len(rows), NONE, dtype=np.int64)
    f = np.full(len(rows), np.inf, dtype=np.float32)
    if ok.any():
        p = space.pos(space.encode(rows[ok]))
        pos[ok] = p
        f[ok] = obj[p]
    return pos, f


def random_rows(space: core.Space, P: int, seed: int, tag: int) -> np.ndarray:
    """Member i, digit j: uniform in [0, r_j) from word j%4 of draw (i, tag, INIT | 1 + j/4)."""
    rows = np.zeros((P, space.D), dtype=np.int32)
    for i in range(P):
        for j in range(space.D):
            rows[i, j] = uniform_below(draw(seed, i, tag, P_INIT, 1 + (j >> 2))[j & 3], int(space.radices[j]))
    return rows


def random_coords(space: core.Space, P: int, seed: int) -> np.ndarray:
    """Particle i, coordinate j: uniform in [0, M 2^16) (PSO's [0,1]^N in index units), same draws."""
    M = int(space.radices.max())
    X = np.zeros((P, space.D), dtype=np.int64)
    for i in range(P):
        for j in range(space.D):
            X[i, j] = uniform_below(draw(seed, i, 0, P_INIT, 1 + (j >> 2))[j & 3], M * 65536)
    return X


def _best(best, f, pos):
    for i in range(len(f)):
        best = _lexmin(best, (float(f[i]), int(pos[i])))
    return best


@dataclasses.dataclass
class UState:
    rows: np.ndarray           # DE / GA members as digit rows
    pos: np.ndarray            # valid-list positions (NONE for invalid members)
    f: np.ndarray              # objective (+inf for invalid members)
    best_f: float
    best_pos: int
    gen: int = 0
    reinits: int = 0
    evaluated: Optional[np.ndarray] = None   # positions the last step evaluated (NONE if invalid)


def u_init(space, obj, P, seed) -> UState:
    rows = random_rows(space, P, seed, 0)
    pos, f = evaluate(space, obj, rows)
    b = _best((np.inf, NONE), f, pos)
    return UState(rows, pos, f, np.float32(b[0]), int(b[1]), evaluated=pos.copy())


def _pop_best(f) -> int:
    """The population's best member: lowest (objective, member index)."""
    return int(min(range(len(f)), key=lambda i: (float(f[i]), i)))


def ude_trials(space: core.Space, st: UState, seed: int, F_q16: int, CR_q32: int, method: int,
               crossover: int = DE_BIN) -> np.ndarray:
    """Non-aware DE trials: the operators of de_trials on the member rows, with "best" the
    population's best member (lowest objective, then index)."""
    P, D, g = len(st.pos), space.D, st.gen
    k = 5 if method in (DE_RAND2, DE_BEST2) else 3
    X = st.rows
    best_row = X[_pop_best(st.f)]
    trials = np.zeros((P, D), dtype=np.int32)
    for i in range(P):
        r = de_picks(seed, i, g, P, k)
        j_rand = uniform_below(draw(seed, i, g, P_DE_PICK)[3], D)
        if crossover == DE_EXP:
            run = 1
            while run < D and draw(seed, i, g, P_DE_CR, run >> 2)[run & 3] < CR_q32:
                run += 1
        for j in range(D):
            base, diff = de_mutant_terms(method, i, r, X, best_row, j)
            num = base * 65536 + F_q16 * diff + 32768
            m = min(max(num // 65536, 0), int(space.radices[j]) - 1)
            if crossover == DE_EXP:
                take = (j - j_rand) % D < run
            else:
                take = draw(seed, i, g, P_DE_CR, j >> 2)[j & 3] < CR_q32 or j == j_rand
            trials[i, j] = m if take else X[i, j]
    return trials


def ude_step(space: core.Space, obj: np.ndarray, st: UState, seed: int, F_q16: int, CR_q32: int,
             method: int = DE_BEST1, crossover: int = DE_BIN) -> UState:
    """Non-aware DE: the trials are evaluated as they are (no repair); u_i replaces x_i when
    f(u_i) <= f(x_i) and u_i is not in X (by configuration), the lowest index winning equal
    trials; a generation without replacement reinitialises randomly."""
    P, g = len(st.pos), st.gen
    trials = ude_trials(space, st, seed, F_q16, CR_q32, method, crossover)
    upos, fu = evaluate(space, obj, trials)
    uL = space.encode(trials)
    members = set(space.encode(st.rows).tolist())
    taken = set()
    rows, pos, f = st.rows.copy(), st.pos.copy(), st.f.copy()
    accepted = 0
    for i in range(P):
        if fu[i] <= st.f[i] and int(uL[i]) not in members and int(uL[i]) not in taken:
            taken.add(int(uL[i]))
            rows[i], pos[i], f[i] = trials[i], upos[i], fu[i]
            accepted += 1
    best = _best((float(st.best_f), st.best_pos), f, pos)
    reinits = st.reinits
    if accepted == 0:
        rows = random_rows(space, P, seed, g + 1)
        pos, f = evaluate(space, obj, rows)
        best = _best(best, f, pos)
        reinits += 1
    return UState(rows, pos, f, np.float32(best[0]), int(best[1]), g + 1, reinits, evaluated=upos.copy())


def uga_step(space: core.Space, obj: np.ndarray, st: UState, seed: int, mutation_chance: int, beta_b: int,
             method: int = GA_SINGLE_POINT) -> UState:
    """Non-aware GA: rank selection over the members sorted by (objective, index), crossover,
    no repair, and with chance 1/mutation_chance one parameter (word 1 of the mutation draw)
    set to another of its values (word 2), valid or not."""
    P, D, g = len(st.pos), space.D, st.gen
    order = sorted(range(P), key=lambda i: (float(st.f[i]), i))
    table = beta_rank_table(P, beta_b)
    kids = np.zeros((P, D), dtype=np.int32)
    for k in range((P + 1) // 2):
        o = draw(seed, k, g, P_GA_SEL)
        A = st.rows[order[rank_from_draw(table, o[0])]]
        B = st.rows[order[rank_from_draw(table, o[1])]]
        c1, c2 = ga_cross_pair(A, B, seed, k, g, o, method)
        kids[2 * k] = c1
        if 2 * k + 1 < P:
            kids[2 * k + 1] = c2
    thresh = (1 << 32) // mutation_chance
    for i in range(P):
        o = draw(seed, i, g, P_GA_MUT)
        if o[0] < thresh:
            j = uniform_below(o[1], D)
            r = int(space.radices[j])
            if r > 1:
                v = uniform_below(o[2], r - 1)
                kids[i, j] = v + 1 if v >= kids[i, j] else v
    pos, f = evaluate(space, obj, kids)
    best = _best((float(st.best_f), st.best_pos), f, pos)
    return UState(kids, pos, f, np.float32(best[0]), int(best[1]), g + 1, evaluated=pos.copy())


def upso_init(space, obj, P, seed) -> PSOState:
    X = random_coords(space, P, seed)
    snapped = np.minimum(X >> 16, space.radices.astype(np.int64) - 1)
    pos, f = evaluate(space, obj, snapped)
    return PSOState(X.copy(), np.zeros_like(X), X.copy(), f.copy(), pos.copy(), _gbest(f), evaluated=pos.copy())


def upso_step(space: core.Space, obj: np.ndarray, st: PSOState, seed: int, w_q16: int, c1_q16: int,
              c2_q16: int) -> PSOState:
    """Non-aware PSO: the snapped position is evaluated as it is (static penalty if invalid)."""
    X, V, snapped = pso_move(space, st, seed, w_q16, c1_q16, c2_q16)
    epos, f = evaluate(space, obj, snapped)
    PB, f_pb, pb_pos = st.PB.copy(), st.f_pb.copy(), st.pb_pos.copy()
    for i in range(X.shape[0]):
        if f[i] < f_pb[i]:
            PB[i], f_pb[i], pb_pos[i] = X[i], f[i], epos[i]
    return PSOState(X, V, PB, f_pb, pb_pos, _gbest(f_pb), st.gen + 1, evaluated=epos.copy())


def uff_init(space, obj, P, seed) -> FFState:
    X = random_coords(space, P, seed)
    snapped = np.minimum(X >> 16, space.radices.astype(np.int64) - 1)
    pos, f = evaluate(space, obj, snapped)
    b = _best((np.inf, NONE), f, pos)
    return FFState(X, f, pos, np.float32(b[0]), int(b[1]), evaluated=pos.copy())


def uff_step(space: core.Space, obj: np.ndarray, st: FFState, seed: int, B0_q16: int, gamma_q16: int,
             alpha_q16: int) -> FFState:
    """Non-aware Firefly: moves as the aware one, the snapped position evaluated as it is."""
    Xn = ff_move(space, st, seed, B0_q16, gamma_q16, alpha_q16)
    snapped = np.minimum(Xn >> 16, space.radices.astype(np.int64) - 1)
    pos, f = evaluate(space, obj, snapped)
    best = _best((float(st.best_f), st.best_pos), f, pos)
    return FFState(Xn, f, pos, np.float32(best[0]), int(best[1]), st.gen + 1, evaluated=pos.copy())
