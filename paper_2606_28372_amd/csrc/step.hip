// Constraint-aware population steps on the GPU, for any number of runs per launch.
//
//   DE  (Alg. 1, Section IV-B): best1bin/rand1bin mutation on value indices in
//       Q16.16 (round half up, clip), binomial crossover with j_rand, repair by
//       index distance, greedy selection requiring u not in X, reinitialisation
//       after a generation in which nothing changed.
//   PSO (Section IV-C): positions in [0,1]^N scaled to index units (centre of
//       value k at k + 1/2, the largest domain spans [0, M)), inertia /
//       cognitive / social update in Q16.16, snap to the nearest value,
//       evaluation through Alg. 2's repair without moving the particle,
//       personal and global best.
//   GA  (Section IV-D): population sorted by objective, Beta(1, b) rank
//       selection, single-point crossover, Alg. 3 repair, then mutation to a
//       random valid Hamming neighbour with chance 1/mutation_chance.
//   Firefly (Section IV-C, last paragraph; Table IV): PSO's sampling, mapping
//       and Alg. 2 evaluation; each firefly moves towards every firefly that
//       was brighter at the start of the generation (ascending index) by
//       B0 exp(-gamma r^2) of the way plus a uniform step of width alpha per
//       dimension, all in Q16.16 with a Q0.32 exponential.
//   Non-constraint-aware variants (Sections IV-B and IV-C, last sentences): a
//       random initial sample over the whole Cartesian space, no repair, and
//       +infinity as the objective of an invalid configuration.  DE and GA
//       members are then digit rows (they may be invalid), DE's "best" is the
//       population's best member, GA ranks by (objective, member index) and
//       mutates one parameter to another of its values.
//
// One generation of a batch of runs is: sort (GA runs, one block each) ->
// propose (one thread per individual of every run) -> repair passes (shared
// kernels over the runs' repair sets) -> select (one block per run).  The
// generation number lives on the device and every random draw is a Philox
// block at a counter (individual, generation, purpose | sub-index), so a step
// is a pure function of the state; the same sequence is captured once into a
// hipGraph and replayed for every generation.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>

#include "ct_host.h"
#include "repair_plan.h"

namespace {

constexpr int kBlock = 256;
constexpr int kSelBlock = 1024;
constexpr uint32_t kGaMaxSort = 8192;

__device__ __forceinline__ uint32_t ford(float f) {
    uint32_t b = __float_as_uint(f);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ __forceinline__ uint64_t best_key(float f, uint32_t pos) { return ((uint64_t)ford(f) << 32) | pos; }

// floor(u * n / 2^32) for a 64-bit n
__device__ __forceinline__ uint64_t below64(uint32_t u, uint64_t n) {
    return (uint64_t)u * (n >> 32) + (((uint64_t)u * (uint32_t)n) >> 32);
}

// member i of the stratified initial sample (stratum [i n / P, (i+1) n / P) of the valid list)
__device__ __forceinline__ uint32_t init_pos(const PopDev& p, uint32_t i, uint32_t tag) {
    const uint64_t n = p.n_valid;
    const uint64_t lo = (uint64_t)i * n / p.P, hi = (uint64_t)(i + 1) * n / p.P;
    U4 o = ct_philox(p.seed, i, tag, (uint32_t)PUR_INIT << 24, 0);
    return (uint32_t)(lo + below64(o.x, hi - lo));
}

__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t v, int m) {
    uint32_t lo = __shfl_xor((uint32_t)v, m, 64), hi = __shfl_xor((uint32_t)(v >> 32), m, 64);
    return ((uint64_t)hi << 32) | lo;
}

// a lane's value from another lane of its row through a DPP permutation
template <int CTRL>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ uint64_t dpp_u64(uint64_t v) {
    return ((uint64_t)dpp_u32<CTRL>((uint32_t)(v >> 32)) << 32) | dpp_u32<CTRL>((uint32_t)v);
}

// Wave reductions through DPP (every lane active): within each row of 16 lanes the two quad swaps
// and the half-row and row mirrors combine disjoint sets of lanes, then row 1 takes row 0's partial
// and row 3 row 2's (lane 15 broadcast to the next row), row 3 takes row 1's (lane 31 broadcast to
// rows 2 and 3), and lane 63 holds the wave's result.  A shuffle through LDS would be one dependent
// LDS round trip per step.
template <int CTRL, int ROWS>
__device__ __forceinline__ uint32_t dpp_rows_u32(uint32_t old, uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)v, CTRL, ROWS, 0xF, false);
}
__device__ __forceinline__ uint64_t wave_min_dpp(uint64_t v) {
    auto step = [](uint64_t x, uint64_t w) { return w < x ? w : x; };
    v = step(v, dpp_u64<0xB1>(v));
    v = step(v, dpp_u64<0x4E>(v));
    v = step(v, dpp_u64<0x141>(v));
    v = step(v, dpp_u64<0x140>(v));
    // rows outside the broadcast's row mask keep their own value
    v = step(v, ((uint64_t)dpp_rows_u32<0x142, 0xA>((uint32_t)(v >> 32), (uint32_t)(v >> 32)) << 32) |
                    dpp_rows_u32<0x142, 0xA>((uint32_t)v, (uint32_t)v));
    v = step(v, ((uint64_t)dpp_rows_u32<0x143, 0xC>((uint32_t)(v >> 32), (uint32_t)(v >> 32)) << 32) |
                    dpp_rows_u32<0x143, 0xC>((uint32_t)v, (uint32_t)v));
    return ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), 63) << 32) |
           (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, 63);
}
__device__ __forceinline__ uint32_t wave_sum_dpp(uint32_t v) {
    v += dpp_u32<0xB1>(v);
    v += dpp_u32<0x4E>(v);
    v += dpp_u32<0x141>(v);
    v += dpp_u32<0x140>(v);
    // rows outside the broadcast's row mask add 0
    v += dpp_rows_u32<0x142, 0xA>(0u, v);
    v += dpp_rows_u32<0x143, 0xC>(0u, v);
    return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

// minimum over the block (all threads get the result; every thread of the block calls it)
__device__ uint64_t block_min_u64(uint64_t v) {
    __shared__ uint64_t part[kSelBlock / 64];
    v = wave_min_dpp(v);
    __syncthreads();
    if ((threadIdx.x & 63u) == 0) part[threadIdx.x >> 6] = v;
    __syncthreads();
    uint64_t r = ~0ull;
    for (uint32_t k = 0; k < blockDim.x / 64; ++k) r = part[k] < r ? part[k] : r;
    __syncthreads();
    return r;
}

__device__ uint32_t block_sum_u32(uint32_t v) {
    __shared__ uint32_t part[kSelBlock / 64];
    v = wave_sum_dpp(v);
    __syncthreads();
    if ((threadIdx.x & 63u) == 0) part[threadIdx.x >> 6] = v;
    __syncthreads();
    uint32_t r = 0;
    for (uint32_t k = 0; k < blockDim.x / 64; ++k) r += part[k];
    __syncthreads();
    return r;
}

constexpr uint32_t kNone = 0xFFFFFFFFu;    // position of an invalid configuration

__device__ __forceinline__ float f_inf() { return __int_as_float(0x7F800000); }

// place of linear index L in the valid list, or kNone when L names an invalid configuration
__device__ __forceinline__ uint32_t pos_of(const DevSpace& S, uint64_t L) {
    return bit_valid(S, L) ? (uint32_t)rank_dir(S, L) : kNone;
}

__device__ __forceinline__ float objective_at(const PopDev& p, uint32_t pos) {
    return pos < p.n_valid ? p.obj[pos] : f_inf();
}

// word j%4 of the draw behind coordinate j of a non-aware sample (tag 0: the initial one, g + 1:
// DE's reinitialisation after generation g)
__device__ __forceinline__ uint32_t sample_word(const PopDev& p, uint32_t i, uint32_t tag, uint32_t j) {
    const U4 o = ct_philox(p.seed, i, tag, ((uint32_t)PUR_INIT << 24) | (1u + (j >> 2)), 0);
    const uint32_t t = j & 3u;
    return t == 0 ? o.x : t == 1 ? o.y : t == 2 ? o.z : o.w;
}

// Non-aware DE/GA member i drawn uniformly over the Cartesian space into its row; returns its
// linear index.
__device__ uint64_t sample_member(const PopDev& p, const DevSpace& S, uint32_t i, uint32_t tag) {
    uint8_t* row = p.prow + (uint64_t)i * p.R;
    uint64_t L = 0;
    for (uint32_t j = 0; j < p.R; ++j) {
        uint32_t d = 0;
        if (j < p.D) {
            d = ct_below(sample_word(p, i, tag, j), gld(&S.radix[j]));
            L += (uint64_t)d * gld(&S.stride[j]);
        }
        row[j] = (uint8_t)d;
    }
    return L;
}

// Non-aware PSO / Firefly particle i: coordinates uniform in [0, M 2^16), written to X (and to
// the personal best, with zero velocity, for PSO); returns the linear index of the snapped position.
__device__ uint64_t sample_particle(const PopDev& p, const DevSpace& S, uint32_t i) {
    uint64_t L = 0;
    for (uint32_t j = 0; j < p.D; ++j) {
        const uint32_t x = ct_below(sample_word(p, i, 0, j), p.M * 65536u);
        const uint32_t r = gld(&S.radix[j]), d = x >> 16;
        L += (uint64_t)(d < r ? d : r - 1u) * gld(&S.stride[j]);
        const uint64_t k = (uint64_t)i * p.D + j;
        p.X[k] = (int32_t)x;
        if (p.algo == CT_PSO) {
            p.PB[k] = (int32_t)x;
            p.V[k] = 0;
        }
    }
    return L;
}

// Non-aware DE/GA: copy the proposal row of individual i into its member row.
__device__ __forceinline__ void adopt_row(const PopDev& p, uint32_t i) {
    const uint32_t* src = reinterpret_cast<const uint32_t*>(p.trial + (uint64_t)i * p.R);
    uint32_t* dst = reinterpret_cast<uint32_t*>(p.prow + (uint64_t)i * p.R);
    for (uint32_t k = 0; k < p.R / 4; ++k) dst[k] = src[k];
}

__device__ __forceinline__ uint64_t index_key(float f, uint32_t i) { return ((uint64_t)ford(f) << 32) | i; }

__device__ __forceinline__ void valid_row(const PopDev& p, uint32_t pos, Row& r) {
    row_load(r, p.S->rows + (uint64_t)pos * p.R, p.R);
}

__device__ __forceinline__ uint32_t member_load(const uint32_t* m, uint32_t pos) {
    return (__hip_atomic_load(m + (pos >> 5), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >> (pos & 31u)) & 1u;
}

// largest s with off[s] <= item
__device__ __forceinline__ uint32_t find_run(const uint32_t* off, uint32_t n, uint32_t item) {
    uint32_t lo = 0, hi = n;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (off[mid] <= item) lo = mid; else hi = mid;
    }
    return lo;
}

// ---------------------------------------------------------------------------
// initial population (generation 0), one run
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_init(PopDev p) {
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= p.P) return;
    if (p.unaware) {
        const DevSpace& S = *p.S;
        const bool particle = p.algo == CT_PSO || p.algo == CT_FIREFLY;
        const uint64_t L = particle ? sample_particle(p, S, i) : sample_member(p, S, i, 0);
        const uint32_t pos = pos_of(S, L);
        const float f = objective_at(p, pos);
        p.tpos[i] = pos;                                  // the configurations generation 0 evaluated
        if (p.algo == CT_PSO) {
            p.f_pb[i] = f;
            p.pb_pos[i] = pos;
        } else {
            p.pos[i] = pos;
            p.f[i] = f;
            if (!particle) p.pL[i] = L;
        }
        return;
    }
    uint32_t pos = init_pos(p, i, 0);
    float f = p.obj[pos];
    p.tpos[i] = pos;
    if (p.algo == CT_PSO) {
        Row r;
        valid_row(p, pos, r);
        for (uint32_t j = 0; j < p.D; ++j) {
            int32_t x = (int32_t)((2u * r.digit(j) + 1u) << 15);
            p.X[(uint64_t)i * p.D + j] = x;
            p.PB[(uint64_t)i * p.D + j] = x;
            p.V[(uint64_t)i * p.D + j] = 0;
        }
        p.f_pb[i] = f;
        p.pb_pos[i] = pos;
    } else if (p.algo == CT_FIREFLY) {
        // PSO's mapping: the centre of each value of the valid sample
        Row r;
        valid_row(p, pos, r);
        for (uint32_t j = 0; j < p.D; ++j) p.X[(uint64_t)i * p.D + j] = (int32_t)((2u * r.digit(j) + 1u) << 15);
        p.pos[i] = pos;
        p.f[i] = f;
    } else {
        p.pos[i] = pos;
        p.f[i] = f;
        if (p.algo == CT_DE) atomicOr(&p.member[pos >> 5], 1u << (pos & 31u));
    }
}

__global__ __launch_bounds__(kSelBlock) void k_init_finish(PopDev p) {
    uint64_t m = ~0ull, mi = ~0ull;
    for (uint32_t i = threadIdx.x; i < p.P; i += blockDim.x) {
        m = min(m, p.algo == CT_PSO ? index_key(p.f_pb[i], i) : best_key(p.f[i], p.pos[i]));
        if (p.algo != CT_PSO) mi = min(mi, index_key(p.f[i], i));
    }
    m = block_min_u64(m);
    mi = block_min_u64(mi);
    if (threadIdx.x < 4) p.rcount[threadIdx.x] = 0;
    if (threadIdx.x == 0) {
        p.state[0] = 0;
        p.state[1] = 0;
        p.state[3] = 0;
        if (p.algo == CT_PSO) {
            uint32_t gi = (uint32_t)m;
            p.state[2] = gi;
            *p.best = best_key(p.f_pb[gi], p.pb_pos[gi]);
        } else {
            p.state[2] = p.unaware && p.algo == CT_DE ? (uint32_t)mi : 0u;   // non-aware DE's best member
            *p.best = m;
        }
    }
}

// ---------------------------------------------------------------------------
// propose: one thread per individual of every run
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t pick_excl(uint32_t u, uint32_t n, const uint32_t* ex, uint32_t n_ex) {
    uint32_t k = ct_below(u, n - n_ex);
    for (uint32_t a = 0; a < n_ex; ++a)          // ex is sorted ascending
        if (k >= ex[a]) ++k;
    return k;
}

__device__ __forceinline__ void sort3(uint32_t* e, uint32_t n) {
    for (uint32_t a = 1; a < n; ++a)
        for (uint32_t b = a; b > 0 && e[b - 1] > e[b]; --b) {
            uint32_t t = e[b]; e[b] = e[b - 1]; e[b - 1] = t;
        }
}

// ---------------------------------------------------------------------------
// One group of G lanes per individual (G = 4 or 16), lane s owning digits s, s + G, s + 2G, ...:
// the digits of a proposal are independent given the individual's shared draws, so the per-digit
// work (a Philox block per PSO dimension, the DE mixing, the GA crossover) runs side by side
// instead of one digit after another in a single thread.  Words are assembled with quad
// shuffles, the linear index and the rank with group reductions.  Small batches take G = 16
// (latency: one digit or two per lane); large ones G = 4, since every lane of a group repeats
// the individual's shared draws and the device is then busy with other individuals anyway.
// ---------------------------------------------------------------------------
constexpr uint32_t kWideGroupMax = 16384;   // individuals up to which a group has 16 lanes

// Group reductions through DPP row permutations (no LDS round trip): the two quad swaps combine
// the four lanes of a quad, then (16-lane groups) the half-row mirror pairs each quad with the
// other quad of its half and the row mirror each half with the other half, so every step adds
// disjoint sets of lanes.
template <uint32_t G>
__device__ __forceinline__ uint32_t grp_or4(uint32_t v) {
    v |= dpp_u32<0xB1>(v);        // quad_perm [1, 0, 3, 2]
    v |= dpp_u32<0x4E>(v);        // quad_perm [2, 3, 0, 1]
    return v;
}
template <uint32_t G>
__device__ __forceinline__ uint64_t grp_sum64(uint64_t v) {
    static_assert(G == 4 || G == 16, "groups of 4 or 16 lanes");
    v += dpp_u64<0xB1>(v);
    v += dpp_u64<0x4E>(v);
    if constexpr (G == 16) {
        v += dpp_u64<0x141>(v);   // row_half_mirror
        v += dpp_u64<0x140>(v);   // row_mirror
    }
    return v;
}

__device__ __forceinline__ uint32_t row_digit(const DevSpace& S, uint32_t pos, uint32_t R, uint32_t j) {
    return gld(S.rows + (uint64_t)pos * R + j);
}

// digit j of member m: its row for the non-aware variant (members may be invalid), else its valid
// configuration
__device__ __forceinline__ uint32_t member_digit(const PopDev& p, const DevSpace& S, uint32_t m, uint32_t j) {
    return p.unaware ? (uint32_t)gld(p.prow + (uint64_t)m * p.R + j) : row_digit(S, gld(p.pos + m), p.R, j);
}

// digit j of a GA rank-order entry: a member index (non-aware) or a valid-list position
__device__ __forceinline__ uint32_t parent_digit(const PopDev& p, const DevSpace& S, uint32_t e, uint32_t j) {
    return p.unaware ? (uint32_t)gld(p.prow + (uint64_t)e * p.R + j) : row_digit(S, e, p.R, j);
}

__device__ __forceinline__ uint32_t beta_rank(const PopDev& p, uint32_t u) {
    uint32_t lo = 0, hi = p.P - 1;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if ((uint64_t)u < gld(p.beta + mid)) hi = mid; else lo = mid + 1;
    }
    return lo;
}

// What the digits of individual i's proposal share (generation g), drawn once per lane before its
// digits: DE's picks, j_rand, exponential crossover run and best configuration; GA's parents, cut
// points and (non-aware) mutation draw; PSO's global best member.  Every lane of the group draws
// the same (same counters, same values).
struct PropCtx {
    uint32_t r[5];        // DE: distinct members other than i
    uint32_t jr;          // DE: j_rand
    uint32_t run;         // DE exponential crossover: length of the circular run from j_rand
    uint32_t best;        // DE: best member (non-aware) or best configuration's position; PSO: global best
    uint32_t pa, pb;      // GA: the parents (rank-order entries)
    uint32_t lo, hi;      // GA: genes [lo, hi) of the even child come from parent B (one or two cuts)
    U4 mut;               // GA non-aware: the mutation draw
};

__device__ __forceinline__ PropCtx propose_ctx(const PopDev& p, uint32_t i, uint32_t g) {
    PropCtx c{};
    if (p.algo == CT_DE) {
        const uint32_t meth = p.de_method;
        const uint32_t k = (meth == CT_DE_RAND2 || meth == CT_DE_BEST2) ? 5u : 3u;
        const U4 o = ct_philox(p.seed, i, g, (uint32_t)PUR_DE_PICK << 24, 0);
        uint32_t u[5] = {o.x, o.y, o.z, 0u, 0u};
        if (k > 3) {
            const U4 o2 = ct_philox(p.seed, i, g, ((uint32_t)PUR_DE_PICK << 24) | 1u, 0);
            u[3] = o2.x;
            u[4] = o2.y;
        }
        uint32_t ex[6] = {i, 0, 0, 0, 0, 0};
#pragma unroll
        for (uint32_t t = 0; t < 5; ++t) {
            if (t < k) {
                c.r[t] = pick_excl(u[t], p.P, ex, t + 1);
                ex[t + 1] = c.r[t];
                sort3(ex, t + 2);
            }
        }
        c.jr = ct_below(o.w, p.D);
        c.best = p.unaware ? gld(p.state + 2) : (uint32_t)(gld(p.best) & 0xFFFFFFFFu);
        if (p.de_cross == CT_DE_EXP) {
            // the circular run from j_rand continues while successive draws stay below CR
            uint32_t run = 1;
            while (run < p.D) {
                const U4 d = ct_philox(p.seed, i, g, ((uint32_t)PUR_DE_CR << 24) | (run >> 2), 0);
                const uint32_t t = run & 3u;
                const uint32_t cu = t == 0 ? d.x : t == 1 ? d.y : t == 2 ? d.z : d.w;
                if ((uint64_t)cu >= p.CR_q32) break;
                ++run;
            }
            c.run = run;
        }
    } else if (p.algo == CT_PSO) {
        c.best = gld(p.state + 2);
    } else if (p.algo == CT_GA) {
        // child i of pair i/2: the pair's parents and cuts
        const uint32_t k = i >> 1;
        const U4 o = ct_philox(p.seed, k, g, (uint32_t)PUR_GA_SEL << 24, 0);
        c.pa = gld(p.sorted + beta_rank(p, o.x));
        c.pb = gld(p.sorted + beta_rank(p, o.y));
        c.lo = 1u;
        c.hi = p.D;
        if (p.ga_cross == CT_GA_TWO_POINT && p.D >= 3) {
            const uint32_t c1 = 1u + ct_below(o.z, p.D - 1u);
            uint32_t c2 = ct_below(o.w, p.D - 2u);
            if (c2 >= c1 - 1u) ++c2;                 // a distinct second cut
            c2 += 1u;
            c.lo = c1 < c2 ? c1 : c2;
            c.hi = c1 < c2 ? c2 : c1;
        } else if (p.ga_cross != CT_GA_UNIFORM && p.ga_cross != CT_GA_DISRUPTIVE_UNIFORM) {
            c.lo = 1u + ct_below(o.z, p.D - 1u);     // single point: genes from the cut on
        }
        if (p.unaware) c.mut = ct_philox(p.seed, i, g, (uint32_t)PUR_GA_MUT << 24, 0);
    }
    return c;
}

// The new digit j (< D) of individual i of run p in generation g, given its shared draws c.
__device__ __forceinline__ uint32_t propose_digit(const PopDev& p, const DevSpace& S, const PropCtx& c, uint32_t i,
                                                  uint32_t g, uint32_t j) {
    const uint32_t radix = gld(&S.radix[j]);
    if (p.algo == CT_DE) {
        const uint32_t meth = p.de_method;
        // the best configuration so far (non-aware: the population's best member)
        const int64_t best = p.unaware ? member_digit(p, S, c.best, j) : row_digit(S, c.best, p.R, j);
        const int64_t x = member_digit(p, S, i, j);
        const int64_t x1 = member_digit(p, S, c.r[0], j);
        const int64_t x2 = member_digit(p, S, c.r[1], j), x3 = member_digit(p, S, c.r[2], j);
        int64_t base, diff = x2 - x3;
        if (meth == CT_DE_RAND1) base = x1;
        else if (meth == CT_DE_BEST1) base = best;
        else if (meth == CT_DE_CURRENTTOBEST1) { base = x; diff += best - x; }
        else if (meth == CT_DE_RANDTOBEST1) { base = x1; diff += best - x1; }
        else {
            base = meth == CT_DE_RAND2 ? x1 : best;
            diff += (int64_t)member_digit(p, S, c.r[3], j) - (int64_t)member_digit(p, S, c.r[4], j);
        }
        const int64_t num = base * 65536 + (int64_t)p.F_q16 * diff + 32768;
        int64_t m = num >> 16;            // floor
        const int64_t hi = (int64_t)radix - 1;
        m = m < 0 ? 0 : (m > hi ? hi : m);
        bool take;
        if (p.de_cross == CT_DE_EXP) {
            take = (j + p.D - c.jr) % p.D < c.run;
        } else {
            // block j/4 of the crossover draws, draw j%4 of it
            const U4 cr = ct_philox(p.seed, i, g, ((uint32_t)PUR_DE_CR << 24) | (j >> 2), 0);
            const uint32_t t = j & 3u;
            const uint32_t cu = t == 0 ? cr.x : t == 1 ? cr.y : t == 2 ? cr.z : cr.w;
            take = (uint64_t)cu < p.CR_q32 || j == c.jr;
        }
        return take ? (uint32_t)m : (uint32_t)x;
    }
    if (p.algo == CT_FIREFLY) {
        // the position after this generation's moves, snapped to the nearest value
        const uint32_t d = (uint32_t)(gld(p.Xn + (uint64_t)i * p.D + j) >> 16);
        return d < radix ? d : radix - 1u;
    }
    if (p.algo == CT_PSO) {
        const int64_t xmax = (int64_t)p.M * 65536 - 1;
        U4 o = ct_philox(p.seed, i, g, ((uint32_t)PUR_PSO_R << 24) | j, 0);
        const int64_t r1 = o.x >> 16, r2 = o.y >> 16;
        const uint64_t k = (uint64_t)i * p.D + j;
        int64_t x = gld(p.X + k), v = gld(p.V + k);
        const int64_t pb = gld(p.PB + k), gb = gld(p.PB + (uint64_t)c.best * p.D + j);
        v = ((p.w_q16 * v) >> 16) + ((((p.c1_q16 * r1) >> 16) * (pb - x)) >> 16) +
            ((((p.c2_q16 * r2) >> 16) * (gb - x)) >> 16);
        x += v;
        x = x < 0 ? 0 : (x > xmax ? xmax : x);
        p.V[k] = v;
        p.X[k] = (int32_t)x;
        const uint32_t d = (uint32_t)(x >> 16);
        return d < radix ? d : radix - 1u;
    }
    // GA: child i of pair i/2 takes gene j from parent A where the even child does (the odd child
    // is its mirror)
    const uint32_t k = i >> 1;
    bool even_a;
    if (p.ga_cross == CT_GA_UNIFORM) {
        const U4 x = ct_philox(p.seed, k, g, ((uint32_t)PUR_GA_XO << 24) | (j >> 2), 0);
        const uint32_t t = j & 3u;
        even_a = ((t == 0 ? x.x : t == 1 ? x.y : t == 2 ? x.z : x.w) >> 31) == 0u;
    } else if (p.ga_cross == CT_GA_DISRUPTIVE_UNIFORM) {
        // of the genes where the parents differ, the half with the smallest keys come from B
        const uint32_t aj = parent_digit(p, S, c.pa, j), bj = parent_digit(p, S, c.pb, j);
        even_a = true;
        if (aj != bj) {
            const U4 kj4 = ct_philox(p.seed, k, g, ((uint32_t)PUR_GA_XO << 24) | (j >> 2), 1);
            const uint32_t t = j & 3u;
            const uint32_t kj = t == 0 ? kj4.x : t == 1 ? kj4.y : t == 2 ? kj4.z : kj4.w;
            uint32_t n_diff = 0, rank = 0;
            for (uint32_t q = 0; q < p.D; ++q) {
                if (parent_digit(p, S, c.pa, q) == parent_digit(p, S, c.pb, q)) continue;
                ++n_diff;
                const U4 kq4 = ct_philox(p.seed, k, g, ((uint32_t)PUR_GA_XO << 24) | (q >> 2), 1);
                const uint32_t tq = q & 3u;
                const uint32_t kq = tq == 0 ? kq4.x : tq == 1 ? kq4.y : tq == 2 ? kq4.z : kq4.w;
                rank += (kq < kj || (kq == kj && q < j)) ? 1u : 0u;
            }
            even_a = rank >= n_diff / 2;
        }
    } else {
        even_a = j < c.lo || j >= c.hi;             // one cut: hi = D
    }
    const bool from_a = even_a != ((i & 1u) != 0);
    uint32_t d = parent_digit(p, S, from_a ? c.pa : c.pb, j);
    if (p.unaware) {
        // with chance 1/mutation_chance one parameter (word 1) takes another of its values (word 2)
        const U4& m = c.mut;
        if ((uint64_t)m.x < p.mut_thresh && j == ct_below(m.y, p.D) && radix > 1) {
            const uint32_t v = ct_below(m.z, radix - 1u);
            d = v >= d ? v + 1u : v;
        }
    }
    return d;
}

// Proposals of every run, one group of G lanes per individual, each proposal listed for the main
// repair pass (`sets`, one per run in run order) the way the pass's preparation would list it: its
// validity from the bitmask, its position (or insertion point) from the rank directory, its entry
// in the list of candidates to repair.  The repair counters were cleared by the previous
// generation's selection (or at creation), never by a memset node inside a captured graph.
template <uint32_t G>
__global__ __launch_bounds__(kBlock) void k_propose(const PopDev* __restrict__ pops, uint32_t n,
                                                    const uint32_t* __restrict__ ind_off,
                                                    const RepairSet* __restrict__ sets, PlanArgs pa) {
    constexpr uint32_t T = CT_DMAX / G;                 // digit slots per lane
    const uint32_t total = ind_off[n];
    const uint32_t slot = threadIdx.x & (G - 1u);
    const uint32_t groups = gridDim.x * (blockDim.x / G);
    // every lane of a group takes the same individual, so a group is active or idle as a whole
    for (uint32_t item = (blockIdx.x * blockDim.x + threadIdx.x) / G; item < total; item += groups) {
        const uint32_t r = find_run(ind_off, n, item);
        const PopDev& p = pops[r];
        const DevSpace& S = *p.S;
        const RepairSet& J = sets[r];
        const uint32_t i = item - ind_off[r];
        const uint32_t g = gld(p.state);
        const PropCtx ctx = propose_ctx(p, i, g);
        uint32_t d[T];
        bool ok = true;
        uint64_t term = 0;                              // digits past D are 0 and add nothing
#pragma unroll
        for (uint32_t t = 0; t < T; ++t) {
            const uint32_t j = slot + G * t;
            d[t] = 0;
            if (j < p.D) {
                d[t] = propose_digit(p, S, ctx, i, g, j);
                ok &= d[t] < gld(&S.radix[j]);
                term += (uint64_t)d[t] * gld(&S.stride[j]);
            }
        }
        const uint64_t L_in = grp_sum64<G>(term);
        const bool dom = grp_sum64<G>(ok ? 0u : 1u) == 0u;
        const uint64_t L = dom ? L_in : ~0ull;
        // validity, then the rank (the position if valid, else the insertion position the repair
        // scan seeds its bound around) from the words of L's 8-word block up to L's word
        const bool valid = dom && bit_valid(S, L);
        uint32_t cnt = 0;
        uint64_t base = 0;
        if (dom) {
            const uint64_t w = L >> 6;
            for (uint32_t u = slot; u < 8; u += G) {
                const uint64_t q = (w & ~7ull) + u;
                if (q <= w) {
                    const uint64_t word = gld(S.words + q);
                    cnt += (uint32_t)__popcll(q < w ? word : word & ((1ull << (L & 63u)) - 1ull));
                }
            }
            base = gld(S.grp_off + (w >> 6)) + gld(S.dir8 + (w >> 3));
        }
        const uint64_t rank = base + grp_sum64<G>(cnt);
        // word (slot / 4) + (G / 4) t holds digit slot + G t at byte slot % 4
        const uint32_t nw = p.R / 4;
        uint32_t* trial = reinterpret_cast<uint32_t*>(p.trial + (uint64_t)i * p.R);
        uint32_t* out = reinterpret_cast<uint32_t*>(J.out_rows + (uint64_t)i * p.R);
#pragma unroll
        for (uint32_t t = 0; t < T; ++t) {
            const uint32_t word = grp_or4<G>(d[t] << ((slot & 3u) * 8u));
            const uint32_t wi = (slot >> 2) + (G / 4) * t;
            if ((slot & 3u) == 0 && wi < nw) {
                trial[wi] = word;
                out[wi] = word;
            }
        }
        if (slot == 0) {
            if (p.algo == CT_GA) {
                // the non-aware GA mutated in the proposal: the mutation pass skips its children
                const U4 m = ct_philox(p.seed, i, g, (uint32_t)PUR_GA_MUT << 24, 0);
                p.apply[i] = !p.unaware && (uint64_t)m.x < p.mut_thresh;
            }
            if (p.unaware && p.algo == CT_DE) p.tL[i] = L;
            J.out_pos[i] = valid ? (uint32_t)rank : kNone;
            if (!valid && !p.unaware) {
                const uint32_t k = atomicAdd(&J.count[0], 1u);
                J.list[k] = i;
                J.list_ins[k] = dom ? rank : ~0ull;
            }
        }
    }
    plan_if_last(sets, n, pa);                          // the last block plans the main scans
}

void launch_propose(const ct_batch* b, const PlanArgs& pa, hipStream_t st) {
    if (b->total_ind <= kWideGroupMax) {
        const uint32_t g = std::max<uint32_t>(1, std::min<uint32_t>((b->total_ind * 16 + kBlock - 1) / kBlock, 4096));
        hipLaunchKernelGGL(k_propose<16>, dim3(g), dim3(kBlock), 0, st, b->d_pops, b->n, b->d_ind_off, b->passA.d_sets, pa);
    } else {
        const uint32_t g = std::max<uint32_t>(1, std::min<uint32_t>((b->total_ind * 4 + kBlock - 1) / kBlock, 4096));
        hipLaunchKernelGGL(k_propose<4>, dim3(g), dim3(kBlock), 0, st, b->d_pops, b->n, b->d_ind_off, b->passA.d_sets, pa);
    }
}

// ---------------------------------------------------------------------------
// Firefly moves: one wave per firefly, lane d holding coordinate d (D <= 32)
// ---------------------------------------------------------------------------
// e^(-x) for x in Q16.16, in Q0.32: the product of the factors e^(-2^(b-16)) over the set bits b of
// x, ascending, each step rounded half up; x >= 32 gives 0 (e^-32 < 2^-32).
struct FFExp {
    uint64_t t[21];
};

FFExp ff_exp_factors() {
    FFExp e;
    for (int b = 0; b < 21; ++b) e.t[b] = (uint64_t)floorl(expl(-ldexpl(1.0L, b - 16)) * 4294967296.0L + 0.5L);
    return e;
}

__device__ __forceinline__ uint64_t ff_exp(const FFExp& ex, uint64_t x) {
    if (x >> 21) return 0;
    uint64_t a = 1ull << 32;
#pragma unroll
    for (int b = 0; b < 21; ++b)
        if ((x >> b) & 1u) a = (a * ex.t[b] + (1ull << 31)) >> 32;
    return a;
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += shfl_xor_u64(v, o);
    return v;
}

// New positions Xn of every firefly of every Firefly run (ff_off: prefix of their population sizes,
// zero for other runs).  Firefly i reads the positions and brightness at the start of the
// generation (X, f) and keeps its own moving position in its lanes, so fireflies are independent.
__global__ __launch_bounds__(kBlock) void k_ff_move(const PopDev* __restrict__ pops, uint32_t n,
                                                    const uint32_t* __restrict__ ff_off, FFExp ex) {
    const uint32_t total = ff_off[n];
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t waves = gridDim.x * (kBlock / 64);
    for (uint32_t item = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6); item < total; item += waves) {
        const uint32_t r = find_run(ff_off, n, item);
        const PopDev& p = pops[r];
        const uint32_t i = item - ff_off[r];
        const uint32_t D = p.D, P = p.P, g = p.state[0];
        const bool act = lane < D;
        const int64_t M = p.M, xmax = M * 65536 - 1;
        const uint64_t mm = (uint64_t)(M * M);
        int64_t x = act ? p.X[(uint64_t)i * D + lane] : 0;
        const float fi = p.f[i];
        for (uint32_t j = 0; j < P; ++j) {
            if (!(p.f[j] < fi)) continue;                 // only brighter fireflies attract
            const int64_t dx = (act ? (int64_t)p.X[(uint64_t)j * D + lane] : 0) - x;
            // r^2 in [0,1]^N units, Q16.16: the sum of squares over (M 2^16)^2
            const uint64_t r2 = (wave_sum_u64((uint64_t)(dx * dx)) >> 16) / mm;
            const uint64_t e = ff_exp(ex, ((uint64_t)p.ff_gamma * r2) >> 16);
            const int64_t beta = (int64_t)(((uint64_t)p.ff_B0 * e + (1ull << 31)) >> 32);
            const U4 o = ct_philox(p.seed, i, g, ((uint32_t)PUR_FF_NOISE << 24) | (lane >> 2), j);
            const uint32_t t = lane & 3u;
            const uint32_t u = t == 0 ? o.x : t == 1 ? o.y : t == 2 ? o.z : o.w;
            const int64_t noise = (p.ff_alpha * M * ((int64_t)(u >> 16) - 32768)) >> 16;
            const int64_t nx = x + ((beta * dx) >> 16) + noise;
            // lanes past D stay at 0, so they add nothing to the next distance
            x = !act ? 0 : nx < 0 ? 0 : (nx > xmax ? xmax : nx);
        }
        if (act) p.Xn[(uint64_t)i * D + lane] = (int32_t)x;
    }
}

void launch_ff_move(const ct_batch* b, hipStream_t st) {
    if (!b->total_ff) return;
    static const FFExp ex = ff_exp_factors();
    ProfScope ps_("k_ff_move", st);
    const uint32_t g = std::max<uint32_t>(1, std::min<uint32_t>((b->total_ff + kBlock / 64 - 1) / (kBlock / 64), 4096));
    hipLaunchKernelGGL(k_ff_move, dim3(g), dim3(kBlock), 0, st, b->d_pops, b->n, b->d_ff_off, ex);
}

// ---------------------------------------------------------------------------
// GA: sort the population by (objective, position), one block per GA run
// ---------------------------------------------------------------------------
// Returns, in thread 0 when the population fits the block, the smallest key (the rank-0
// individual's); `own`, when given, is the calling thread's individual's key (individual
// threadIdx.x), so it need not be read back from memory.
// GA rank-sort key of member i: (objective, position), or (objective, member index) for the
// non-aware variant, whose members need not have a position; the low word is what the rank order
// holds (a position, or a member index)
__device__ __forceinline__ uint64_t ga_key(const PopDev& p, uint32_t i) {
    return p.unaware ? index_key(p.f[i], i) : best_key(p.f[i], p.pos[i]);
}

__device__ uint64_t ga_sort_block(const PopDev& p, const uint64_t* own = nullptr) {
    __shared__ uint64_t key[kGaMaxSort];
    uint32_t m = 1;
    while (m < p.P) m <<= 1;
    if (m <= blockDim.x) {
        // one key per thread.  Each wave sorts its 64 keys ascending with a bitonic network over
        // cross-lane shuffles; then rounds of pairwise merges double the sorted runs: a key's
        // place in the merged run is its place in its own run plus the number of keys of the
        // other run that go before it (found by binary search in LDS; on equal keys the left
        // run's go first), so each round is one binary search and one barrier, not a series of
        // exchange stages.
        const uint32_t i = threadIdx.x;
        uint64_t v = i < p.P ? (own ? *own : ga_key(p, i)) : ~0ull;
        const uint32_t w = m < 64 ? m : 64;
        for (uint32_t k = 2; k <= w; k <<= 1) {
            for (uint32_t j = k >> 1; j > 0; j >>= 1) {
                const uint64_t o = shfl_xor_u64(v, (int)j);
                const bool up = k == w || (i & k) == 0;       // the last stage sorts every run upward
                const bool keep_min = ((i & j) == 0) == up;
                v = keep_min ? (o < v ? o : v) : (o > v ? o : v);
            }
        }
        uint64_t* src = key;
        uint64_t* dst = key + kSelBlock;
        if (i < m) src[i] = v;
        __syncthreads();
        for (uint32_t L = w; L < m; L <<= 1) {
            if (i < m) {
                const uint32_t base = i & ~(2 * L - 1), r = i & (L - 1);
                const bool left = (i & L) == 0;
                const uint64_t* other = src + base + (left ? L : 0);
                uint32_t lo = 0, hi = L;
                while (lo < hi) {
                    const uint32_t mid = (lo + hi) >> 1;
                    const uint64_t x = other[mid];
                    if (left ? x < v : x <= v) lo = mid + 1; else hi = mid;
                }
                dst[base + r + lo] = v;
            }
            __syncthreads();
            uint64_t* t = src; src = dst; dst = t;
            if (i < m) v = src[i];
        }
        if (i < p.P) p.sorted[i] = (uint32_t)v;
        return v;
    }
    constexpr uint32_t kMaxPerThread = kGaMaxSort / kSelBlock;
    const uint32_t q = m / blockDim.x;                    // keys per thread
    if ((blockDim.x & 63u) == 0 && q <= kMaxPerThread) {
        // More keys than threads: wave w holds keys w*64q + 64r + lane (r < q) in registers, so
        // every stage whose partners lie less than 64 apart pairs lanes of one wave in one
        // register and runs on cross-lane shuffles; only the stages 64 or more apart go through
        // LDS and a barrier (4,096 keys: 21 of 78 stages).  The compare-exchange network is the
        // plain bitonic one, so the order is the same.
        const uint32_t base = (threadIdx.x >> 6) * 64u * q + (threadIdx.x & 63u);
        uint64_t v[kMaxPerThread];
#pragma unroll
        for (uint32_t r = 0; r < kMaxPerThread; ++r) {
            const uint32_t i = base + 64u * r;
            v[r] = r < q && i < p.P ? ga_key(p, i) : ~0ull;
        }
        for (uint32_t k = 2; k <= m; k <<= 1) {
            uint32_t j = k >> 1;
            if (j >= 64) {
#pragma unroll
                for (uint32_t r = 0; r < kMaxPerThread; ++r)
                    if (r < q) key[base + 64u * r] = v[r];
                __syncthreads();
                for (; j >= 64; j >>= 1) {
                    for (uint32_t i = threadIdx.x; i < m; i += blockDim.x) {
                        const uint32_t l = i ^ j;
                        if (l > i) {
                            const bool up = (i & k) == 0;
                            const uint64_t a = key[i], b = key[l];
                            if ((a > b) == up) { key[i] = b; key[l] = a; }
                        }
                    }
                    __syncthreads();
                }
#pragma unroll
                for (uint32_t r = 0; r < kMaxPerThread; ++r)
                    if (r < q) v[r] = key[base + 64u * r];
            }
            for (; j > 0; j >>= 1) {
#pragma unroll
                for (uint32_t r = 0; r < kMaxPerThread; ++r) {
                    if (r < q) {
                        const uint32_t i = base + 64u * r;
                        const uint64_t o = shfl_xor_u64(v[r], (int)j);
                        const bool up = (i & k) == 0;
                        const bool keep_min = ((i & j) == 0) == up;
                        v[r] = keep_min ? (o < v[r] ? o : v[r]) : (o > v[r] ? o : v[r]);
                    }
                }
            }
        }
#pragma unroll
        for (uint32_t r = 0; r < kMaxPerThread; ++r) {
            const uint32_t i = base + 64u * r;
            if (r < q && i < p.P) p.sorted[i] = (uint32_t)v[r];
        }
        return ~0ull;
    }
    for (uint32_t i = threadIdx.x; i < m; i += blockDim.x) key[i] = i < p.P ? ga_key(p, i) : ~0ull;
    __syncthreads();
    for (uint32_t k = 2; k <= m; k <<= 1) {
        for (uint32_t j = k >> 1; j > 0; j >>= 1) {
            for (uint32_t i = threadIdx.x; i < m; i += blockDim.x) {
                const uint32_t l = i ^ j;
                if (l > i) {
                    const bool up = (i & k) == 0;
                    const uint64_t a = key[i], b = key[l];
                    if ((a > b) == up) { key[i] = b; key[l] = a; }
                }
            }
            __syncthreads();
        }
    }
    for (uint32_t i = threadIdx.x; i < p.P; i += blockDim.x) p.sorted[i] = (uint32_t)key[i];
    return ~0ull;
}

// The rank order of a GA run's population (read by the next generation's proposals): sorted at
// creation, after a restore, and by the selection kernel at the end of every generation.
__global__ __launch_bounds__(kSelBlock) void k_ga_sort_one(PopDev p) { (void)ga_sort_block(p); }

// ---------------------------------------------------------------------------
// select: one block per run
// ---------------------------------------------------------------------------
__device__ void de_select(const PopDev& p) {
    const uint32_t g = p.state[0];
    // pre-accept: no worse than the member it would replace and not already in X
    for (uint32_t i = threadIdx.x; i < p.P; i += blockDim.x) {
        const uint32_t t = p.tpos[i];
        const bool pa = t < p.n_valid && p.obj[t] <= p.f[i] && !member_load(p.member, t);
        p.apply[i] = pa ? 1 : 0;
        if (pa) atomicMin(&p.claim[t], i);
    }
    __syncthreads();
    // equal trials: the lowest individual index wins
    uint32_t acc = 0;
    for (uint32_t i = threadIdx.x; i < p.P; i += blockDim.x) {
        if (p.apply[i]) {
            const uint32_t owner = __hip_atomic_load(&p.claim[p.tpos[i]], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (owner == i) { p.apply[i] = 2; ++acc; }
        }
    }
    acc = block_sum_u32(acc);
    for (uint32_t i = threadIdx.x; i < p.P; i += blockDim.x) {
        if (p.apply[i]) atomicExch(&p.claim[p.tpos[i]], 0xFFFFFFFFu);
        if (p.apply[i] == 2) atomicAnd(&p.member[p.pos[i] >> 5], ~(1u << (p.pos[i] & 31u)));
    }
    __syncthreads();
    uint64_t m = ~0ull;
    for (uint32_t i = threadIdx.x; i < p.P; i += blockDim.x) {
        if (p.apply[i] == 2) {
            const uint32_t t = p.tpos[i];
            atomicOr(&p.member[t >> 5], 1u << (t & 31u));
            p.pos[i] = t;
            p.f[i] = p.obj[t];
        }
        m = min(m, best_key(p.f[i], p.pos[i]));
    }
    m = block_min_u64(m);
    if (acc == 0) {
        // the population did not change: reinitialise it from the valid list
        for (uint32_t i = threadIdx.x; i < p.P; i += blockDim.x)
            atomicAnd(&p.member[p.pos[i] >> 5], ~(1u << (p.pos[i] & 31u)));
        __syncthreads();
        uint64_t m2 = ~0ull;
        for (uint32_t i = threadIdx.x; i < p.P; i += blockDim.x) {
            const uint32_t t = init_pos(p, i, g + 1);
            atomicOr(&p.member[t >> 5], 1u << (t & 31u));
            p.pos[i] = t;
            p.f[i] = p.obj[t];
            m2 = min(m2, best_key(p.f[i], t));
        }
        m2 = block_min_u64(m2);
        m = min(m, m2);
    }
    if (threadIdx.x == 0) {
        const uint64_t b = *p.best;
        *p.best = m < b ? m : b;
        p.state[3] = acc;
        if (acc == 0) p.state[1] += 1;
        p.state[0] = g + 1;
    }
}

// Non-aware DE selection (population <= 8,192: at most 8 members per thread, one bit each in
// `pre` and `lost`).  Trial u_i replaces x_i when f(u_i) <= f(x_i) and no member has u_i's
// configuration; of equal trials the lowest index wins.  Both tests compare linear indices,
// member ones and trial ones, chunk by chunk through LDS (P^2 / 1,024 comparisons a thread).
__device__ void de_select_unaware(const PopDev& p) {
    __shared__ uint64_t chunk[kSelBlock];
    const DevSpace& S = *p.S;
    const uint32_t g = p.state[0];
    const uint32_t per = (p.P + blockDim.x - 1) / blockDim.x;
    uint32_t pre = 0, lost = 0;
    for (uint32_t k = 0; k < per; ++k) {
        const uint32_t i = threadIdx.x + k * blockDim.x;
        if (i < p.P && objective_at(p, p.tpos[i]) <= p.f[i]) pre |= 1u << k;
    }
    for (uint32_t c0 = 0; c0 < p.P; c0 += blockDim.x) {
        const uint32_t n = min(blockDim.x, p.P - c0);
        __syncthreads();
        if (threadIdx.x < n) chunk[threadIdx.x] = p.pL[c0 + threadIdx.x];
        __syncthreads();
        for (uint32_t k = 0; k < per; ++k) {
            if (!((pre >> k) & 1u)) continue;
            const uint64_t L = p.tL[threadIdx.x + k * blockDim.x];
            bool hit = false;
            for (uint32_t t = 0; t < n; ++t) hit |= chunk[t] == L;
            if (hit) pre &= ~(1u << k);
        }
    }
    for (uint32_t k = 0; k < per; ++k) {
        const uint32_t i = threadIdx.x + k * blockDim.x;
        if (i < p.P) p.apply[i] = (pre >> k) & 1u;
    }
    for (uint32_t c0 = 0; c0 < p.P; c0 += blockDim.x) {
        const uint32_t n = min(blockDim.x, p.P - c0);
        __syncthreads();
        if (threadIdx.x < n) chunk[threadIdx.x] = p.apply[c0 + threadIdx.x] ? p.tL[c0 + threadIdx.x] : ~0ull;
        __syncthreads();
        for (uint32_t k = 0; k < per; ++k) {
            const uint32_t i = threadIdx.x + k * blockDim.x;
            if (!((pre >> k) & 1u) || c0 >= i) continue;
            const uint64_t L = p.tL[i];
            const uint32_t lim = min(n, i - c0);          // earlier individuals only
            bool hit = false;
            for (uint32_t t = 0; t < lim; ++t) hit |= chunk[t] == L;
            if (hit) lost |= 1u << k;
        }
    }
    const uint32_t acc_bits = pre & ~lost;
    const uint32_t acc = block_sum_u32((uint32_t)__popc(acc_bits));
    uint64_t m = ~0ull, mi = ~0ull;
    for (uint32_t k = 0; k < per; ++k) {
        const uint32_t i = threadIdx.x + k * blockDim.x;
        if (i >= p.P) continue;
        if ((acc_bits >> k) & 1u) {
            adopt_row(p, i);
            p.pL[i] = p.tL[i];
            p.pos[i] = p.tpos[i];
            p.f[i] = objective_at(p, p.tpos[i]);
        }
        m = min(m, best_key(p.f[i], p.pos[i]));
        mi = min(mi, index_key(p.f[i], i));
    }
    m = block_min_u64(m);
    mi = block_min_u64(mi);
    if (acc == 0) {
        // no member replaced: a new random population (tag g + 1)
        uint64_t m2 = ~0ull, mi2 = ~0ull;
        for (uint32_t i = threadIdx.x; i < p.P; i += blockDim.x) {
            const uint64_t L = sample_member(p, S, i, g + 1);
            const uint32_t t = pos_of(S, L);
            p.pL[i] = L;
            p.pos[i] = t;
            p.f[i] = objective_at(p, t);
            m2 = min(m2, best_key(p.f[i], t));
            mi2 = min(mi2, index_key(p.f[i], i));
        }
        m = min(m, block_min_u64(m2));
        mi = block_min_u64(mi2);
    }
    if (threadIdx.x == 0) {
        const uint64_t b = *p.best;
        *p.best = m < b ? m : b;
        p.state[2] = (uint32_t)mi;
        p.state[3] = acc;
        if (acc == 0) p.state[1] += 1;
        p.state[0] = g + 1;
    }
}

__device__ void pso_select(const PopDev& p) {
    const uint32_t g = p.state[0];
    uint64_t m = ~0ull;
    for (uint32_t i = threadIdx.x; i < p.P; i += blockDim.x) {
        const uint32_t t = p.tpos[i];
        const float fv = t < p.n_valid ? p.obj[t] : __int_as_float(0x7F800000);   // +inf: never improves
        if (fv < p.f_pb[i]) {
            for (uint32_t j = 0; j < p.D; ++j) p.PB[(uint64_t)i * p.D + j] = p.X[(uint64_t)i * p.D + j];
            p.f_pb[i] = fv;
            p.pb_pos[i] = t;
        }
        m = min(m, ((uint64_t)ford(p.f_pb[i]) << 32) | i);
    }
    m = block_min_u64(m);
    if (threadIdx.x == 0) {
        const uint32_t gi = (uint32_t)m;
        p.state[2] = gi;
        *p.best = best_key(p.f_pb[gi], p.pb_pos[gi]);
        p.state[0] = g + 1;
    }
}

__device__ void ff_select(const PopDev& p) {
    const uint32_t g = p.state[0];
    uint64_t m = ~0ull;
    for (uint32_t i = threadIdx.x; i < p.P; i += blockDim.x) {
        uint32_t t = p.tpos[i];
        // aware: unreachable, every evaluation goes to a valid configuration; non-aware: +inf
        if (t >= p.n_valid && !p.unaware) t = p.pos[i];
        p.pos[i] = t;
        p.f[i] = objective_at(p, t);
        m = min(m, best_key(p.f[i], t));
        for (uint32_t j = 0; j < p.D; ++j) p.X[(uint64_t)i * p.D + j] = p.Xn[(uint64_t)i * p.D + j];
    }
    m = block_min_u64(m);
    if (threadIdx.x == 0) {
        const uint64_t b = *p.best;
        *p.best = m < b ? m : b;
        p.state[0] = g + 1;
    }
}

// child i becomes member i: its position (non-aware: kNone if invalid, and its row) and objective
__device__ __forceinline__ float ga_adopt(const PopDev& p, uint32_t i) {
    uint32_t t = p.tpos[i];
    if (p.unaware) adopt_row(p, i);
    else if (t >= p.n_valid) t = p.pos[i];             // unreachable: every repaired child is valid
    const float fv = objective_at(p, t);
    p.pos[i] = t;
    p.f[i] = fv;
    return fv;
}

__device__ void ga_select(const PopDev& p) {
    const uint32_t g = p.state[0];
    uint64_t m = ~0ull;
    for (uint32_t i = threadIdx.x; i < p.P; i += blockDim.x) {
        ga_adopt(p, i);
        m = min(m, best_key(p.f[i], p.pos[i]));
    }
    m = block_min_u64(m);
    if (threadIdx.x == 0) {
        const uint64_t b = *p.best;
        *p.best = m < b ? m : b;
        p.state[0] = g + 1;
    }
}

__global__ __launch_bounds__(kSelBlock) void k_select(const PopDev* __restrict__ pops, uint32_t n) {
    const PopDev& p = pops[blockIdx.x];
    if (p.algo == CT_DE && p.unaware) de_select_unaware(p);
    else if (p.algo == CT_DE) de_select(p);
    else if (p.algo == CT_PSO) pso_select(p);
    else if (p.algo == CT_FIREFLY) ff_select(p);
    else if (p.P <= blockDim.x) {
        // one child per thread: its key goes to the rank sort (the next generation's rank order)
        // in a register, and the sorted order's first key is the generation's best
        const uint32_t g = p.state[0];
        uint64_t k = ~0ull, bk = ~0ull;
        const uint32_t i = threadIdx.x;
        if (i < p.P) {
            const float fv = ga_adopt(p, i);
            bk = best_key(fv, p.pos[i]);
            k = p.unaware ? index_key(fv, i) : bk;
        }
        uint64_t m = ga_sort_block(p, &k);
        if (p.unaware) m = block_min_u64(bk);            // the sort keys hold member indices
        if (threadIdx.x == 0) {
            const uint64_t b = *p.best;
            *p.best = m < b ? m : b;
            p.state[0] = g + 1;
        }
    } else {
        ga_select(p);
        __syncthreads();
        (void)ga_sort_block(p);                           // the next generation's rank order
    }
    if (threadIdx.x < 4) p.rcount[threadIdx.x] = 0;      // repair counters of the next generation
}

}  // namespace

int pop_init_device(ct_pop* p, hipStream_t st) {
    const PopDev& d = p->dev;
    { ProfScope ps_("k_init", st); hipLaunchKernelGGL(k_init, dim3((d.P + kBlock - 1) / kBlock), dim3(kBlock), 0, st, d); }
    { ProfScope ps_("k_init_finish", st); hipLaunchKernelGGL(k_init_finish, dim3(1), dim3(kSelBlock), 0, st, d); }
    if (d.algo == CT_GA) return pop_sort_device(p, st);
    CT_HIP(hipGetLastError());
    return CT_OK;
}

int pop_sort_device(ct_pop* p, hipStream_t st) {
    if (p->dev.algo != CT_GA) return CT_OK;
    { ProfScope ps_("k_ga_sort", st); hipLaunchKernelGGL(k_ga_sort_one, dim3(1), dim3(kSelBlock), 0, st, p->dev); }
    CT_HIP(hipGetLastError());
    return CT_OK;
}

int batch_generation(ct_batch* b, hipStream_t st) {
    if (b->n == 0) return CT_OK;
    launch_ff_move(b, st);
    {
        ProfScope ps_("k_propose", st);
        launch_propose(b, main_plan(b->passA), st);
    }
    int rc = launch_repair_passes(b->passA, false, st, true, false);
    if (rc) return rc;
    if (b->n_ga) {
        rc = launch_mutation(b->passC, st);
        if (rc) return rc;
    }
    {
        ProfScope ps_("k_select", st);
        hipLaunchKernelGGL(k_select, dim3(b->n), dim3(kSelBlock), 0, st, b->d_pops, b->n);
    }
    CT_HIP(hipGetLastError());
    return CT_OK;
}

namespace {

// Sweep of one tuning generation: the main repair pass reads the proposals and writes only its
// outputs, lists and counters (the counters are cleared first and the scan tally is left alone),
// so it can run once per candidate partitioning with identical results; each candidate's time is
// added to its total over the batch's tuning generations.
int autotune_sweep(ct_batch* b, hipStream_t st) {
    if (b->tune_cand.empty()) {
        std::vector<uint32_t> modes = {kScanSerial, kScanFused};
        if (b->fan.fork) modes.push_back(kScanStreams);
        // item targets up to the slots' limit (large batches split their long scans finely);
        // grids from a quarter of the target to four times it (a fused launch holds the items
        // of several classes)
        for (uint32_t mode : modes)
            for (uint32_t it : {2048u, 4096u, 8192u, 16384u, 32768u})
                for (uint32_t ms : {8u, 16u, 32u, 64u})
                    for (uint32_t gw : {4096u, 8192u, 16384u, 32768u})
                        if (gw <= 4 * it && 4 * gw >= it) b->tune_cand.push_back(RepairTune{it, ms, gw, mode});
        b->tune_ms.assign(b->tune_cand.size(), 0.0);
    }
    const std::vector<RepairTune>& cand = b->tune_cand;
    // The candidates run back to back with one wait at the end, so that each is timed with the
    // launch queue full, as in the generations that follow.  A pass on side streams delays the
    // launches after its join, so each candidate's window holds the tail of the pass before it:
    // candidates are grouped by that setting and every group starts after an untimed pass of
    // its own kind.
    std::vector<hipEvent_t> ev(2 * cand.size(), nullptr);
    int rc = CT_OK;
    for (hipEvent_t& e : ev)
        if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess)
            rc = ct_fail(CT_EDEVICE, "autotune: event create failed");
    prof_suspend(true);
    RepairPasses rp = b->passA;
    for (size_t v = 0; v < cand.size() && !rc; ++v) {
        rp.tune = cand[v];
        if (v == 0 || cand[v].mode != cand[v - 1].mode) rc = launch_repair_passes(rp, true, st, false);
        if (!rc && hipEventRecord(ev[2 * v], st) != hipSuccess) rc = ct_fail(CT_EDEVICE, "autotune: event record failed");
        if (!rc) rc = launch_repair_passes(rp, true, st, false);
        if (!rc && hipEventRecord(ev[2 * v + 1], st) != hipSuccess)
            rc = ct_fail(CT_EDEVICE, "autotune: event record failed");
    }
    if (!rc && hipEventSynchronize(ev.back()) != hipSuccess) rc = ct_fail(CT_EDEVICE, "autotune: event wait failed");
    for (size_t v = 0; v < cand.size() && !rc; ++v) {
        float t = 0;
        if (hipEventElapsedTime(&t, ev[2 * v], ev[2 * v + 1]) != hipSuccess) rc = ct_fail(CT_EDEVICE, "autotune: no timing");
        b->tune_ms[v] += t;
    }
    prof_suspend(false);
    for (hipEvent_t e : ev)
        if (e) (void)hipEventDestroy(e);
    return rc;
}

// Candidate with the lowest sweep total: streams < 0 any, 0 without side streams, 1 with them.
RepairTune sweep_best(const ct_batch* b, int streams) {
    size_t pick = b->tune_cand.size();
    for (size_t v = 0; v < b->tune_cand.size(); ++v)
        if ((streams < 0 || (b->tune_cand[v].mode == kScanStreams) == (streams == 1)) &&
            (pick == b->tune_cand.size() || b->tune_ms[v] < b->tune_ms[pick]))
            pick = v;
    return pick < b->tune_cand.size() ? b->tune_cand[pick] : b->passA.tune;
}

// One generation whose main repair pass is first swept over every candidate partitioning.
int autotune_generation(ct_batch* b, hipStream_t st) {
    launch_ff_move(b, st);
    {
        // the sweep lists and plans again for every candidate
        launch_propose(b, PlanArgs{}, st);
    }
    CT_HIP(hipGetLastError());
    int rc = autotune_sweep(b, st);
    if (rc) return rc;
    b->passA.tune = sweep_best(b, -1);
    // the generation's own pass, counting its scans
    if ((rc = launch_repair_passes(b->passA, true, st, true))) return rc;
    if (b->n_ga && (rc = launch_mutation(b->passC, st))) return rc;
    hipLaunchKernelGGL(k_select, dim3(b->n), dim3(kSelBlock), 0, st, b->d_pops, b->n);
    CT_HIP(hipGetLastError());
    return CT_OK;
}

}  // namespace

int batch_autotune(ct_batch* b, uint32_t n_generations, uint32_t sample_every, hipStream_t st) {
    if (b->n == 0 || n_generations == 0) return CT_OK;
    const uint32_t every = std::max<uint32_t>(sample_every, 1);
    b->tune_cand.clear();
    b->tune_ms.clear();
    // The sweep times the main pass alone on the device, but side streams cost more than that: the
    // host spends longer issuing a generation that forks and joins streams, and the device waits
    // at the joins.  Streams or not is therefore decided on whole generations by the host clock:
    // the generations between sweeps run in blocks of kBlockGens with the best candidate with or
    // without streams so far, alternating, each block between two stream waits; the lower mean
    // block time wins.
    constexpr uint32_t kBlockGens = 4;
    double block_ms[2] = {0, 0};
    uint32_t block_n[2] = {0, 0};
    int rc = CT_OK;
    uint32_t blocks = 0;
    for (uint32_t g = 0; g < n_generations && !rc;) {
        if (g % every == 0) {
            rc = autotune_generation(b, st);
            ++g;
            continue;
        }
        const uint32_t k = std::min(every - g % every, n_generations - g);   // generations before the next sweep
        if (!b->fan.fork || k < kBlockGens) {
            for (uint32_t i = 0; i < k && !rc; ++i) rc = batch_generation(b, st);
            g += k;
            continue;
        }
        const uint32_t ov = blocks++ & 1u;
        b->passA.tune = sweep_best(b, (int)ov);
        if (hipStreamSynchronize(st) != hipSuccess) { rc = ct_fail(CT_EDEVICE, "autotune: stream wait failed"); break; }
        const auto t0 = std::chrono::steady_clock::now();
        for (uint32_t i = 0; i < kBlockGens && !rc; ++i) rc = batch_generation(b, st);
        if (!rc && hipStreamSynchronize(st) != hipSuccess) rc = ct_fail(CT_EDEVICE, "autotune: stream wait failed");
        block_ms[ov] += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        block_n[ov] += 1;
        g += kBlockGens;
    }
    if (rc) return rc;
    if (block_n[0] && block_n[1])
        b->passA.tune = sweep_best(b, block_ms[1] / block_n[1] < block_ms[0] / block_n[0] ? 1 : 0);
    else
        b->passA.tune = sweep_best(b, -1);
    return CT_OK;
}

