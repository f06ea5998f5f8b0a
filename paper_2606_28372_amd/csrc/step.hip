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

// minimum over the block (all threads get the result)
__device__ uint64_t block_min_u64(uint64_t v) {
    __shared__ uint64_t part[kSelBlock / 64];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        uint64_t w = shfl_xor_u64(v, o);
        v = w < v ? w : v;
    }
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
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    __syncthreads();
    if ((threadIdx.x & 63u) == 0) part[threadIdx.x >> 6] = v;
    __syncthreads();
    uint32_t r = 0;
    for (uint32_t k = 0; k < blockDim.x / 64; ++k) r += part[k];
    __syncthreads();
    return r;
}

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
    uint32_t pos = init_pos(p, i, 0);
    float f = p.obj[pos];
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
    } else {
        p.pos[i] = pos;
        p.f[i] = f;
        if (p.algo == CT_DE) atomicOr(&p.member[pos >> 5], 1u << (pos & 31u));
    }
}

__global__ __launch_bounds__(kSelBlock) void k_init_finish(PopDev p) {
    uint64_t m = ~0ull;
    for (uint32_t i = threadIdx.x; i < p.P; i += blockDim.x)
        m = min(m, p.algo == CT_PSO ? (((uint64_t)ford(p.f_pb[i]) << 32) | i) : best_key(p.f[i], p.pos[i]));
    m = block_min_u64(m);
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
            p.state[2] = 0;
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

__device__ Row de_propose(const PopDev& p, uint32_t i, uint32_t g) {
    U4 o = ct_philox(p.seed, i, g, (uint32_t)PUR_DE_PICK << 24, 0);
    uint32_t ex[3] = {i, 0, 0};
    const uint32_t r1 = pick_excl(o.x, p.P, ex, 1);
    ex[1] = r1;
    sort3(ex, 2);
    const uint32_t r2 = pick_excl(o.y, p.P, ex, 2);
    ex[2] = r2;
    sort3(ex, 3);
    const uint32_t r3 = pick_excl(o.z, p.P, ex, 3);
    const uint32_t jr = ct_below(o.w, p.D);
    Row base, x, a, b, u;
    valid_row(p, p.de_best ? (uint32_t)(*p.best & 0xFFFFFFFFu) : p.pos[r1], base);
    valid_row(p, p.pos[i], x);
    valid_row(p, p.pos[r2], a);
    valid_row(p, p.pos[r3], b);
    u = x;
    // words of 4 digits, one Philox block per word (draw t of block j/4 decides digit j); both
    // loops unrolled so every digit index is a compile-time constant and the rows stay in registers
#pragma unroll
    for (uint32_t q = 0; q < CT_DMAX / 4; ++q) {
        if (q * 4u >= p.D) break;
        const U4 cr = ct_philox(p.seed, i, g, ((uint32_t)PUR_DE_CR << 24) | q, 0);
#pragma unroll
        for (uint32_t t = 0; t < 4; ++t) {
            const uint32_t j = q * 4u + t;
            if (j < p.D) {
                const int64_t num = (int64_t)base.digit(j) * 65536 +
                                    (int64_t)p.F_q16 * ((int64_t)a.digit(j) - (int64_t)b.digit(j)) + 32768;
                int64_t m = num >> 16;            // floor
                const int64_t hi = (int64_t)p.S->radix[j] - 1;
                m = m < 0 ? 0 : (m > hi ? hi : m);
                const uint32_t cu = t == 0 ? cr.x : t == 1 ? cr.y : t == 2 ? cr.z : cr.w;
                if ((uint64_t)cu < p.CR_q32 || j == jr) u.set(j, (uint32_t)m);
            }
        }
    }
    row_store(u, p.trial + (uint64_t)i * p.R, p.R);
    return u;
}

__device__ Row pso_propose(const PopDev& p, uint32_t i, uint32_t g) {
    const uint32_t gi = p.state[2];
    const int64_t xmax = (int64_t)p.M * 65536 - 1;
    Row c;
#pragma unroll
    for (int q = 0; q < CT_DMAX / 4; ++q) c.w[q] = 0;
    // every load first, every store after: a store before a load would make the load's wait
    // (one in-order counter for both) wait for the store too, one round trip per parameter
    int32_t x_new[CT_DMAX];
    int64_t v_new[CT_DMAX];
#pragma unroll
    for (uint32_t j = 0; j < CT_DMAX; ++j) {
        if (j >= p.D) break;
        U4 o = ct_philox(p.seed, i, g, ((uint32_t)PUR_PSO_R << 24) | j, 0);
        const int64_t r1 = o.x >> 16, r2 = o.y >> 16;
        const uint64_t k = (uint64_t)i * p.D + j;
        int64_t x = p.X[k], v = p.V[k];
        const int64_t pb = p.PB[k], gb = p.PB[(uint64_t)gi * p.D + j];
        v = ((p.w_q16 * v) >> 16) + ((((p.c1_q16 * r1) >> 16) * (pb - x)) >> 16) +
            ((((p.c2_q16 * r2) >> 16) * (gb - x)) >> 16);
        x += v;
        x = x < 0 ? 0 : (x > xmax ? xmax : x);
        x_new[j] = (int32_t)x;
        v_new[j] = v;
        const uint32_t d = (uint32_t)(x >> 16);
        c.set(j, d < p.S->radix[j] ? d : p.S->radix[j] - 1u);
    }
#pragma unroll
    for (uint32_t j = 0; j < CT_DMAX; ++j) {
        if (j >= p.D) break;
        const uint64_t k = (uint64_t)i * p.D + j;
        p.V[k] = v_new[j];
        p.X[k] = x_new[j];
    }
    row_store(c, p.trial + (uint64_t)i * p.R, p.R);
    return c;
}

__device__ __forceinline__ uint32_t beta_rank(const PopDev& p, uint32_t u) {
    uint32_t lo = 0, hi = p.P - 1;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if ((uint64_t)u < p.beta[mid]) hi = mid; else lo = mid + 1;
    }
    return lo;
}

// child i of pair i/2: A[:cut] + B[cut:] for even i, B[:cut] + A[cut:] for odd i
__device__ Row ga_propose(const PopDev& p, uint32_t i, uint32_t g) {
    const uint32_t k = i >> 1;
    U4 o = ct_philox(p.seed, k, g, (uint32_t)PUR_GA_SEL << 24, 0);
    const uint32_t a = beta_rank(p, o.x), b = beta_rank(p, o.y);
    const uint32_t cut = 1u + ct_below(o.z, p.D - 1u);
    Row A, B;
    valid_row(p, p.sorted[a], A);
    valid_row(p, p.sorted[b], B);
    // word-wise selects keep both rows in registers (a reference picked at run time would not)
    const bool odd = (i & 1u) != 0;
    Row c, tail;
#pragma unroll
    for (int q = 0; q < CT_DMAX / 4; ++q) {
        c.w[q] = odd ? B.w[q] : A.w[q];
        tail.w[q] = odd ? A.w[q] : B.w[q];
    }
#pragma unroll
    for (uint32_t j = 1; j < CT_DMAX; ++j)
        if (j >= cut && j < p.D) c.set(j, tail.digit(j));
    row_store(c, p.trial + (uint64_t)i * p.R, p.R);
    U4 m = ct_philox(p.seed, i, g, (uint32_t)PUR_GA_MUT << 24, 0);
    p.apply[i] = m.x < p.mut_thresh;
    return c;
}

// What the main repair pass's prep step computes for a proposal -- its validity from the
// bitmask, its position (or insertion point) from the rank directory, and its entry in the
// list of candidates to repair -- done here while the row is still in registers.
__device__ __forceinline__ void list_for_repair(const PopDev& p, const RepairSet& J, uint32_t i, const Row& u) {
    const DevSpace& S = *p.S;
    uint64_t L = 0;
    bool dom = true;
#pragma unroll
    for (uint32_t j = 0; j < CT_DMAX; ++j) {
        if (j >= p.D) break;
        dom &= u.digit(j) < S.radix[j];
        L += (uint64_t)u.digit(j) * S.stride[j];
    }
    if (!dom) L = ~0ull;
    const bool valid = dom && bit_valid(S, L);
    const uint32_t pos = valid ? (uint32_t)rank_dir(S, L) : 0xFFFFFFFFu;   // loads before any store
    row_store(u, J.out_rows + (uint64_t)i * p.R, p.R);
    J.out_pos[i] = pos;
    if (!valid) {
        const uint32_t k = atomicAdd(&J.count[0], 1u);
        J.list[k] = i;
        J.list_L[k] = L;
    }
}

// Proposals of every run, one thread per individual, each listed for the main repair pass
// (`sets`, one per run in run order).  The repair counters were cleared by the previous
// generation's selection (or at creation), never by a memset node inside a captured graph.
__global__ __launch_bounds__(kBlock) void k_propose(const PopDev* __restrict__ pops, uint32_t n,
                                                    const uint32_t* __restrict__ ind_off,
                                                    const RepairSet* __restrict__ sets, PlanArgs pa) {
    const uint32_t total = ind_off[n];
    for (uint32_t item = blockIdx.x * blockDim.x + threadIdx.x; item < total; item += gridDim.x * blockDim.x) {
        const uint32_t r = find_run(ind_off, n, item);
        const PopDev& p = pops[r];
        const uint32_t i = item - ind_off[r];
        const uint32_t g = p.state[0];
        const Row u = p.algo == CT_DE ? de_propose(p, i, g) : p.algo == CT_PSO ? pso_propose(p, i, g) : ga_propose(p, i, g);
        list_for_repair(p, sets[r], i, u);
    }
    plan_if_last(sets, n, pa);                          // the last block plans the main scans
}

// ---------------------------------------------------------------------------
// GA: sort the population by (objective, position), one block per GA run
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kSelBlock) void k_ga_sort(const PopDev* __restrict__ pops, uint32_t n) {
    __shared__ uint64_t key[kGaMaxSort];
    const PopDev& p = pops[blockIdx.x];
    if (p.algo != CT_GA) return;
    uint32_t m = 1;
    while (m < p.P) m <<= 1;
    if (m <= blockDim.x) {
        // one key per thread: bitonic stages whose partner is in the same wave exchange through
        // cross-lane shuffles; only partners 64 or more apart go through LDS and a barrier
        const uint32_t i = threadIdx.x;
        uint64_t v = i < p.P ? best_key(p.f[i], p.pos[i]) : ~0ull;
        for (uint32_t k = 2; k <= m; k <<= 1) {
            for (uint32_t j = k >> 1; j > 0; j >>= 1) {
                uint64_t o;
                if (j >= 64) {
                    key[i] = v;
                    __syncthreads();
                    o = key[i ^ j];
                    __syncthreads();
                } else {
                    o = shfl_xor_u64(v, (int)j);
                }
                const bool keep_min = ((i & j) == 0) == ((i & k) == 0);
                v = keep_min ? (o < v ? o : v) : (o > v ? o : v);
            }
        }
        if (i < p.P) p.sorted[i] = (uint32_t)v;
        return;
    }
    for (uint32_t i = threadIdx.x; i < m; i += blockDim.x) key[i] = i < p.P ? best_key(p.f[i], p.pos[i]) : ~0ull;
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
}

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

__device__ void ga_select(const PopDev& p) {
    const uint32_t g = p.state[0];
    uint64_t m = ~0ull;
    for (uint32_t i = threadIdx.x; i < p.P; i += blockDim.x) {
        uint32_t t = p.tpos[i];
        if (t >= p.n_valid) t = p.pos[i];      // unreachable: every repaired child is valid
        p.pos[i] = t;
        p.f[i] = p.obj[t];
        m = min(m, best_key(p.f[i], t));
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
    if (p.algo == CT_DE) de_select(p);
    else if (p.algo == CT_PSO) pso_select(p);
    else ga_select(p);
    if (threadIdx.x < 4) p.rcount[threadIdx.x] = 0;      // repair counters of the next generation
}

}  // namespace

int pop_init_device(ct_pop* p, hipStream_t st) {
    const PopDev& d = p->dev;
    { ProfScope ps_("k_init", st); hipLaunchKernelGGL(k_init, dim3((d.P + kBlock - 1) / kBlock), dim3(kBlock), 0, st, d); }
    { ProfScope ps_("k_init_finish", st); hipLaunchKernelGGL(k_init_finish, dim3(1), dim3(kSelBlock), 0, st, d); }
    CT_HIP(hipGetLastError());
    return CT_OK;
}

int batch_generation(ct_batch* b, hipStream_t st) {
    if (b->n == 0) return CT_OK;
    if (b->n_ga) {
        ProfScope ps_("k_ga_sort", st);
        hipLaunchKernelGGL(k_ga_sort, dim3(b->n), dim3(kSelBlock), 0, st, b->d_pops, b->n);
    }
    {
        ProfScope ps_("k_propose", st);
        const uint32_t g = std::max<uint32_t>(1, std::min<uint32_t>((b->total_ind + kBlock - 1) / kBlock, 4096));
        hipLaunchKernelGGL(k_propose, dim3(g), dim3(kBlock), 0, st, b->d_pops, b->n, b->d_ind_off, b->passA.d_sets,
                           main_plan(b->passA));
    }
    int rc = launch_repair_passes(b->passA, false, st, true, false);
    if (rc) return rc;
    if (b->n_ga) {
        rc = launch_repair_passes(b->passC, false, st);
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
        for (uint32_t mode : modes)
            for (uint32_t it : {2048u, 4096u, 8192u})
                for (uint32_t ms : {8u, 16u, 32u, 64u})
                    for (uint32_t gw : {4096u, 8192u}) b->tune_cand.push_back(RepairTune{it, ms, gw, mode});
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
    if (b->n_ga) hipLaunchKernelGGL(k_ga_sort, dim3(b->n), dim3(kSelBlock), 0, st, b->d_pops, b->n);
    {
        const uint32_t g = std::max<uint32_t>(1, std::min<uint32_t>((b->total_ind + kBlock - 1) / kBlock, 4096));
        // the sweep lists and plans again for every candidate
        hipLaunchKernelGGL(k_propose, dim3(g), dim3(kBlock), 0, st, b->d_pops, b->n, b->d_ind_off, b->passA.d_sets,
                           PlanArgs{});
    }
    CT_HIP(hipGetLastError());
    int rc = autotune_sweep(b, st);
    if (rc) return rc;
    b->passA.tune = sweep_best(b, -1);
    // the generation's own pass, counting its scans
    if ((rc = launch_repair_passes(b->passA, true, st, true))) return rc;
    if (b->n_ga && (rc = launch_repair_passes(b->passC, false, st))) return rc;
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

