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

#include "ct_host.h"

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

__device__ void de_propose(const PopDev& p, uint32_t i, uint32_t g) {
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
    U4 cr{0, 0, 0, 0};
    for (uint32_t j = 0; j < p.D; ++j) {
        const int64_t num = (int64_t)base.digit(j) * 65536 +
                            (int64_t)p.F_q16 * ((int64_t)a.digit(j) - (int64_t)b.digit(j)) + 32768;
        int64_t m = num >> 16;                    // floor
        const int64_t hi = (int64_t)p.S->radix[j] - 1;
        m = m < 0 ? 0 : (m > hi ? hi : m);
        if ((j & 3u) == 0) cr = ct_philox(p.seed, i, g, ((uint32_t)PUR_DE_CR << 24) | (j >> 2), 0);
        const uint32_t cu = (j & 3u) == 0 ? cr.x : (j & 3u) == 1 ? cr.y : (j & 3u) == 2 ? cr.z : cr.w;
        if ((uint64_t)cu < p.CR_q32 || j == jr) u.set(j, (uint32_t)m);
    }
    row_store(u, p.trial + (uint64_t)i * p.R, p.R);
}

__device__ void pso_propose(const PopDev& p, uint32_t i, uint32_t g) {
    const uint32_t gi = p.state[2];
    const int64_t xmax = (int64_t)p.M * 65536 - 1;
    Row c;
#pragma unroll
    for (int q = 0; q < CT_DMAX / 4; ++q) c.w[q] = 0;
    for (uint32_t j = 0; j < p.D; ++j) {
        U4 o = ct_philox(p.seed, i, g, ((uint32_t)PUR_PSO_R << 24) | j, 0);
        const int64_t r1 = o.x >> 16, r2 = o.y >> 16;
        const uint64_t k = (uint64_t)i * p.D + j;
        int64_t x = p.X[k], v = p.V[k];
        const int64_t pb = p.PB[k], gb = p.PB[(uint64_t)gi * p.D + j];
        v = ((p.w_q16 * v) >> 16) + ((((p.c1_q16 * r1) >> 16) * (pb - x)) >> 16) +
            ((((p.c2_q16 * r2) >> 16) * (gb - x)) >> 16);
        x += v;
        x = x < 0 ? 0 : (x > xmax ? xmax : x);
        p.V[k] = v;
        p.X[k] = (int32_t)x;
        const uint32_t d = (uint32_t)(x >> 16);
        c.set(j, d < p.S->radix[j] ? d : p.S->radix[j] - 1u);
    }
    row_store(c, p.trial + (uint64_t)i * p.R, p.R);
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
__device__ void ga_propose(const PopDev& p, uint32_t i, uint32_t g) {
    const uint32_t k = i >> 1;
    U4 o = ct_philox(p.seed, k, g, (uint32_t)PUR_GA_SEL << 24, 0);
    const uint32_t a = beta_rank(p, o.x), b = beta_rank(p, o.y);
    const uint32_t cut = 1u + ct_below(o.z, p.D - 1u);
    Row A, B;
    valid_row(p, p.sorted[a], A);
    valid_row(p, p.sorted[b], B);
    Row c = (i & 1u) ? B : A;
    const Row& tail = (i & 1u) ? A : B;
    for (uint32_t j = cut; j < p.D; ++j) c.set(j, tail.digit(j));
    row_store(c, p.trial + (uint64_t)i * p.R, p.R);
    U4 m = ct_philox(p.seed, i, g, (uint32_t)PUR_GA_MUT << 24, 0);
    p.apply[i] = m.x < p.mut_thresh;
}

__global__ __launch_bounds__(kBlock) void k_propose(const PopDev* __restrict__ pops, uint32_t n,
                                                    const uint32_t* __restrict__ ind_off) {
    const uint32_t total = ind_off[n];
    for (uint32_t item = blockIdx.x * blockDim.x + threadIdx.x; item < total; item += gridDim.x * blockDim.x) {
        const uint32_t r = find_run(ind_off, n, item);
        const PopDev& p = pops[r];
        const uint32_t i = item - ind_off[r];
        const uint32_t g = p.state[0];
        if (i == 0) {
            // repair counters of this generation (no memset nodes inside captured graphs)
            p.rcount[0] = 0;
            p.rcount[1] = 0;
            p.rcount[2] = 0;
            p.rcount[3] = 0;
        }
        if (p.algo == CT_DE) de_propose(p, i, g);
        else if (p.algo == CT_PSO) pso_propose(p, i, g);
        else ga_propose(p, i, g);
    }
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
        hipLaunchKernelGGL(k_propose, dim3(g), dim3(kBlock), 0, st, b->d_pops, b->n, b->d_ind_off);
    }
    int rc = launch_repair_passes(b->passA, false, st);
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

int batch_autotune_generation(ct_batch* b, hipStream_t st) {
    if (b->n == 0) return CT_OK;
    if (b->n_ga) hipLaunchKernelGGL(k_ga_sort, dim3(b->n), dim3(kSelBlock), 0, st, b->d_pops, b->n);
    {
        const uint32_t g = std::max<uint32_t>(1, std::min<uint32_t>((b->total_ind + kBlock - 1) / kBlock, 4096));
        hipLaunchKernelGGL(k_propose, dim3(g), dim3(kBlock), 0, st, b->d_pops, b->n, b->d_ind_off);
    }
    CT_HIP(hipGetLastError());
    // The main repair pass reads the proposals and writes only its outputs, lists and counters (the
    // counters are cleared first and the scan tally is left alone), so it can run once per candidate
    // partitioning with identical results; the fastest one is kept.
    hipEvent_t e0 = nullptr, e1 = nullptr;
    CT_HIP(hipEventCreate(&e0));
    CT_HIP(hipEventCreate(&e1));
    prof_suspend(true);
    RepairPasses rp = b->passA;
    int rc = launch_repair_passes(rp, true, st, false);     // warm the caches
    float best = 3.0e38f;
    RepairTune choice = b->passA.tune;
    const uint32_t items[] = {2048, 4096, 8192};
    const uint32_t min_sub[] = {8, 16, 32, 64};
    const uint32_t grid[] = {4096, 8192};
    for (uint32_t it : items)
        for (uint32_t ms : min_sub)
            for (uint32_t gw : grid) {
                if (rc) break;
                rp.tune = RepairTune{it, ms, gw};
                (void)hipEventRecord(e0, st);
                rc = launch_repair_passes(rp, true, st, false);
                (void)hipEventRecord(e1, st);
                if (hipEventSynchronize(e1) != hipSuccess) rc = ct_fail(CT_EDEVICE, "autotune: event wait failed");
                float t = 0;
                if (!rc && hipEventElapsedTime(&t, e0, e1) == hipSuccess && t < best) {
                    best = t;
                    choice = rp.tune;
                }
            }
    prof_suspend(false);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    b->passA.tune = choice;
    // the generation's own pass, with the chosen partitioning, counting its scans
    if ((rc = launch_repair_passes(b->passA, true, st, true))) return rc;
    if (b->n_ga && (rc = launch_repair_passes(b->passC, false, st))) return rc;
    hipLaunchKernelGGL(k_select, dim3(b->n), dim3(kSelBlock), 0, st, b->d_pops, b->n);
    CT_HIP(hipGetLastError());
    return CT_OK;
}

