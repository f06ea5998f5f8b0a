// Repair by enumeration: the neighbour shells of a candidate, tested against the validity bitmask.
//
// Once the space is resolved (Section IV-A), whether a configuration is valid is one bit of the
// bitmask, so a repair's argmin can be found by visiting the candidate's neighbours in order of
// their leading key instead of scanning the valid list: the first shell (the configurations that
// share the leading key) holding a valid configuration holds the winner, which inside the shell
// is the (sub-key, L) minimum.  Shells per metric:
//   HAMMING      Hamming spheres of radius 1, 2, ...
//   INDEX_L1     index-distance spheres of radius 1, 2, ...
//   TIER_*       tier 0: the strictly-adjacent box (every v_j in {c_j - 1, c_j, c_j + 1});
//                tier 1: the adjacent box (every v_j in {c_j, nearest present value below,
//                above}); tier 2: the Hamming-1 sphere; tier 3: Hamming spheres of radius 2, 3, ...
//                Sub-key: squared distance from the particle to the value centres (TIER_EUCLID) or
//                the Philox draw of L (TIER_RANDOM); in tier 3 the radius.
// When the tier-0 box holds no valid configuration, every valid member of the tier-1 box is of
// tier 1, and so on down, so the shells are exactly the scan's tiers.  A shell is counted before
// it is visited: a candidate whose next shell would take its lookups past the caller's limit,
// that lies outside the domain, or that needs a sphere beyond radius kMaxRadius is handed to the
// scan.  Results are the scan's bit for bit (the same keys and the same lowest-L ties).
//
// Sphere members are unranked from per-candidate counting tables: E[j][k], the configurations
// that differ from c in exactly k of the parameters j..D-1 (Hamming), and N[j][s], those whose
// index distance to c over parameters j..D-1 is exactly s (index distance), each built by one
// lane per radius with shuffles.  Box members are mixed-radix over per-parameter choice lists of
// at most three values.
#include <hip/hip_runtime.h>

#include "ct_host.h"
#include "repair_plan.h"

namespace {

constexpr int kBlock = 256;
constexpr uint32_t kWaves = kBlock / 64;
constexpr uint32_t kMaxRadius = 8;               // spheres up to this radius
constexpr uint32_t kTabW = kMaxRadius + 1;
constexpr uint64_t kHuge = 1ull << 62;           // saturated count
constexpr uint32_t kNoPos = 0xFFFFFFFFu;

// one wave's working set: the candidate, its particle position, the counting table and the box
struct EnumLds {
    uint64_t tab[(CT_DMAX + 1) * kTabW];
    uint64_t stride[CT_DMAX];
    int32_t x[CT_DMAX];
    uint32_t c[CT_DMAX];
    uint32_t r[CT_DMAX];
    uint32_t ch[CT_DMAX][3];
    uint32_t nch[CT_DMAX];
};

__device__ __forceinline__ uint32_t lane_id() { return threadIdx.x & 63u; }
__device__ __forceinline__ uint32_t uni(uint32_t x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ uint64_t uni64(uint64_t x) {
    return ((uint64_t)uni((uint32_t)(x >> 32)) << 32) | uni((uint32_t)x);
}
__device__ __forceinline__ uint64_t shfl64(uint64_t v, int src) {
    const uint32_t lo = __shfl((uint32_t)v, src, 64), hi = __shfl((uint32_t)(v >> 32), src, 64);
    return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ uint64_t sat_add(uint64_t a, uint64_t b) { return a + b >= kHuge ? kHuge : a + b; }
__device__ __forceinline__ uint64_t sat_mul(uint64_t a, uint64_t b) {
    if (a == 0 || b == 0) return 0;
    return (__umul64hi(a, b) != 0 || a * b >= kHuge) ? kHuge : a * b;
}
__device__ __forceinline__ void lds_sync() {
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
}

// lexicographic (key, L) minimum over the wave; every lane gets it
__device__ __forceinline__ void wave_min(uint64_t& k, uint64_t& L) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const uint64_t k2 = shfl64(k, (int)(lane_id() ^ (uint32_t)o)), L2 = shfl64(L, (int)(lane_id() ^ (uint32_t)o));
        if (k2 < k || (k2 == k && L2 < L)) { k = k2; L = L2; }
    }
}

// contribution of value v of parameter j to the squared particle distance (TIER_EUCLID)
__device__ __forceinline__ uint64_t sq_dist(const EnumLds& w, uint32_t j, uint32_t v) {
    const int64_t d = (int64_t)w.x[j] - (int64_t)(2u * v + 1u) * 32768;
    return (uint64_t)(d * d);
}

struct Shell {
    uint32_t kind;      // 0 box, 1 Hamming sphere, 2 index-distance sphere
    uint32_t radius;
};

// member t of a shell: its linear index and squared particle distance
__device__ __forceinline__ void unrank(const EnumLds& w, uint32_t D, Shell sh, uint32_t t, bool euclid, uint64_t& L,
                                       uint64_t& d2) {
    L = 0;
    d2 = 0;
    if (sh.kind == 0) {
        for (int j = (int)D - 1; j >= 0; --j) {
            const uint32_t n = w.nch[j];
            const uint32_t q = n == 1 ? t : (n == 2 ? t >> 1 : t / 3u);
            const uint32_t v = w.ch[j][t - q * n];
            t = q;
            L += (uint64_t)v * w.stride[j];
            if (euclid) d2 += sq_dist(w, (uint32_t)j, v);
        }
        return;
    }
    uint32_t left = sh.radius;
    uint64_t idx = t;
    for (uint32_t j = 0; j < D; ++j) {
        const uint32_t c = w.c[j];
        const uint64_t* next = w.tab + (j + 1) * kTabW;
        uint32_t v = c;
        if (sh.kind == 1) {
            const uint64_t e0 = next[left];
            if (idx >= e0) {
                idx -= e0;
                const uint64_t e1 = next[left - 1];
                const uint64_t q = idx / e1;
                idx -= q * e1;
                v = q < c ? (uint32_t)q : (uint32_t)q + 1u;
                --left;
            }
        } else {
            const uint64_t n0 = next[left];
            if (idx >= n0) {
                idx -= n0;
                for (uint32_t a = 1; a <= left; ++a) {
                    const uint64_t n = next[left - a];
                    if (c >= a) {
                        if (idx < n) { v = c - a; left -= a; break; }
                        idx -= n;
                    }
                    if (c + a < w.r[j]) {
                        if (idx < n) { v = c + a; left -= a; break; }
                        idx -= n;
                    }
                }
            }
        }
        L += (uint64_t)v * w.stride[j];
        if (euclid) d2 += sq_dist(w, j, v);
    }
}

// Counting tables of the spheres around the candidate (lane k <= kMaxRadius builds column k):
// kind 1: E[j][k] = E[j+1][k] + (r_j - 1) E[j+1][k-1]; kind 2: N[j][s] = sum over a <= s of
// (ways to move parameter j by a) N[j+1][s-a].
__device__ void build_table(EnumLds& w, uint32_t D, uint32_t kind) {
    const uint32_t k = lane_id();
    uint64_t col = k == 0 ? 1u : 0u;                  // row D
    if (k < kTabW) w.tab[D * kTabW + k] = col;
    for (int j = (int)D - 1; j >= 0; --j) {
        const uint32_t c = w.c[j], r = w.r[j];
        uint64_t nv;
        if (kind == 1) {
            const uint64_t below = shfl64(col, (int)(k == 0 ? 0u : k - 1u));
            nv = sat_add(col, k == 0 ? 0ull : sat_mul(r - 1u, below));
        } else {
            nv = col;
            for (uint32_t a = 1; a < kTabW; ++a) {
                const uint64_t prev = shfl64(col, (int)(k >= a ? k - a : 0u));
                const uint32_t ways = (c >= a ? 1u : 0u) + (c + a < r ? 1u : 0u);
                if (a <= k && ways) nv = sat_add(nv, sat_mul(ways, prev));
            }
        }
        col = nv;
        if (k < kTabW) w.tab[(uint32_t)j * kTabW + k] = col;
    }
    lds_sync();
}

// choice lists of a tier box (0: strictly adjacent, 1: adjacent); returns the box size
__device__ uint64_t build_box(EnumLds& w, const DevSpace& S, uint32_t D, uint32_t tier) {
    const uint32_t j = lane_id();
    uint64_t n = 1;
    bool sub = true;
    if (j < D) {
        const uint32_t c = w.c[j], r = w.r[j];
        uint32_t m = 0;
        if (tier == 0) {
            if (c >= 1) w.ch[j][m++] = c - 1u;
            w.ch[j][m++] = c;
            if (c + 1u < r) w.ch[j][m++] = c + 1u;
        } else {
            const uint8_t* pn = S.prevnext + ((uint64_t)j * 256u + c) * 2u;
            w.ch[j][m++] = c;
            if (pn[0] != 0xFFu) w.ch[j][m++] = pn[0];
            if (pn[1] != 0xFFu) w.ch[j][m++] = pn[1];
            // inside the strictly-adjacent choices (visited already, with nothing valid)?
            sub = (pn[0] == 0xFFu || pn[0] + 1u == c) && (pn[1] == 0xFFu || pn[1] == c + 1u);
        }
        w.nch[j] = m;
        n = m;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) n *= shfl64(n, (int)(lane_id() ^ (uint32_t)o));
    lds_sync();
    // an adjacent box inside the strictly-adjacent one holds nothing valid either
    if (tier == 1 && __all(sub)) return 0;
    return uni64(n);
}

// Visits every member of a shell; the wave's (key, L) minimum over the valid ones goes into
// (bk, bL).  Sub-keys: TIER_EUCLID the squared distance, TIER_RANDOM the Philox draw, otherwise 0.
__device__ void visit(const EnumLds& w, const DevSpace& S, uint32_t D, Shell sh, uint32_t size, uint32_t metric,
                      uint64_t seed, uint32_t who, uint32_t gen, uint64_t& bk, uint64_t& bL) {
    const bool euclid = metric == CT_TIER_EUCLID && sh.kind == 0;
    const bool euclid_h1 = metric == CT_TIER_EUCLID && sh.kind == 1 && sh.radius == 1;
    const bool random = metric == CT_TIER_RANDOM && (sh.kind == 0 || sh.radius == 1);
    for (uint32_t base = 0; base < size; base += 64) {
        const uint32_t t = base + lane_id();
        uint64_t k = ~0ull, L = ~0ull;
        if (t < size) {
            uint64_t l, d2;
            unrank(w, D, sh, t, euclid || euclid_h1, l, d2);
            if (bit_valid(S, l)) {
                L = l;
                k = 0;
                if (euclid || euclid_h1) k = d2;
                else if (random) {
                    const U4 o = ct_philox(seed, who, gen, (PUR_REPAIR_KEY << 24) | (uint32_t)((l >> 32) & 0xFFFFFFu),
                                           (uint32_t)l);
                    k = o.x;
                }
            }
        }
        wave_min(k, L);
        if (k < bk || (k == bk && L < bL)) { bk = k; bL = L; }
    }
}

__global__ __launch_bounds__(kBlock) void k_repair_enum(const RepairSet* __restrict__ sets,
                                                        const RepairSet* __restrict__ rest, uint32_t n_sets,
                                                        uint64_t max_lookups, unsigned long long* stats,
                                                        PlanArgs pa) {
    __shared__ EnumLds lds[kWaves];
    EnumLds& w = lds[threadIdx.x >> 6];
    const uint32_t lane = lane_id();
    const uint32_t wave = blockIdx.x * kWaves + (threadIdx.x >> 6), waves = gridDim.x * kWaves;
    uint64_t settled = 0, looked = 0;
    for (uint32_t s = 0; s < n_sets; ++s) {
        const RepairSet& J = sets[s];
        const RepairSet& K = rest[s];
        const DevSpace& S = *J.S;
        const uint32_t D = S.D, metric = J.metric;
        const uint32_t count = __hip_atomic_load(J.count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const uint32_t gen = J.gen ? *J.gen : J.gen_value;
        for (uint32_t li = wave; li < count; li += waves) {
            const uint32_t ci = uni(J.list[li]);
            const uint32_t who = J.who ? J.who[ci] : ci;
            // the candidate, its domain and (TIER_EUCLID) its particle position, one lane per parameter
            bool in = true;
            if (lane < D) {
                const uint32_t c = J.rows[(uint64_t)ci * S.R + lane];
                w.c[lane] = c;
                w.r[lane] = S.radix[lane];
                w.stride[lane] = S.stride[lane];
                w.x[lane] = metric == CT_TIER_EUCLID ? J.pos_q16[(uint64_t)ci * D + lane] : 0;
                in = c < S.radix[lane];
            }
            lds_sync();
            // (the GA mutation metric is enumerated by its own kernel: its rows go to the scan here)
            const bool inside = __all(in) && metric <= CT_TIER_RANDOM;
            uint64_t bk = ~0ull, bL = ~0ull, used = 0;
            bool over = !inside;
            auto shell = [&](Shell sh, uint64_t size) {
                if (over || bL != ~0ull) return;
                if (size >= (1ull << 32) || used + size > max_lookups) { over = true; return; }
                used += size;
                visit(w, S, D, sh, (uint32_t)size, metric, J.seed, who, gen, bk, bL);
            };
            if (!over) {
                if (metric == CT_TIER_EUCLID || metric == CT_TIER_RANDOM) {
                    shell(Shell{0, 0}, build_box(w, S, D, 0));
                    if (!over && bL == ~0ull) shell(Shell{0, 1}, build_box(w, S, D, 1));
                    if (!over && bL == ~0ull) {
                        build_table(w, D, 1);
                        for (uint32_t rad = 1; rad <= kMaxRadius && rad <= D && !over && bL == ~0ull; ++rad)
                            shell(Shell{1, rad}, uni64(w.tab[rad]));
                    }
                } else {
                    const uint32_t kind = metric == CT_HAMMING ? 1u : 2u;
                    build_table(w, D, kind);
                    for (uint32_t rad = 1; rad <= kMaxRadius && !over && bL == ~0ull; ++rad)
                        shell(Shell{kind, rad}, uni64(w.tab[rad]));
                }
                if (bL == ~0ull) over = true;             // nothing within the largest radius
            }
            looked += used;
            if (!over) {
                const uint32_t pos = (uint32_t)rank_dir(S, bL);
                const uint32_t* src = reinterpret_cast<const uint32_t*>(S.rows + (uint64_t)pos * S.R);
                uint32_t* dst = reinterpret_cast<uint32_t*>(J.out_rows + (uint64_t)ci * S.R);
                if (lane < S.R / 4) dst[lane] = src[lane];
                if (lane == 0) J.out_pos[ci] = pos;
                ++settled;
            } else if (lane == 0) {
                const uint32_t k = atomicAdd(&K.count[0], 1u);
                K.list[k] = ci;
                K.list_ins[k] = J.list_ins[li];
            }
        }
    }
    if (lane == 0 && stats && (settled || looked)) {
        atomicAdd(&stats[0], (unsigned long long)settled);
        atomicAdd(&stats[1], (unsigned long long)looked);
    }
    plan_if_last(rest, n_sets, pa);                        // the last block plans the scans of the rest
}

__global__ void k_enum_zero(const RepairSet* __restrict__ rest, uint32_t n_sets, unsigned long long* stats) {
    const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < n_sets) {
        rest[s].count[0] = 0;
        rest[s].count[1] = 0;
    }
    if (s == 0 && stats) {
        stats[0] = 0;
        stats[1] = 0;
    }
}

}  // namespace

int launch_repair_enum(const RepairPasses& listed, const RepairPasses& rest, uint64_t max_lookups,
                       unsigned long long* d_stats, hipStream_t st) {
    if (listed.n_sets == 0 || listed.total_n == 0) return CT_OK;
    {
        ProfScope ps_("k_repair_zero", st);
        hipLaunchKernelGGL(k_enum_zero, dim3((rest.n_sets + 255) / 256), dim3(256), 0, st, rest.d_sets, rest.n_sets,
                           d_stats);
    }
    if (int rc = launch_repair_prep(listed, st)) return rc;
    {
        ProfScope ps_("k_repair_enum", st);
        const uint32_t g = std::max<uint32_t>(1, std::min<uint32_t>((listed.total_n + kWaves - 1) / kWaves, 4096));
        hipLaunchKernelGGL(k_repair_enum, dim3(g), dim3(kBlock), 0, st, listed.d_sets, rest.d_sets, listed.n_sets,
                           max_lookups, d_stats, main_plan(rest));
    }
    CT_HIP(hipGetLastError());
    // the candidates enumeration left go through the scans (already planned)
    return launch_repair_passes(rest, false, st, false, false);
}
