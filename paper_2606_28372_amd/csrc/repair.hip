// Repair of invalid configurations (Section IV-A neighbour rules; Alg. 1
// Repair, Alg. 2, Alg. 3) and the GA mutation to a random valid Hamming
// neighbour (Section IV-D), as argmin scans over the ascending valid list.
//
// For every candidate c that needs it, the scan returns
//     argmin_{v in V} (k(c, v), L(v))
// with a metric-specific key k.  The work is a branch-and-bound scan:
//   - the valid list is cut into 64-row blocks, each with a per-parameter
//     bounding box [min, max] of its value indices (built with the space);
//   - one wave owns one (candidate, part of the list) item and holds the
//     candidate wave-uniform; its lanes first test 64 boxes at once against
//     the candidate's current bound (a lower bound of the key over the box),
//     then evaluate each surviving block with one row per lane;
//   - the bound starts from the 64 valid rows around the candidate's place in
//     linear-index order, so pruning is effective from the first block;
//   - keys use byte-SIMD instructions (v_sad_u8 for index distance, a
//     byte-equality mask for Hamming); only rows whose tier can still win pay
//     for the expensive part (Euclidean distance, Philox draw);
//   - per-part winners are reduced lexicographically (key, position) by one
//     wave per candidate; ties resolve to the lowest linear index because rows
//     are visited in ascending order within a part.
// The tiered rules of Alg. 2 / Alg. 3 search the strictly-adjacent, adjacent
// and Hamming-1 neighbours first; only candidates with none of those fall
// back to a Hamming scan of the whole list.
//
// Every kernel walks an array of RepairSets (device memory), so one launch per
// phase serves any number of candidate batches over any number of spaces; a
// one-block plan kernel turns the per-set candidate counts into the item
// space of each scan without a round trip to the host.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "ct_host.h"

namespace {

constexpr int kBlock = 256;
constexpr uint32_t kTargetWaves = kRepairTargetWaves;
constexpr uint32_t kMinSubPerPart = 32;   // 64-row blocks per part, at least
constexpr uint64_t kNoKey = ~0ull;
constexpr uint32_t kNoPos = 0xFFFFFFFFu;
constexpr uint64_t kTier3 = 3ull << 62;
constexpr uint32_t kMaxSets = 4096;
constexpr uint32_t kNumMetrics = 5;

__device__ __forceinline__ uint32_t ne_bytes(uint32_t x) {
    // 0x80 in every byte of x that is non-zero
    return ((((x & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | x) & 0x80808080u);
}

__device__ __forceinline__ uint32_t wave_lane() { return threadIdx.x & 63u; }
__device__ __forceinline__ uint32_t uni(uint32_t x) { return __builtin_amdgcn_readfirstlane(x); }

__device__ __forceinline__ uint64_t wave_min_u64(uint64_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const uint32_t lo = __shfl_xor((uint32_t)v, o, 64), hi = __shfl_xor((uint32_t)(v >> 32), o, 64);
        const uint64_t w = ((uint64_t)hi << 32) | lo;
        v = w < v ? w : v;
    }
    return v;
}

// largest s with off[s] <= item, for off[0] = 0 <= item < off[n]
__device__ __forceinline__ uint32_t find_set(const uint32_t* off, uint32_t n, uint32_t item) {
    uint32_t lo = 0, hi = n;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (off[mid] <= item) lo = mid; else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ bool tiered_metric(uint32_t m) { return m == CT_TIER_EUCLID || m == CT_TIER_RANDOM; }

// ---------------------------------------------------------------------------
// Per-candidate state, wave-uniform (the candidate is the same in every lane).
// ---------------------------------------------------------------------------
template <int M, int RW>
struct Cand {
    uint32_t c[RW];
    uint32_t pv[RW], nx[RW];     // nearest present value index below / above each digit
    bool adj_is_sa;
    int32_t X[RW * 4];           // particle position (TIER_EUCLID)
    uint32_t who, gen;
    uint64_t seed;

    __device__ void load(const RepairSet& J, const DevSpace& S, uint32_t ci) {
        const uint32_t* cr = reinterpret_cast<const uint32_t*>(J.rows + (uint64_t)ci * S.R);
#pragma unroll
        for (int k = 0; k < RW; ++k) {
            // bytes past the last parameter are padding: force them to zero
            const int live = (int)S.D - 4 * k;
            const uint32_t keep = live >= 4 ? 0xFFFFFFFFu : (live <= 0 ? 0u : ((1u << (8 * live)) - 1u));
            c[k] = uni(cr[k] & keep);
        }
        adj_is_sa = true;
        if constexpr (M == CT_TIER_EUCLID || M == CT_TIER_RANDOM) {
#pragma unroll
            for (int k = 0; k < RW; ++k) { pv[k] = 0; nx[k] = 0; }
#pragma unroll
            for (int j = 0; j < RW * 4; ++j) {
                const uint32_t d = (c[j >> 2] >> ((j & 3) * 8)) & 0xFFu;
                uint32_t p = d, n = d;
                if ((uint32_t)j < S.D) {
                    p = uni(S.prevnext[((uint32_t)j * 256u + d) * 2u + 0u]);
                    n = uni(S.prevnext[((uint32_t)j * 256u + d) * 2u + 1u]);
                    // the two rules agree on parameter j unless a present value lies below (above) d while
                    // d-1 (d+1) itself never occurs in a solution; "none" is 0xFF, which no digit equals
                    adj_is_sa &= (p == d - 1u || p == 0xFFu) && (n == d + 1u || n == 0xFFu);
                }
                pv[j >> 2] |= p << ((j & 3) * 8);
                nx[j >> 2] |= n << ((j & 3) * 8);
            }
        }
        if constexpr (M == CT_TIER_EUCLID) {
#pragma unroll
            for (int j = 0; j < RW * 4; ++j)
                X[j] = (uint32_t)j < S.D ? (int32_t)uni((uint32_t)J.pos_q16[(uint64_t)ci * S.D + j]) : 0;
        }
        if constexpr (M == CT_TIER_RANDOM || M == CT_HAM1_RANDOM) {
            who = uni(J.who ? J.who[ci] : ci);
            gen = uni(J.gen ? *J.gen : J.gen_value);
            seed = J.seed;
        }
    }

    // key of row v (at list position pos) if it can go below `bound`, else kNoKey
    __device__ __forceinline__ uint64_t key(const DevSpace& S, const uint32_t* v, uint64_t pos, uint64_t bound) const {
        if constexpr (M == CT_HAMMING) {
            uint32_t h = 0;
#pragma unroll
            for (int k = 0; k < RW; ++k) h += __popc(ne_bytes(c[k] ^ v[k]));
            return h;
        } else if constexpr (M == CT_INDEX_L1) {
            uint32_t s = 0;
#pragma unroll
            for (int k = 0; k < RW; ++k) s = __builtin_amdgcn_sad_u8(v[k], c[k], s);
            return s;
        } else {
            uint32_t h = 0;
#pragma unroll
            for (int k = 0; k < RW; ++k) h += __popc(ne_bytes(c[k] ^ v[k]));
            if constexpr (M == CT_HAM1_RANDOM) {
                if (h != 1u) return kNoKey;
                const uint64_t L = S.lin[pos];
                U4 o = ct_philox(seed, who, gen, (PUR_MUT_KEY << 24) | (uint32_t)((L >> 32) & 0xFFFFFFu), (uint32_t)L);
                return o.x;
            } else {
                uint32_t s = 0;
#pragma unroll
                for (int k = 0; k < RW; ++k) s = __builtin_amdgcn_sad_u8(v[k], c[k], s);
                uint32_t tier;
                if (s == h) {
                    tier = 0;                      // every differing digit differs by exactly one
                } else {
                    bool adj = false;
                    if (!adj_is_sa) {
                        adj = true;
#pragma unroll
                        for (int k = 0; k < RW; ++k) {
                            uint32_t eq = (~ne_bytes(v[k] ^ c[k]) | ~ne_bytes(v[k] ^ pv[k]) | ~ne_bytes(v[k] ^ nx[k])) &
                                          0x80808080u;
                            adj &= eq == 0x80808080u;
                        }
                    }
                    tier = adj ? 1u : (h == 1u ? 2u : 3u);
                }
                if (((uint64_t)tier << 62) >= bound) return kNoKey;
                if (tier == 3u) return kTier3 | h;
                if constexpr (M == CT_TIER_EUCLID) {
                    uint64_t d2 = 0;
#pragma unroll
                    for (int j = 0; j < RW * 4; ++j) {
                        const int32_t cen = (int32_t)((((v[j >> 2] >> ((j & 3) * 8)) & 0xFFu) << 16) + 32768u);
                        const int64_t d = (int64_t)(X[j] - cen);
                        d2 += (uint64_t)(d * d);   // padding digits add the same constant to every row
                    }
                    return ((uint64_t)tier << 62) | d2;
                } else {
                    const uint64_t L = S.lin[pos];
                    U4 o = ct_philox(seed, who, gen, (PUR_REPAIR_KEY << 24) | (uint32_t)((L >> 32) & 0xFFFFFFu),
                                     (uint32_t)L);
                    return ((uint64_t)tier << 62) | o.x;
                }
            }
        }
    }

    // lower bound of key() over every row inside the box [lo, hi]
    __device__ __forceinline__ uint64_t bound_box(const uint32_t* lo32, const uint32_t* hi32) const {
        uint32_t miss = 0, sum = 0, far = 0;
        bool adj_ok = true;
        uint64_t e2 = 0;
#pragma unroll
        for (int k = 0; k < RW; ++k) {
            const uint32_t lw = lo32[k], hw = hi32[k];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                // padding digits are 0 in the candidate and in both box rows, so they add nothing
                const int32_t cj = (int32_t)((c[k] >> (q * 8)) & 0xFFu);
                const int32_t a = (int32_t)((lw >> (q * 8)) & 0xFFu), b = (int32_t)((hw >> (q * 8)) & 0xFFu);
                const uint32_t d = (uint32_t)max(max(a - cj, cj - b), 0);
                miss += d != 0u;
                sum += d;
                far += d > 1u;
                if constexpr (M == CT_TIER_EUCLID || M == CT_TIER_RANDOM) {
                    if (!adj_is_sa && d != 0u) {
                        const int32_t p = (int32_t)((pv[k] >> (q * 8)) & 0xFFu);
                        const int32_t n = (int32_t)((nx[k] >> (q * 8)) & 0xFFu);
                        adj_ok &= (p != 0xFF && p >= a && p <= b) || (n != 0xFF && n >= a && n <= b);
                    }
                }
                if constexpr (M == CT_TIER_EUCLID) {
                    // distance from the particle to the nearest value centre inside [a, b]
                    const int32_t x = X[k * 4 + q];
                    const int32_t ca = (a << 16) + 32768, cb = (b << 16) + 32768;
                    const int64_t t = (int64_t)max(max(ca - x, x - cb), 0);
                    e2 += (uint64_t)(t * t);
                }
            }
        }
        if constexpr (M == CT_HAMMING) return miss;
        else if constexpr (M == CT_INDEX_L1) return sum;
        else if constexpr (M == CT_HAM1_RANDOM) return miss <= 1u ? 0ull : kNoKey;
        else {
            const uint64_t sub = M == CT_TIER_EUCLID ? e2 : 0ull;
            if (far == 0u) return sub;                              // strictly adjacent rows possible
            if (!adj_is_sa && adj_ok) return (1ull << 62) | sub;     // adjacent rows possible
            if (miss <= 1u) return (2ull << 62) | sub;               // Hamming-1 rows possible
            return kTier3;
        }
    }
};

// One (candidate, part) item.  For the tiered metrics the bound starts at tier 3, so only
// neighbours of tiers 0-2 are wanted; the Hamming fallback pass handles the rest.
template <int M, int RW>
__device__ void scan_item(const RepairSet& J, const DevSpace& S, const uint32_t* list, const uint64_t* list_L,
                          uint32_t li, uint32_t part, uint32_t parts) {
    const uint32_t lane = wave_lane();
    const uint32_t ci = uni(list[li]);
    Cand<M, RW> C;
    C.load(J, S, ci);
    const uint32_t* rows32 = reinterpret_cast<const uint32_t*>(S.rows);

    constexpr bool tiered = (M == CT_TIER_EUCLID || M == CT_TIER_RANDOM);
    uint64_t bk = tiered ? kTier3 : kNoKey;        // wave-uniform exclusive bound: keys below it are wanted
    const uint64_t L = ((uint64_t)uni((uint32_t)(list_L[li] >> 32)) << 32) | uni((uint32_t)list_L[li]);
    if (L != ~0ull) {
        // seed the bound from the 64 valid rows around the candidate's place in linear-index order
        const uint64_t ins = rank_dir(S, L);
        const int64_t q = (int64_t)ins - 32 + (int64_t)lane;
        uint64_t k = kNoKey;
        if (q >= 0 && (uint64_t)q < S.n_valid) {
            uint32_t v[RW];
#pragma unroll
            for (int w = 0; w < RW; ++w) v[w] = rows32[(uint64_t)q * RW + w];
            k = C.key(S, v, (uint64_t)q, bk);
        }
        k = wave_min_u64(k);
        if (k != kNoKey && k + 1 < bk) bk = k + 1;
    }

    uint64_t mk = bk;                               // this lane's best key (exclusive until a row is found)
    uint32_t mp = kNoPos;
    const uint64_t b0 = (uint64_t)part * S.n_sub / parts, b1 = (uint64_t)(part + 1) * S.n_sub / parts;
    const uint32_t* box32 = reinterpret_cast<const uint32_t*>(S.boxes);
    for (uint64_t cb = b0; cb < b1; cb += 64) {
        // lanes over 64 boxes: which ones can hold a row below the bound?
        const uint64_t b = cb + lane;
        uint64_t lb = kNoKey;
        if (b < b1) {
            uint32_t lo[RW], hi[RW];
#pragma unroll
            for (int w = 0; w < RW; ++w) {
                lo[w] = box32[b * 2u * RW + w];
                hi[w] = box32[b * 2u * RW + RW + w];
            }
            lb = C.bound_box(lo, hi);
        }
        uint64_t m = __ballot(lb < bk);
        while (m) {
            const uint32_t t = (uint32_t)__ffsll((long long)m) - 1u;
            m &= m - 1ull;
            // lanes over the 64 rows of box cb + t
            const uint64_t r = (cb + t) * 64u + lane;
            if (r < S.n_valid) {
                uint32_t v[RW];
#pragma unroll
                for (int w = 0; w < RW; ++w) v[w] = rows32[r * RW + w];
                const uint64_t k = C.key(S, v, r, mk < bk ? mk : bk);
                if (k < mk) { mk = k; mp = (uint32_t)r; }
            }
            const uint64_t wm = wave_min_u64(mk);
            bk = wm < bk ? wm : bk;
            if (m) m &= __ballot(lb < bk);          // drop boxes the tighter bound now rules out
        }
    }
    // lexicographic (key, position) minimum over the wave
    uint64_t k2 = mp == kNoPos ? kNoKey : mk;
    uint32_t p2 = mp;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const uint32_t klo = __shfl_xor((uint32_t)k2, o, 64), khi = __shfl_xor((uint32_t)(k2 >> 32), o, 64);
        const uint32_t pq = __shfl_xor(p2, o, 64);
        const uint64_t kq = ((uint64_t)khi << 32) | klo;
        if (kq < k2 || (kq == k2 && pq < p2)) { k2 = kq; p2 = pq; }
    }
    if (lane == 0) {
        J.part_key[(uint64_t)li * parts + part] = k2;
        J.part_pos[(uint64_t)li * parts + part] = p2;
    }
}

// ---------------------------------------------------------------------------
// kernels over set arrays
// ---------------------------------------------------------------------------
__global__ void k_repair_zero(const RepairSet* __restrict__ sets, uint32_t n_sets) {
    const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < n_sets) {
        sets[s].count[0] = 0;
        sets[s].count[1] = 0;
    }
}

// Validity from the bitmask, rank from the directory, list of the candidates that need a scan.
__global__ __launch_bounds__(kBlock) void k_repair_prep(const RepairSet* __restrict__ sets, uint32_t n_sets,
                                                        const uint32_t* __restrict__ prep_off) {
    const uint32_t total = prep_off[n_sets];
    for (uint32_t item = blockIdx.x * blockDim.x + threadIdx.x; item < total; item += gridDim.x * blockDim.x) {
        const uint32_t s = find_set(prep_off, n_sets, item);
        const RepairSet& J = sets[s];
        const DevSpace& S = *J.S;
        const uint32_t i = item - prep_off[s];
        Row c;
        row_load(c, J.rows + (uint64_t)i * S.R, S.R);
        const bool dom = row_in_domain(S, c);
        const uint64_t L = dom ? row_encode(S, c) : ~0ull;
        const bool valid = dom && bit_valid(S, L);
        row_store(c, J.out_rows + (uint64_t)i * S.R, S.R);
        J.out_pos[i] = valid ? (uint32_t)rank_dir(S, L) : kNoPos;
        const bool act = J.apply == nullptr || J.apply[i];
        if (act && (J.metric == CT_HAM1_RANDOM || !valid)) {
            const uint32_t k = atomicAdd(&J.count[0], 1u);
            J.list[k] = i;
            J.list_L[k] = L;
        }
    }
}

__device__ __forceinline__ uint32_t wave_excl_scan(uint32_t v, uint32_t lane) {
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(x, o, 64);
        if (lane >= (uint32_t)o) x += y;
    }
    return x - v;
}

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// One wave: per-set candidate counts -> parts and item offsets of one scan pass.  Lane l owns
// a contiguous slice of the sets; offsets are the wave prefix of the lanes' totals plus the
// running sum inside the slice.  which = 0: main lists with each set's metric; which = 1:
// fallback lists, Hamming.
__global__ __launch_bounds__(64) void k_repair_plan(const RepairSet* __restrict__ sets, uint32_t n_sets,
                                                    uint32_t which, RepairPlan plan) {
    const uint32_t lane = threadIdx.x;
    const uint32_t chunk = (n_sets + 63u) / 64u;
    const uint32_t s0 = min(n_sets, lane * chunk), s1 = min(n_sets, s0 + chunk);
    uint32_t local = 0;
    for (uint32_t s = s0; s < s1; ++s) local += sets[s].count[which];
    const uint32_t total = wave_sum_u32(local);
    uint64_t gp = total ? kTargetWaves / total : 1;
    if (gp < 1) gp = 1;
    uint32_t tc = 0, ti[kNumMetrics] = {0, 0, 0, 0, 0};
    for (uint32_t s = s0; s < s1; ++s) {
        const uint64_t pmax = sets[s].S->n_sub / kMinSubPerPart;
        uint64_t p = gp > pmax ? pmax : gp;
        if (p < 1) p = 1;
        plan.parts[s] = (uint32_t)p;
        const uint32_t c = sets[s].count[which];
        const uint32_t m = which ? (uint32_t)CT_HAMMING : sets[s].metric;
        tc += c;
#pragma unroll
        for (uint32_t q = 0; q < kNumMetrics; ++q) ti[q] += q == m ? c * (uint32_t)p : 0u;
    }
    uint32_t oc = wave_excl_scan(tc, lane), oi[kNumMetrics];
#pragma unroll
    for (uint32_t q = 0; q < kNumMetrics; ++q) oi[q] = wave_excl_scan(ti[q], lane);
    for (uint32_t s = s0; s < s1; ++s) {
        const uint32_t p = plan.parts[s];
        const uint32_t c = sets[s].count[which];
        const uint32_t m = which ? (uint32_t)CT_HAMMING : sets[s].metric;
        plan.cand_off[s] = oc;
#pragma unroll
        for (uint32_t q = 0; q < kNumMetrics; ++q) plan.item_off[q * (n_sets + 1) + s] = oi[q];
        oc += c;
#pragma unroll
        for (uint32_t q = 0; q < kNumMetrics; ++q) oi[q] += q == m ? c * p : 0u;
    }
    if (lane == 63) {
        plan.cand_off[n_sets] = oc;
#pragma unroll
        for (uint32_t q = 0; q < kNumMetrics; ++q) plan.item_off[q * (n_sets + 1) + n_sets] = oi[q];
    }
}

template <int M>
__global__ __launch_bounds__(kBlock) void k_repair_scan(const RepairSet* __restrict__ sets, uint32_t n_sets,
                                                        RepairPlan plan, uint32_t which) {
    const uint32_t* off = plan.item_off + M * (n_sets + 1);
    const uint32_t total = off[n_sets];
    const uint32_t waves = gridDim.x * (kBlock / 64);
    for (uint32_t item = uni(blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6)); item < total; item += waves) {
        const uint32_t s = uni(find_set(off, n_sets, item));
        const RepairSet& J = sets[s];
        const DevSpace& S = *J.S;
        const uint32_t parts = uni(plan.parts[s]);
        const uint32_t local = item - off[s];
        const uint32_t li = local / parts, part = local % parts;
        const uint32_t* list = which ? J.fb_list : J.list;
        const uint64_t* list_L = which ? J.fb_L : J.list_L;
        switch (uni(S.R)) {
        case 4: scan_item<M, 1>(J, S, list, list_L, li, part, parts); break;
        case 8: scan_item<M, 2>(J, S, list, list_L, li, part, parts); break;
        case 16: scan_item<M, 4>(J, S, list, list_L, li, part, parts); break;
        default: scan_item<M, 8>(J, S, list, list_L, li, part, parts); break;
        }
    }
}

// Reduce the parts of every candidate (one wave per candidate) and write the result.  In the main
// pass of a tiered set, candidates without a tier 0-2 neighbour go to the fallback list.
__global__ __launch_bounds__(kBlock) void k_repair_finish(const RepairSet* __restrict__ sets, uint32_t n_sets,
                                                          RepairPlan plan, uint32_t which) {
    const uint32_t total = plan.cand_off[n_sets];
    const uint32_t lane = wave_lane();
    const uint32_t waves = gridDim.x * (kBlock / 64);
    for (uint32_t item = uni(blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6)); item < total; item += waves) {
        const uint32_t s = uni(find_set(plan.cand_off, n_sets, item));
        const RepairSet& J = sets[s];
        const DevSpace& S = *J.S;
        const uint32_t parts = plan.parts[s];
        const uint32_t li = item - plan.cand_off[s];
        if (which == 0 && li == 0 && lane == 0 && J.tally)
            atomicAdd(J.tally, (unsigned long long)(plan.cand_off[s + 1] - plan.cand_off[s]));
        uint64_t bk = kNoKey;
        uint32_t bp = kNoPos;
        for (uint32_t p = lane; p < parts; p += 64) {
            const uint64_t k = J.part_key[(uint64_t)li * parts + p];
            const uint32_t q = J.part_pos[(uint64_t)li * parts + p];
            if (q != kNoPos && (k < bk || (k == bk && q < bp))) { bk = k; bp = q; }
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const uint32_t klo = __shfl_xor((uint32_t)bk, o, 64), khi = __shfl_xor((uint32_t)(bk >> 32), o, 64);
            const uint32_t q = __shfl_xor(bp, o, 64);
            const uint64_t k = ((uint64_t)khi << 32) | klo;
            if (k < bk || (k == bk && q < bp)) { bk = k; bp = q; }
        }
        const uint32_t ci = (which ? J.fb_list : J.list)[li];
        if (bp != kNoPos) {
            const uint32_t* src = reinterpret_cast<const uint32_t*>(S.rows + (uint64_t)bp * S.R);
            uint32_t* dst = reinterpret_cast<uint32_t*>(J.out_rows + (uint64_t)ci * S.R);
            if (lane < S.R / 4) dst[lane] = src[lane];
            if (lane == 0) J.out_pos[ci] = bp;
        } else if (which == 0 && tiered_metric(J.metric) && lane == 0) {
            const uint32_t k = atomicAdd(&J.count[1], 1u);
            J.fb_list[k] = ci;
            J.fb_L[k] = ~0ull;           // no seed: the fallback scans the whole list
        }
    }
}

template <int M>
void launch_scan(const RepairPasses& rp, uint32_t which, hipStream_t st) {
    ProfScope ps_("k_repair_scan", st);
    hipLaunchKernelGGL((k_repair_scan<M>), dim3(kTargetWaves / (kBlock / 64)), dim3(kBlock), 0, st, rp.d_sets,
                       rp.n_sets, rp.plan, which);
}

uint32_t finish_grid(uint32_t n) { return std::max<uint32_t>(1, std::min<uint32_t>((n + 3) / 4, 2048)); }

}  // namespace

int repair_plan_alloc(RepairPlan& p, uint32_t n_sets, std::vector<void*>& owned) {
    if (n_sets > kMaxSets) return ct_fail(CT_EINVAL, "repair: at most 4096 candidate sets per launch");
    void* a = nullptr;
    const size_t words = (size_t)(n_sets + 1) * (1 + kNumMetrics) + n_sets;
    CT_HIP(hipMalloc(&a, words * sizeof(uint32_t)));
    owned.push_back(a);
    uint32_t* w = static_cast<uint32_t*>(a);
    p.cand_off = w;
    p.item_off = w + (n_sets + 1);
    p.parts = w + (n_sets + 1) * (1 + kNumMetrics);
    return CT_OK;
}

int launch_repair_passes(const RepairPasses& rp, bool zero_counts, hipStream_t st) {
    if (rp.n_sets == 0 || rp.total_n == 0) return CT_OK;
    if (zero_counts) {
        ProfScope ps_("k_repair_zero", st);
        hipLaunchKernelGGL(k_repair_zero, dim3((rp.n_sets + 255) / 256), dim3(256), 0, st, rp.d_sets, rp.n_sets);
    }
    {
        ProfScope ps_("k_repair_prep", st);
        const uint32_t g = std::max<uint32_t>(1, std::min<uint32_t>((rp.total_n + kBlock - 1) / kBlock, 4096));
        hipLaunchKernelGGL(k_repair_prep, dim3(g), dim3(kBlock), 0, st, rp.d_sets, rp.n_sets, rp.d_prep_off);
    }
    {
        ProfScope ps_("k_repair_plan", st);
        hipLaunchKernelGGL(k_repair_plan, dim3(1), dim3(64), 0, st, rp.d_sets, rp.n_sets, 0u, rp.plan);
    }
    if (rp.metrics_mask & (1u << CT_HAMMING)) launch_scan<CT_HAMMING>(rp, 0, st);
    if (rp.metrics_mask & (1u << CT_INDEX_L1)) launch_scan<CT_INDEX_L1>(rp, 0, st);
    if (rp.metrics_mask & (1u << CT_TIER_EUCLID)) launch_scan<CT_TIER_EUCLID>(rp, 0, st);
    if (rp.metrics_mask & (1u << CT_TIER_RANDOM)) launch_scan<CT_TIER_RANDOM>(rp, 0, st);
    if (rp.metrics_mask & (1u << CT_HAM1_RANDOM)) launch_scan<CT_HAM1_RANDOM>(rp, 0, st);
    {
        ProfScope ps_("k_repair_finish", st);
        hipLaunchKernelGGL(k_repair_finish, dim3(finish_grid(rp.total_n)), dim3(kBlock), 0, st, rp.d_sets, rp.n_sets,
                           rp.plan, 0u);
    }
    if (rp.metrics_mask & ((1u << CT_TIER_EUCLID) | (1u << CT_TIER_RANDOM))) {
        {
            ProfScope ps_("k_repair_plan", st);
            hipLaunchKernelGGL(k_repair_plan, dim3(1), dim3(64), 0, st, rp.d_sets, rp.n_sets, 1u, rp.plan);
        }
        launch_scan<CT_HAMMING>(rp, 1, st);
        {
            ProfScope ps_("k_repair_finish", st);
            hipLaunchKernelGGL(k_repair_finish, dim3(finish_grid(rp.total_n)), dim3(kBlock), 0, st, rp.d_sets,
                               rp.n_sets, rp.plan, 1u);
        }
    }
    CT_HIP(hipGetLastError());
    return CT_OK;
}
