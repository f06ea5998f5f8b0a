// Repair of invalid configurations (Section IV-A neighbour rules; Alg. 1
// Repair, Alg. 2, Alg. 3) and the GA mutation to a random valid Hamming
// neighbour (Section IV-D), as argmin scans over the ascending valid list.
//
// For every candidate c that needs it, the scan returns
//     argmin_{v in V} (k(c, v), L(v))
// with a metric-specific key k.  The work is a branch-and-bound scan:
//   - the valid list is cut into 64-row blocks, each with a per-parameter
//     bounding box [min, max] of its value indices (built with the space);
//   - a wave holds 64 candidates (sorted by linear index so that lanes are
//     close in the space), one per lane, and walks a contiguous part of the
//     list; for every block each lane computes a lower bound of its key over
//     the box, and the whole wave skips the block when no lane could improve;
//   - every lane starts from an upper bound taken from the valid rows next to
//     the candidate in linear-index order, so pruning starts at once;
//   - rows of a block are wave-uniform loads; keys are computed with byte-SIMD
//     instructions (v_sad_u8 for index distance, a byte-equality mask for
//     Hamming) and only rows whose tier can still win pay for the expensive
//     part (Euclidean distance, Philox draw);
//   - parts are reduced lexicographically (key, position) by one wave per
//     candidate, and ties resolve to the lowest linear index everywhere
//     because rows are visited in ascending order within a part.
// The tiered rules of Alg. 2 / Alg. 3 search the strictly-adjacent,
// adjacent and Hamming-1 neighbours first; only candidates with none of
// those fall back to a Hamming scan of the whole list.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "ct_host.h"

namespace {

constexpr int kBlock = 256;
constexpr uint32_t kTargetWaves = 8192;   // scan items launched per pass
constexpr uint32_t kMinSubPerPart = 32;   // 64-row blocks per part, at least
constexpr uint64_t kNoKey = ~0ull;
constexpr uint32_t kNoPos = 0xFFFFFFFFu;
constexpr uint64_t kTier3 = 3ull << 62;

__device__ __forceinline__ uint32_t ne_bytes(uint32_t x) {
    // 0x80 in every byte of x that is non-zero
    return ((((x & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | x) & 0x80808080u);
}

__device__ __forceinline__ uint32_t job_gen(const RepairJob& j) { return j.d_gen ? *j.d_gen : j.gen_value; }

// Parts of the valid list per candidate: enough (candidate, part) waves to fill the chip,
// each part at least kMinSubPerPart 64-row blocks.  count * parts <= max(count, kTargetWaves).
__device__ __forceinline__ void scan_parts(uint32_t count, uint64_t n_sub, uint32_t* parts) {
    uint64_t p = count ? kTargetWaves / count : 1;
    const uint64_t pmax = n_sub / kMinSubPerPart;
    if (p > pmax) p = pmax;
    if (p < 1) p = 1;
    *parts = (uint32_t)p;
}

__device__ __forceinline__ uint32_t wave_lane() { return threadIdx.x & 63u; }

// ---------------------------------------------------------------------------
// prep: validity from the bitmask, rank from the directory, list of the
// candidates that need a scan (with their linear index for sorting)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_repair_prep(RepairJob J, uint32_t* __restrict__ list,
                                                        uint64_t* __restrict__ list_L, uint32_t* __restrict__ count) {
    const DevSpace& S = J.S;
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool in = i < J.n;
    bool need = false;
    uint64_t L = ~0ull;
    if (in) {
        Row c;
        row_load(c, J.rows + i * S.R, S.R);
        const bool dom = row_in_domain(S, c);
        L = dom ? row_encode(S, c) : ~0ull;
        const bool valid = dom && bit_valid(S, L);
        row_store(c, J.out_rows + i * S.R, S.R);
        J.out_pos[i] = valid ? (uint32_t)rank_dir(S, L) : kNoPos;
        const bool act = J.apply == nullptr || J.apply[i];
        need = act && (J.metric == CT_HAM1_RANDOM || !valid);
    }
    uint64_t m = __ballot(need);
    if (m) {
        uint32_t lane = wave_lane();
        uint32_t leader = (uint32_t)__ffsll((long long)m) - 1u;
        uint32_t base = 0;
        if (lane == leader) base = atomicAdd(count, (uint32_t)__popcll(m));
        base = __shfl(base, (int)leader, 64);
        if (need) {
            uint32_t k = base + (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
            list[k] = (uint32_t)i;
            list_L[k] = L;
        }
    }
}

// ---------------------------------------------------------------------------
// the scan: one candidate per wave, lanes over boxes and then over rows
// ---------------------------------------------------------------------------
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

// Per-candidate state, wave-uniform (the candidate is the same in every lane).
template <int M, int RW>
struct Cand {
    uint32_t c[RW];
    uint32_t pv[RW], nx[RW];     // nearest present value index below / above each digit
    bool adj_is_sa;
    int32_t X[RW * 4];           // particle position (TIER_EUCLID)
    uint32_t who, gen;
    uint64_t seed;

    __device__ void load(const RepairJob& J, uint32_t ci) {
        const DevSpace& S = J.S;
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
            gen = uni(job_gen(J));
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

// One wave = one (candidate, part) item.  For the tiered metrics the bound starts at tier 3,
// so only neighbours of tiers 0-2 are wanted; the Hamming fallback handles the rest.
template <int M, int RW>
__global__ __launch_bounds__(kBlock) void k_repair_scan(RepairJob J, const uint32_t* __restrict__ list,
                                                        const uint64_t* __restrict__ list_L,
                                                        const uint32_t* __restrict__ count_p,
                                                        uint64_t* __restrict__ part_key,
                                                        uint32_t* __restrict__ part_pos) {
    const DevSpace& S = J.S;
    const uint32_t count = *count_p;
    if (count == 0) return;
    uint32_t parts;
    scan_parts(count, S.n_sub, &parts);
    const uint32_t item = uni(blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6));
    if (item >= count * parts) return;
    const uint32_t li = item / parts, part = item % parts;
    const uint32_t lane = wave_lane();
    const uint32_t ci = uni(list[li]);
    Cand<M, RW> C;
    C.load(J, ci);
    const uint32_t* rows32 = reinterpret_cast<const uint32_t*>(S.rows);

    constexpr bool tiered = (M == CT_TIER_EUCLID || M == CT_TIER_RANDOM);
    uint64_t bk = tiered ? kTier3 : kNoKey;        // wave-uniform exclusive bound: keys below it are wanted
    // seed the bound from the 64 valid rows around the candidate's place in linear-index order
    const uint64_t L = ((uint64_t)uni((uint32_t)(list_L[li] >> 32)) << 32) | uni((uint32_t)list_L[li]);
    if (L != ~0ull) {
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
        bool pass = false;
        uint64_t lb = kNoKey;
        if (b < b1) {
            uint32_t lo[RW], hi[RW];
#pragma unroll
            for (int w = 0; w < RW; ++w) {
                lo[w] = box32[b * 2u * RW + w];
                hi[w] = box32[b * 2u * RW + RW + w];
            }
            lb = C.bound_box(lo, hi);
            pass = lb < bk;
        }
        uint64_t m = __ballot(pass);
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
            if (m) {
                // drop boxes of this chunk that the tighter bound now rules out
                m &= __ballot(lb < bk);
            }
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
        part_key[(uint64_t)li * parts + part] = k2;
        part_pos[(uint64_t)li * parts + part] = p2;
    }
}

// Reduce the parts of every candidate (one wave per candidate) and write the result.
// fb_list / fb_count (nullable): candidates whose first pass found nothing.
__global__ __launch_bounds__(kBlock) void k_repair_finish(RepairJob J, const uint32_t* __restrict__ list,
                                                          const uint32_t* __restrict__ count_p,
                                                          const uint64_t* __restrict__ part_key,
                                                          const uint32_t* __restrict__ part_pos,
                                                          uint32_t* __restrict__ fb_list, uint64_t* __restrict__ fb_L,
                                                          uint32_t* __restrict__ fb_count) {
    const DevSpace& S = J.S;
    const uint32_t count = *count_p;
    uint32_t parts;
    scan_parts(count, S.n_sub, &parts);
    if (J.tally && blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(J.tally, (unsigned long long)count);
    const uint32_t lane = wave_lane();
    const uint32_t waves = gridDim.x * (kBlock / 64);
    for (uint32_t li = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6); li < count; li += waves) {
        uint64_t bk = kNoKey;
        uint32_t bp = kNoPos;
        for (uint32_t p = lane; p < parts; p += 64) {
            const uint64_t k = part_key[(uint64_t)li * parts + p];
            const uint32_t q = part_pos[(uint64_t)li * parts + p];
            if (q != kNoPos && (k < bk || (k == bk && q < bp))) { bk = k; bp = q; }
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const uint32_t klo = __shfl_xor((uint32_t)bk, o, 64), khi = __shfl_xor((uint32_t)(bk >> 32), o, 64);
            const uint32_t q = __shfl_xor(bp, o, 64);
            const uint64_t k = ((uint64_t)khi << 32) | klo;
            if (k < bk || (k == bk && q < bp)) { bk = k; bp = q; }
        }
        const uint32_t ci = list[li];
        if (bp != kNoPos) {
            const uint32_t* src = reinterpret_cast<const uint32_t*>(S.rows + (uint64_t)bp * S.R);
            uint32_t* dst = reinterpret_cast<uint32_t*>(J.out_rows + (uint64_t)ci * S.R);
            if (lane < S.R / 4) dst[lane] = src[lane];
            if (lane == 0) J.out_pos[ci] = bp;
        } else if (fb_count && lane == 0) {
            const uint32_t k = atomicAdd(fb_count, 1u);
            fb_list[k] = ci;
            fb_L[k] = ~0ull;             // no seed: the fallback scans the whole list
        }
    }
}

template <int M>
void launch_scan_w(const RepairJob& J, uint32_t RW, const uint32_t* list, const uint64_t* list_L,
                   const uint32_t* count, const RepairScratch& rs, hipStream_t st) {
    const uint64_t items = std::max<uint64_t>(kTargetWaves, J.n);   // >= count * parts
    dim3 g((uint32_t)((items + 3) / 4)), b(kBlock);
    ProfScope ps_("k_repair_scan", st);
    switch (RW) {
    case 1: hipLaunchKernelGGL((k_repair_scan<M, 1>), g, b, 0, st, J, list, list_L, count, rs.part_key, rs.part_pos); break;
    case 2: hipLaunchKernelGGL((k_repair_scan<M, 2>), g, b, 0, st, J, list, list_L, count, rs.part_key, rs.part_pos); break;
    case 4: hipLaunchKernelGGL((k_repair_scan<M, 4>), g, b, 0, st, J, list, list_L, count, rs.part_key, rs.part_pos); break;
    default: hipLaunchKernelGGL((k_repair_scan<M, 8>), g, b, 0, st, J, list, list_L, count, rs.part_key, rs.part_pos); break;
    }
}

void launch_finish(const RepairJob& J, const uint32_t* list, const uint32_t* count, const RepairScratch& rs,
                   uint32_t* fb_list, uint64_t* fb_L, uint32_t* fb_count, hipStream_t st) {
    uint32_t gf = (uint32_t)std::min<uint64_t>((J.n + 3) / 4, 4096);
    ProfScope ps_("k_repair_finish", st);
    hipLaunchKernelGGL(k_repair_finish, dim3(gf), dim3(kBlock), 0, st, J, list, count, rs.part_key, rs.part_pos,
                       fb_list, fb_L, fb_count);
}

}  // namespace

int repair_scratch_alloc(RepairScratch& rs, uint64_t cap, uint32_t max_parts, hipStream_t st) {
    (void)max_parts;
    rs.cap = cap ? cap : 1;
    // parts * count <= max(count, kTargetWaves)
    const uint64_t slots = std::max<uint64_t>(rs.cap, (uint64_t)kTargetWaves);
    rs.max_parts = kTargetWaves;
    CT_HIP(hipMallocAsync((void**)&rs.list, 2 * rs.cap * sizeof(uint32_t), st));
    CT_HIP(hipMallocAsync((void**)&rs.list_L, 2 * rs.cap * sizeof(uint64_t), st));
    CT_HIP(hipMallocAsync((void**)&rs.count, 2 * sizeof(uint32_t), st));
    CT_HIP(hipMallocAsync((void**)&rs.part_key, slots * sizeof(uint64_t), st));
    CT_HIP(hipMallocAsync((void**)&rs.part_pos, slots * sizeof(uint32_t), st));
    return CT_OK;
}

void repair_scratch_free(RepairScratch& rs, hipStream_t st) {
    if (rs.list) (void)hipFreeAsync(rs.list, st);
    if (rs.list_L) (void)hipFreeAsync(rs.list_L, st);
    if (rs.count) (void)hipFreeAsync(rs.count, st);
    if (rs.part_key) (void)hipFreeAsync(rs.part_key, st);
    if (rs.part_pos) (void)hipFreeAsync(rs.part_pos, st);
    rs = RepairScratch{};
}

int launch_repair(const ct_space* s, const RepairJob& J, RepairScratch& rs, hipStream_t st) {
    if (J.n == 0) return CT_OK;
    if (J.n > rs.cap) return ct_fail(CT_EINVAL, "repair: more candidates than the scratch holds");
    uint32_t* list = rs.list;
    uint64_t* list_L = rs.list_L;
    uint32_t* fb_list = rs.list + rs.cap;
    uint64_t* fb_L = rs.list_L + rs.cap;
    uint32_t* count = rs.count;
    uint32_t* fb_count = rs.count + 1;
    CT_HIP(hipMemsetAsync(rs.count, 0, 2 * sizeof(uint32_t), st));
    uint32_t gp = (uint32_t)std::min<uint64_t>((J.n + kBlock - 1) / kBlock, 0x7FFFFFFFull);
    { ProfScope ps_("k_repair_prep", st); hipLaunchKernelGGL(k_repair_prep, dim3(gp), dim3(kBlock), 0, st, J, list, list_L, count); }
    const uint32_t RW = s->R / 4;
    switch (J.metric) {
    case CT_HAMMING:
        launch_scan_w<CT_HAMMING>(J, RW, list, list_L, count, rs, st);
        launch_finish(J, list, count, rs, nullptr, nullptr, nullptr, st);
        break;
    case CT_INDEX_L1:
        launch_scan_w<CT_INDEX_L1>(J, RW, list, list_L, count, rs, st);
        launch_finish(J, list, count, rs, nullptr, nullptr, nullptr, st);
        break;
    case CT_HAM1_RANDOM:
        launch_scan_w<CT_HAM1_RANDOM>(J, RW, list, list_L, count, rs, st);
        launch_finish(J, list, count, rs, nullptr, nullptr, nullptr, st);
        break;
    default: {
        // tiered rules: neighbours first, Hamming over the whole list for candidates without any
        if (J.metric == CT_TIER_EUCLID) launch_scan_w<CT_TIER_EUCLID>(J, RW, list, list_L, count, rs, st);
        else launch_scan_w<CT_TIER_RANDOM>(J, RW, list, list_L, count, rs, st);
        launch_finish(J, list, count, rs, fb_list, fb_L, fb_count, st);
        RepairJob J2 = J;
        J2.metric = CT_HAMMING;
        J2.tally = nullptr;
        launch_scan_w<CT_HAMMING>(J2, RW, fb_list, fb_L, fb_count, rs, st);
        launch_finish(J2, fb_list, fb_count, rs, nullptr, nullptr, nullptr, st);
        break;
    }
    }
    CT_HIP(hipGetLastError());
    return CT_OK;
}
