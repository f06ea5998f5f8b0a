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
constexpr uint32_t kMinSubPerPart = 4;    // 64-row blocks per part, at least
constexpr uint32_t kSortCap = 4096;       // candidates sorted by linear index up to this count
constexpr uint64_t kNoKey = ~0ull;
constexpr uint32_t kNoPos = 0xFFFFFFFFu;
constexpr uint64_t kTier3 = 3ull << 62;

__device__ __forceinline__ uint32_t ne_bytes(uint32_t x) {
    // 0x80 in every byte of x that is non-zero
    return ((((x & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | x) & 0x80808080u);
}

__device__ __forceinline__ uint32_t job_gen(const RepairJob& j) { return j.d_gen ? *j.d_gen : j.gen_value; }

__device__ __forceinline__ void scan_shape(uint32_t count, uint64_t n_sub, uint32_t* n_cw, uint32_t* parts) {
    uint32_t nc = (count + 63u) / 64u;
    if (nc == 0) nc = 1;
    uint64_t p = kTargetWaves / nc;
    uint64_t pmax = n_sub / kMinSubPerPart;
    if (p > pmax) p = pmax;
    if (p < 1) p = 1;
    *n_cw = nc;
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

// Sort (L, candidate) pairs of the list by L (one block; lists above kSortCap stay unsorted).
__global__ __launch_bounds__(1024) void k_repair_sort(uint32_t* __restrict__ list, uint64_t* __restrict__ list_L,
                                                      const uint32_t* __restrict__ count_p) {
    __shared__ uint64_t key[kSortCap];
    __shared__ uint32_t val[kSortCap];
    const uint32_t count = *count_p;
    if (count <= 1 || count > kSortCap) return;
    uint32_t n = 1;
    while (n < count) n <<= 1;
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) {
        key[i] = i < count ? list_L[i] : ~0ull;
        val[i] = i < count ? list[i] : 0xFFFFFFFFu;
    }
    __syncthreads();
    for (uint32_t k = 2; k <= n; k <<= 1) {
        for (uint32_t j = k >> 1; j > 0; j >>= 1) {
            for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) {
                uint32_t l = i ^ j;
                if (l > i) {
                    bool up = (i & k) == 0;
                    uint64_t a = key[i], b = key[l];
                    uint32_t va = val[i], vb = val[l];
                    bool gt = a > b || (a == b && va > vb);
                    if (gt == up) { key[i] = b; key[l] = a; val[i] = vb; val[l] = va; }
                }
            }
            __syncthreads();
        }
    }
    for (uint32_t i = threadIdx.x; i < count; i += blockDim.x) {
        list_L[i] = key[i];
        list[i] = val[i];
    }
}

// ---------------------------------------------------------------------------
// per-candidate state and the metric keys
// ---------------------------------------------------------------------------
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
            c[k] = cr[k] & keep;
        }
        adj_is_sa = true;
        if constexpr (M == CT_TIER_EUCLID || M == CT_TIER_RANDOM) {
#pragma unroll
            for (int k = 0; k < RW; ++k) { pv[k] = 0; nx[k] = 0; }
#pragma unroll
            for (int j = 0; j < RW * 4; ++j) {
                uint32_t d = (c[j >> 2] >> ((j & 3) * 8)) & 0xFFu;
                uint32_t p = d, n = d;
                if ((uint32_t)j < S.D) {
                    p = S.prevnext[((uint32_t)j * 256u + d) * 2u + 0u];
                    n = S.prevnext[((uint32_t)j * 256u + d) * 2u + 1u];
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
            for (int j = 0; j < RW * 4; ++j) X[j] = (uint32_t)j < S.D ? J.pos_q16[(uint64_t)ci * S.D + j] : 0;
        }
        if constexpr (M == CT_TIER_RANDOM || M == CT_HAM1_RANDOM) {
            who = J.who ? J.who[ci] : ci;
            gen = job_gen(J);
            seed = J.seed;
        }
    }

    // key of row v (at list position pos) if it can beat `bound`, else kNoKey
    __device__ __forceinline__ uint64_t key(const DevSpace& S, const uint32_t* v, uint64_t pos, uint64_t bound) const {
        if constexpr (M == CT_HAMMING) {
            uint32_t h = 0;
#pragma unroll
            for (int k = 0; k < RW; ++k) h += __popc(ne_bytes(c[k] ^ v[k]));
            return h;
        } else if constexpr (M == CT_INDEX_L1) {
            uint32_t s = 0;
#pragma unroll
            for (int k = 0; k < RW; ++k) s = __builtin_amdgcn_sad_u8(c[k], v[k], s);
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
                for (int k = 0; k < RW; ++k) s = __builtin_amdgcn_sad_u8(c[k], v[k], s);
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
                        int64_t cen = (int64_t)((((v[j >> 2] >> ((j & 3) * 8)) & 0xFFu) * 2u + 1u) << 15);
                        int64_t d = (int64_t)X[j] - cen;
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
    __device__ __forceinline__ uint64_t bound_box(const DevSpace& S, const uint8_t* lo, const uint8_t* hi) const {
        uint32_t miss = 0, sum = 0, far = 0;
        bool adj_ok = true;
        const uint32_t* lo32 = reinterpret_cast<const uint32_t*>(lo);
        const uint32_t* hi32 = reinterpret_cast<const uint32_t*>(hi);
#pragma unroll
        for (int k = 0; k < RW; ++k) {
            const uint32_t lw = lo32[k], hw = hi32[k];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                // padding digits are 0 in the candidate and in both box rows, so they add nothing
                const uint32_t cj = (c[k] >> (q * 8)) & 0xFFu;
                const uint32_t a = (lw >> (q * 8)) & 0xFFu, b = (hw >> (q * 8)) & 0xFFu;
                const uint32_t d = a > cj ? a - cj : (cj > b ? cj - b : 0u);
                miss += d != 0u;
                sum += d;
                far += d > 1u;
                if constexpr (M == CT_TIER_EUCLID || M == CT_TIER_RANDOM) {
                    if (!adj_is_sa && d != 0u) {
                        const uint32_t p = (pv[k] >> (q * 8)) & 0xFFu;
                        const uint32_t n = (nx[k] >> (q * 8)) & 0xFFu;
                        adj_ok &= (p != 0xFFu && p >= a && p <= b) || (n != 0xFFu && n >= a && n <= b);
                    }
                }
            }
        }
        (void)S;
        if constexpr (M == CT_HAMMING) return miss;
        else if constexpr (M == CT_INDEX_L1) return sum;
        else if constexpr (M == CT_HAM1_RANDOM) return miss <= 1u ? 0ull : kNoKey;
        else {
            if (far == 0u) return 0ull;                         // strictly adjacent rows possible
            if (!adj_is_sa && adj_ok) return 1ull << 62;         // adjacent rows possible
            if (miss <= 1u) return 2ull << 62;                   // Hamming-1 rows possible
            return kTier3;
        }
    }
};

// Scan one part of the valid list for the 64 candidates of one wave.  For the tiered
// metrics the bound starts at tier 3, so only neighbours of tiers 0-2 are wanted.
template <int M, int RW>
__global__ __launch_bounds__(kBlock) void k_repair_scan(RepairJob J, const uint32_t* __restrict__ list,
                                                        const uint64_t* __restrict__ list_L,
                                                        const uint32_t* __restrict__ count_p,
                                                        uint64_t* __restrict__ part_key,
                                                        uint32_t* __restrict__ part_pos) {
    const DevSpace& S = J.S;
    const uint32_t count = *count_p;
    if (count == 0) return;
    uint32_t n_cw, parts;
    scan_shape(count, S.n_sub, &n_cw, &parts);
    const uint32_t item = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    if (item >= n_cw * parts) return;
    const uint32_t cw = item / parts, part = item % parts;
    const uint32_t lane = wave_lane();
    const uint32_t li = cw * 64u + lane;
    const bool active = li < count;
    const uint32_t lj = active ? li : cw * 64u;              // inactive lanes mirror an active one
    const uint32_t ci = list[lj];
    Cand<M, RW> C;
    C.load(J, ci);

    constexpr bool tiered = (M == CT_TIER_EUCLID || M == CT_TIER_RANDOM);
    uint64_t bk = tiered ? kTier3 : kNoKey;                  // exclusive bound: keys below it are wanted
    uint32_t bp = kNoPos;
    // seed the bound from the valid rows adjacent in linear-index order
    const uint64_t L = list_L[lj];
    if (L != ~0ull && S.n_valid) {
        const uint64_t ins = rank_dir(S, L);
        for (int t = -1; t <= 1; ++t) {
            const int64_t q = (int64_t)ins + t;
            if (q < 0 || (uint64_t)q >= S.n_valid) continue;
            const uint32_t* v = reinterpret_cast<const uint32_t*>(S.rows + (uint64_t)q * S.R);
            uint32_t vv[RW];
#pragma unroll
            for (int k = 0; k < RW; ++k) vv[k] = v[k];
            const uint64_t k = C.key(S, vv, (uint64_t)q, bk);
            if (k != kNoKey && k + 1 < bk) bk = k + 1;
        }
    }

    const uint64_t s0 = (uint64_t)part * S.n_sub / parts, s1 = (uint64_t)(part + 1) * S.n_sub / parts;
    for (uint64_t sb = s0; sb < s1; ++sb) {
        const uint8_t* box = S.boxes + sb * 2u * S.R;
        const uint64_t lb = C.bound_box(S, box, box + S.R);
        if (!__any(active && lb < bk)) continue;
        const uint64_t r0 = sb * 64u;
        const uint32_t nr = (uint32_t)min((uint64_t)64, S.n_valid - r0);
        const uint32_t* rows32 = reinterpret_cast<const uint32_t*>(S.rows) + r0 * RW;
        for (uint32_t r = 0; r < nr; ++r) {
            uint32_t v[RW];
#pragma unroll
            for (int k = 0; k < RW; ++k) v[k] = rows32[r * RW + k];
            const uint64_t k = C.key(S, v, r0 + r, bk);
            if (k < bk) {
                bk = k;
                bp = (uint32_t)(r0 + r);
            }
        }
    }
    if (active) {
        part_key[(uint64_t)li * parts + part] = bp == kNoPos ? kNoKey : bk;
        part_pos[(uint64_t)li * parts + part] = bp;
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
    uint32_t n_cw, parts;
    scan_shape(count, S.n_sub, &n_cw, &parts);
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
            fb_L[k] = ~0ull;             // no seed needed: the fallback scans everything
        }
    }
}

template <int M>
void launch_scan_w(const RepairJob& J, uint32_t RW, const uint32_t* list, const uint64_t* list_L,
                   const uint32_t* count, const RepairScratch& rs, hipStream_t st) {
    const uint64_t ncw = (J.n + 63) / 64;
    const uint64_t items = std::max<uint64_t>(kTargetWaves, ncw);
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
    // parts * count <= max(count, kTargetWaves * 64)
    const uint64_t slots = std::max<uint64_t>(rs.cap, (uint64_t)kTargetWaves * 64u);
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
    { ProfScope ps_("k_repair_sort", st); hipLaunchKernelGGL(k_repair_sort, dim3(1), dim3(1024), 0, st, list, list_L, count); }
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
