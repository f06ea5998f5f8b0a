// Repair of invalid configurations (Section IV-A neighbour rules; Alg. 1
// Repair, Alg. 2, Alg. 3) and the GA mutation to a random valid Hamming
// neighbour (Section IV-D), as one argmin scan over the valid list.
//
// For every candidate c that needs it, the scan computes
//     argmin_{v in V} (k(c, v), L(v))
// with a metric-specific key k.  Work layout: a block holds 256 candidates,
// one per lane of its 4 waves; the block streams a contiguous part of the
// valid list through LDS in tiles, and every lane reads each row as a
// wave-uniform (broadcast) LDS load.  Because rows arrive in ascending L
// order, a strict "key smaller" update keeps the lowest L among ties.  The
// valid list is split into parts so that few candidates still fill the chip;
// a final pass reduces the per-part winners lexicographically.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "ct_host.h"

namespace {

constexpr int kBlock = 256;
constexpr int kTileRows = 1024;        // rows per LDS tile
constexpr uint32_t kScanBlocks = 2048; // blocks launched for the scan
constexpr uint32_t kMinRowsPerPart = 512;
constexpr uint64_t kNoKey = ~0ull;

__device__ __forceinline__ uint32_t ne_bytes(uint32_t x) {
    // 0x80 in every byte of x that is non-zero
    return ((((x & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | x) & 0x80808080u);
}

__device__ __forceinline__ uint32_t job_gen(const RepairJob& j) { return j.d_gen ? *j.d_gen : j.gen_value; }

// How the scan splits its work for `count` candidates (same on both kernels).
__device__ __forceinline__ void scan_shape(uint32_t count, uint64_t n_valid, uint32_t* n_cblk, uint32_t* parts) {
    uint32_t nc = (count + kBlock - 1) / kBlock;
    if (nc == 0) nc = 1;
    uint32_t p = kScanBlocks / nc;          // n_cblk * parts never exceeds the launched grid
    uint64_t pmax = (n_valid + kMinRowsPerPart - 1) / kMinRowsPerPart;
    if (pmax < 1) pmax = 1;
    if (p > pmax) p = (uint32_t)pmax;
    if (p < 1) p = 1;
    *n_cblk = nc;
    *parts = p;
}

__global__ __launch_bounds__(kBlock) void k_repair_prep(RepairJob J, uint32_t n_vals, uint32_t* __restrict__ list,
                                                        uint32_t* __restrict__ count) {
    extern __shared__ int64_t lds_vals[];
    const DevSpace& S = J.S;
    for (uint32_t i = threadIdx.x; i < n_vals; i += blockDim.x) lds_vals[i] = S.values[i];
    __syncthreads();
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool in = i < J.n;
    Row c;
    if (in) row_load(c, J.rows + i * S.R, S.R);
    else
        for (int q = 0; q < CT_DMAX / 4; ++q) c.w[q] = 0;
    bool dom = in && row_in_domain(S, c);
    Row e = c;
    if (!dom)
        for (int q = 0; q < CT_DMAX / 4; ++q) e.w[q] = 0;
    bool valid = ct_eval(S, 0, S.n_cons, e, lds_vals) && dom;
    bool act = in && (J.apply == nullptr || J.apply[i]);
    bool need = act && (J.metric == CT_HAM1_RANDOM || !valid);
    if (in) {
        row_store(c, J.out_rows + i * S.R, S.R);
        int64_t p = valid ? rank_of(S, row_encode(S, c)) : -1;
        J.out_pos[i] = p < 0 ? 0xFFFFFFFFu : (uint32_t)p;
    }
    // wave-aggregated append
    uint64_t m = __ballot(need);
    if (m) {
        uint32_t lane = threadIdx.x & 63u;
        uint32_t base = 0;
        uint32_t leader = (uint32_t)__ffsll((long long)m) - 1u;
        if (lane == leader) base = atomicAdd(count, (uint32_t)__popcll(m));
        base = __shfl(base, (int)leader, 64);
        if (need) {
            uint32_t below = (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
            list[base + below] = (uint32_t)i;
        }
    }
}

template <int M, int RW>
__global__ __launch_bounds__(kBlock) void k_repair_scan(RepairJob J, const uint32_t* __restrict__ list,
                                                        const uint32_t* __restrict__ count_p,
                                                        uint64_t* __restrict__ part_key,
                                                        uint32_t* __restrict__ part_pos) {
    __shared__ uint32_t tile[kTileRows * RW];
    const DevSpace& S = J.S;
    const uint32_t count = *count_p;
    uint32_t n_cblk, parts;
    scan_shape(count, S.n_valid, &n_cblk, &parts);
    const uint32_t item = blockIdx.x;
    if (count == 0 || item >= n_cblk * parts) return;
    const uint32_t cblk = item / parts, part = item % parts;
    const uint32_t li = cblk * kBlock + threadIdx.x;     // list index of this lane's candidate
    const bool active = li < count;
    const uint32_t ci = active ? list[li] : 0u;          // candidate index

    uint32_t c[RW], pv[RW], nx[RW];
    const uint32_t* cr = reinterpret_cast<const uint32_t*>(J.rows + (uint64_t)ci * S.R);
#pragma unroll
    for (int k = 0; k < RW; ++k) c[k] = cr[k];
    bool adj_is_sa = true;
    int32_t X[RW * 4];
    uint32_t who = 0, gen = 0;
    if constexpr (M == CT_TIER_EUCLID || M == CT_TIER_RANDOM) {
        // nearest present value index below/above each digit ("adjacent" rule)
#pragma unroll
        for (int k = 0; k < RW; ++k) { pv[k] = 0; nx[k] = 0; }
#pragma unroll
        for (int j = 0; j < RW * 4; ++j) {
            uint32_t d = (c[j >> 2] >> ((j & 3) * 8)) & 0xFFu;
            uint32_t p = d, n = d;
            if ((uint32_t)j < S.D) {
                p = S.prevnext[((uint32_t)j * 256u + d) * 2u + 0u];
                n = S.prevnext[((uint32_t)j * 256u + d) * 2u + 1u];
                // the two rules agree on parameter j unless a present value exists below (above)
                // d while d-1 (d+1) itself never occurs in a solution; "none" is 0xFF, which no
                // digit can equal
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
    }

    uint64_t best = kNoKey;
    uint32_t best_pos = 0xFFFFFFFFu;
    const uint64_t v0 = (uint64_t)part * S.n_valid / parts, v1 = (uint64_t)(part + 1) * S.n_valid / parts;
    const uint32_t* rows32 = reinterpret_cast<const uint32_t*>(S.rows);
    for (uint64_t t0 = v0; t0 < v1; t0 += kTileRows) {
        const uint32_t nt = (uint32_t)std::min<uint64_t>(kTileRows, v1 - t0);
        __syncthreads();
        for (uint32_t q = threadIdx.x; q < nt * RW; q += kBlock) tile[q] = rows32[t0 * RW + q];
        __syncthreads();
        if (!__any(active)) continue;
        for (uint32_t r = 0; r < nt; ++r) {
            uint32_t v[RW];
#pragma unroll
            for (int k = 0; k < RW; ++k) v[k] = tile[r * RW + k];
            const uint32_t pos = (uint32_t)(t0 + r);
            uint64_t key;
            if constexpr (M == CT_HAMMING) {
                uint32_t h = 0;
#pragma unroll
                for (int k = 0; k < RW; ++k) h += __popc(ne_bytes(c[k] ^ v[k]));
                key = h;
            } else if constexpr (M == CT_INDEX_L1) {
                uint32_t s = 0;
#pragma unroll
                for (int k = 0; k < RW; ++k) s = __builtin_amdgcn_sad_u8(c[k], v[k], s);
                key = s;
            } else {
                uint32_t h = 0, s = 0;
#pragma unroll
                for (int k = 0; k < RW; ++k) {
                    h += __popc(ne_bytes(c[k] ^ v[k]));
                    s = __builtin_amdgcn_sad_u8(c[k], v[k], s);
                }
                if constexpr (M == CT_HAM1_RANDOM) {
                    if (h != 1u) continue;
                    uint64_t L = S.lin[pos];
                    U4 o = ct_philox(J.seed, who, gen, (PUR_MUT_KEY << 24) | (uint32_t)((L >> 32) & 0xFFFFFFu),
                                     (uint32_t)L);
                    key = o.x;
                } else {
                    uint32_t tier;
                    if (s == h) {
                        tier = 0;                         // every differing digit differs by exactly 1
                    } else {
                        bool adj = false;
                        if (!adj_is_sa) {
                            adj = true;
#pragma unroll
                            for (int k = 0; k < RW; ++k) {
                                uint32_t eq = (~ne_bytes(v[k] ^ c[k]) | ~ne_bytes(v[k] ^ pv[k]) |
                                               ~ne_bytes(v[k] ^ nx[k])) & 0x80808080u;
                                adj &= eq == 0x80808080u;
                            }
                        }
                        tier = adj ? 1u : (h == 1u ? 2u : 3u);
                    }
                    const uint64_t btier = best >> 62;
                    if (tier > btier) continue;
                    uint64_t sub;
                    if (tier == 3u) {
                        sub = h;
                    } else if constexpr (M == CT_TIER_EUCLID) {
                        uint64_t d2 = 0;
#pragma unroll
                        for (int j = 0; j < RW * 4; ++j) {
                            int64_t cen = (int64_t)((((v[j >> 2] >> ((j & 3) * 8)) & 0xFFu) * 2u + 1u) << 15);
                            int64_t d = (int64_t)X[j] - cen;
                            d2 += (uint64_t)(d * d);
                        }
                        // padding digits: X = 0, centre = 2^15, same constant for every row
                        sub = d2;
                    } else {
                        uint64_t L = S.lin[pos];
                        U4 o = ct_philox(J.seed, who, gen,
                                         (PUR_REPAIR_KEY << 24) | (uint32_t)((L >> 32) & 0xFFFFFFu), (uint32_t)L);
                        sub = o.x;
                    }
                    key = ((uint64_t)tier << 62) | sub;
                }
            }
            if (key < best) {
                best = key;
                best_pos = pos;
            }
        }
    }
    if (active) {
        part_key[(uint64_t)part * count + li] = best;
        part_pos[(uint64_t)part * count + li] = best_pos;
    }
}

__global__ __launch_bounds__(kBlock) void k_repair_finish(RepairJob J, const uint32_t* __restrict__ list,
                                                          const uint32_t* __restrict__ count_p,
                                                          const uint64_t* __restrict__ part_key,
                                                          const uint32_t* __restrict__ part_pos) {
    const DevSpace& S = J.S;
    const uint32_t count = *count_p;
    uint32_t n_cblk, parts;
    scan_shape(count, S.n_valid, &n_cblk, &parts);
    for (uint32_t li = blockIdx.x * blockDim.x + threadIdx.x; li < count; li += gridDim.x * blockDim.x) {
        uint64_t bk = kNoKey;
        uint32_t bp = 0xFFFFFFFFu;
        for (uint32_t p = 0; p < parts; ++p) {
            uint64_t k = part_key[(uint64_t)p * count + li];
            uint32_t q = part_pos[(uint64_t)p * count + li];
            if (k < bk || (k == bk && q < bp)) { bk = k; bp = q; }
        }
        const uint32_t ci = list[li];
        if (bp != 0xFFFFFFFFu) {
            Row r;
            row_load(r, S.rows + (uint64_t)bp * S.R, S.R);
            row_store(r, J.out_rows + (uint64_t)ci * S.R, S.R);
            J.out_pos[ci] = bp;
        }
    }
}

template <int M>
void launch_scan_w(const RepairJob& J, uint32_t RW, const RepairScratch& rs, hipStream_t st) {
    // items = n_cblk * parts <= max(kScanBlocks, n_cblk) for every count <= J.n
    const uint64_t ncb = (J.n + kBlock - 1) / kBlock;
    dim3 g((uint32_t)std::max<uint64_t>(kScanBlocks, ncb)), b(kBlock);
    switch (RW) {
    case 1: hipLaunchKernelGGL((k_repair_scan<M, 1>), g, b, 0, st, J, rs.list, rs.count, rs.part_key, rs.part_pos); break;
    case 2: hipLaunchKernelGGL((k_repair_scan<M, 2>), g, b, 0, st, J, rs.list, rs.count, rs.part_key, rs.part_pos); break;
    case 4: hipLaunchKernelGGL((k_repair_scan<M, 4>), g, b, 0, st, J, rs.list, rs.count, rs.part_key, rs.part_pos); break;
    default: hipLaunchKernelGGL((k_repair_scan<M, 8>), g, b, 0, st, J, rs.list, rs.count, rs.part_key, rs.part_pos); break;
    }
}

}  // namespace

int repair_scratch_alloc(RepairScratch& rs, uint64_t cap, uint32_t max_parts, hipStream_t st) {
    (void)max_parts;
    rs.cap = cap ? cap : 1;
    // per-part winners: parts * count <= (kScanBlocks + ceil(count/kBlock)) * kBlock entries
    uint64_t slots = ((uint64_t)kScanBlocks + (rs.cap + kBlock - 1) / kBlock) * kBlock;
    rs.max_parts = kScanBlocks;
    CT_HIP(hipMallocAsync((void**)&rs.list, rs.cap * sizeof(uint32_t), st));
    CT_HIP(hipMallocAsync((void**)&rs.count, sizeof(uint32_t), st));
    CT_HIP(hipMallocAsync((void**)&rs.part_key, slots * sizeof(uint64_t), st));
    CT_HIP(hipMallocAsync((void**)&rs.part_pos, slots * sizeof(uint32_t), st));
    return CT_OK;
}

void repair_scratch_free(RepairScratch& rs, hipStream_t st) {
    if (rs.list) (void)hipFreeAsync(rs.list, st);
    if (rs.count) (void)hipFreeAsync(rs.count, st);
    if (rs.part_key) (void)hipFreeAsync(rs.part_key, st);
    if (rs.part_pos) (void)hipFreeAsync(rs.part_pos, st);
    rs = RepairScratch{};
}

int launch_repair(const ct_space* s, const RepairJob& J, RepairScratch& rs, hipStream_t st) {
    if (J.n == 0) return CT_OK;
    if (J.n > rs.cap) return ct_fail(CT_EINVAL, "repair: more candidates than the scratch holds");
    CT_HIP(hipMemsetAsync(rs.count, 0, sizeof(uint32_t), st));
    uint32_t gp = (uint32_t)std::min<uint64_t>((J.n + kBlock - 1) / kBlock, 0x7FFFFFFFull);
    hipLaunchKernelGGL(k_repair_prep, dim3(gp), dim3(kBlock), s->lds_values_bytes, st, J,
                       (uint32_t)s->values.size(), rs.list, rs.count);
    const uint32_t RW = s->R / 4;
    switch (J.metric) {
    case CT_HAMMING: launch_scan_w<CT_HAMMING>(J, RW, rs, st); break;
    case CT_INDEX_L1: launch_scan_w<CT_INDEX_L1>(J, RW, rs, st); break;
    case CT_TIER_EUCLID: launch_scan_w<CT_TIER_EUCLID>(J, RW, rs, st); break;
    case CT_TIER_RANDOM: launch_scan_w<CT_TIER_RANDOM>(J, RW, rs, st); break;
    default: launch_scan_w<CT_HAM1_RANDOM>(J, RW, rs, st); break;
    }
    uint32_t gf = (uint32_t)std::min<uint64_t>((J.n + kBlock - 1) / kBlock, 4096);
    hipLaunchKernelGGL(k_repair_finish, dim3(gf), dim3(kBlock), 0, st, J, rs.list, rs.count, rs.part_key,
                       rs.part_pos);
    CT_HIP(hipGetLastError());
    return CT_OK;
}
