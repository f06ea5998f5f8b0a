// Repair of invalid configurations (Section IV-A neighbour rules; Alg. 1
// Repair, Alg. 2, Alg. 3) and the GA mutation to a random valid Hamming
// neighbour (Section IV-D), as argmin scans over the ascending valid list.
//
// For every candidate c that needs it, the scan returns
//     argmin_{v in V} (k(c, v), L(v))
// with a metric-specific key k.  The work is a branch-and-bound scan:
//   - the valid list is cut into 64-row blocks, each with a per-parameter
//     bounding box [min, max] of its value indices, and the boxes into chunks
//     of 64 with a box over each chunk (both built with the space);
//   - one wave owns one (candidate, part of the list) item and holds the
//     candidate wave-uniform; its lanes first test 64 of the part's chunk
//     boxes at once against the candidate's current bound (a lower bound of
//     the key over the box), then the row boxes the part owns in up to 8
//     surviving chunks, then evaluate each surviving block with one row per
//     lane (the parts of a candidate share each chunk's boxes, so a dense
//     region is split between them);
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
// one-wave plan (run by the last block of the kernel that listed the
// candidates, or as a launch of its own before the fallback) turns the per-set
// candidate counts into the item space of each scan without a round trip to
// the host.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "ct_host.h"
#include "repair_plan.h"

namespace {

constexpr int kBlock = 256;
// Scan blocks are single waves: items differ in length, and a block's resources are only freed
// when its last wave ends, so a wave that finishes early in a larger block would hold its slot
// idle (one-wave blocks: the gemm13 job's scan 59.0 -> 56.9 us)
constexpr uint32_t kScanWavesPerBlock = 1;
constexpr uint64_t kNoKey = ~0ull;
constexpr uint32_t kNoPos = 0xFFFFFFFFu;
constexpr uint64_t kTier3 = 3ull << 62;
constexpr uint32_t kMaxSets = 4096;
constexpr uint32_t kFallbackMinSub = 16;   // least boxes per part of the fallback pass, at most
constexpr uint32_t kNumClasses = kRepairClasses;

__device__ __forceinline__ uint32_t ne_bytes(uint32_t x) {
    // 0x80 in every byte of x that is non-zero
    return ((((x & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | x) & 0x80808080u);
}

// 0x80 in every byte where x < y (unsigned bytes): z's high bit says whether the low seven bits
// of x reach those of y (no borrow crosses a byte), the high bits of x and y decide the rest
__device__ __forceinline__ uint32_t lt_bytes(uint32_t x, uint32_t y) {
    const uint32_t z = (x | 0x80808080u) - (y & 0x7F7F7F7Fu);
    return ((~x & y) | (~(x ^ y) & ~z)) & 0x80808080u;
}

// 0xFF in every byte whose high bit is set in m (m holds only 0x80 or 0x00 bytes)
__device__ __forceinline__ uint32_t byte_mask(uint32_t m) { return m | (m - (m >> 7)); }

__device__ __forceinline__ uint32_t wave_lane() { return threadIdx.x & 63u; }
__device__ __forceinline__ uint32_t uni(uint32_t x) { return __builtin_amdgcn_readfirstlane(x); }

// One step of a minimum over lanes through a DPP permutation (no LDS round trip): lanes of the
// rows in ROWS take the minimum of their value and the permuted one, the others keep theirs.
template <int CTRL, int ROWS = 0xF>
__device__ __forceinline__ uint64_t dpp_min_u64(uint64_t v) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp((int)(uint32_t)v, (int)(uint32_t)v, CTRL, ROWS, 0xF, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp((int)(uint32_t)(v >> 32), (int)(uint32_t)(v >> 32), CTRL,
                                                             ROWS, 0xF, false);
    const uint64_t w = ((uint64_t)hi << 32) | lo;
    return w < v ? w : v;
}

// Minimum over the 64 lanes, wave-uniform result; every lane must be active.  Within each row of
// 16 lanes the two quad swaps, then the half-row and row mirrors, pair every lane with one whose
// partial minimum covers the other lanes; then row 1 takes row 0's minimum and row 3 row 2's
// (lane 15 of a row broadcast to the next row), row 3 takes row 1's (lane 31 broadcast to rows 2
// and 3), and lane 63 holds the wave's.  Cross-lane shuffles through LDS cost a dependent LDS round
// trip per step, and this runs once per opened box (the gemm13 job's scan 57.5 -> 53.4 us).
__device__ __forceinline__ uint64_t wave_min_u64(uint64_t v) {
    v = dpp_min_u64<0xB1>(v);          // quad_perm [1, 0, 3, 2]
    v = dpp_min_u64<0x4E>(v);          // quad_perm [2, 3, 0, 1]
    v = dpp_min_u64<0x141>(v);         // row_half_mirror
    v = dpp_min_u64<0x140>(v);         // row_mirror
    v = dpp_min_u64<0x142, 0xA>(v);    // row_bcast:15 into rows 1 and 3
    v = dpp_min_u64<0x143, 0xC>(v);    // row_bcast:31 into rows 2 and 3
    return ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), 63) << 32) |
           (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, 63);
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

// The same for a wave-uniform item, every lane active: each round the lanes read 64 evenly spaced
// offsets of the remaining range at once and a ballot narrows it 64-fold, so up to 64 sets cost
// one memory round trip instead of one per halving (256 sets: two instead of eight).
__device__ __forceinline__ uint32_t find_set_wave(const uint32_t* off, uint32_t n, uint32_t item) {
    const uint32_t lane = threadIdx.x & 63u;
    uint32_t lo = 0, hi = n;                  // off[lo] <= item < off[hi]
    while (hi - lo > 1) {
        const uint32_t step = (hi - lo + 63u) >> 6;
        const uint32_t s = lo + lane * step;
        const bool ok = s < hi && off[s] <= item;     // lane 0 (s = lo) always holds
        const uint64_t b = __ballot(ok);
        const uint32_t last = 63u - (uint32_t)__builtin_clzll(b);
        lo += last * step;
        hi = min(hi, lo + step);
    }
    return lo;
}

__device__ __forceinline__ bool tiered_metric(uint32_t m) { return m == CT_TIER_EUCLID || m == CT_TIER_RANDOM; }

// ---------------------------------------------------------------------------
// Per-candidate state, wave-uniform (the candidate is the same in every lane).
// ---------------------------------------------------------------------------
template <int M, int RW>
struct Cand {
    // (32-byte rows keep the even stride: 255 values x 33 entries would not fit in 64 KiB of LDS)
    static constexpr uint32_t kTabStride = RW < 8 ? RW * 4 + 1 : RW * 4;
    uint32_t c[RW];
    uint32_t pv[RW], nx[RW];     // nearest present value index below / above each digit
    bool adj_is_sa;
    // TIER_EUCLID: squared distance of the particle to each value centre, T[v * (4RW + 1) + j] =
    // (X_j - (v * 2^16 + 2^15))^2 (0 for the padding digits j >= D) in this wave's LDS slice, so
    // every digit of a row is looked up unconditionally.  The odd row stride (in 8-byte entries)
    // puts the entries of one digit for different values in different LDS bank pairs: with a
    // stride of 4RW = 16 entries (128 bytes) every lane reading digit j hit the same banks.  And
    // the value index s_j whose centre
    // is nearest to X_j (the squared distance is convex in v, so over a box's range [a, b] its
    // minimum is at clamp(s_j, a, b))
    const CT_LDS uint64_t* tab;
    const CT_GLOBAL uint64_t* lin;   // linear indices of the valid list
    uint32_t D;
    uint32_t s[RW];
    uint32_t who, gen;
    uint64_t seed;

    __device__ __forceinline__ void load(const RepairSet& J, const CT_GLOBAL DevSpace* Sg, uint32_t ci, CT_LDS uint64_t* lds_tab) {
        const CT_GLOBAL DevSpace& S = *Sg;
        const CT_GLOBAL uint32_t* cr = gptr(reinterpret_cast<const uint32_t*>(J.rows + (uint64_t)ci * S.R));
        lin = gptr(S.lin);
        D = S.D;
#pragma unroll
        for (int k = 0; k < RW; ++k) {
            // bytes past the last parameter are padding: force them to zero
            const int live = (int)S.D - 4 * k;
            const uint32_t keep = live >= 4 ? 0xFFFFFFFFu : (live <= 0 ? 0u : ((1u << (8 * live)) - 1u));
            c[k] = uni(cr[k] & keep);
        }
        adj_is_sa = true;
        // Per-digit tables are looked up by lane (lane j: parameter j), so all digits cost one
        // round trip to memory instead of one dependent round trip each.
        const uint32_t lane = wave_lane();
        if constexpr (M == CT_TIER_EUCLID || M == CT_TIER_RANDOM) {
            uint32_t dj = 0;
#pragma unroll
            for (int k = 0; k < RW; ++k) dj = (lane >> 2) == (uint32_t)k ? (c[k] >> ((lane & 3u) * 8u)) & 0xFFu : dj;
            // (previous, next) present value index of digit j, low byte first; 0 past the last parameter
            const uint32_t pnj = lane < D ? (uint32_t)gptr(reinterpret_cast<const uint16_t*>(S.prevnext))[lane * 256u + dj] : 0u;
            const uint32_t pj = pnj & 0xFFu, nj = pnj >> 8;
            // the two rules agree on parameter j unless a present value lies below (above) d while
            // d-1 (d+1) itself never occurs in a solution; "none" is 0xFF, which no digit equals
            const bool ok = lane >= D || ((pj == dj - 1u || pj == 0xFFu) && (nj == dj + 1u || nj == 0xFFu));
            adj_is_sa = __ballot(!ok) == 0ull;
#pragma unroll
            for (int k = 0; k < RW; ++k) {
                uint32_t pw = 0, nw = 0;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const uint32_t v = (uint32_t)__builtin_amdgcn_readlane((int)pnj, k * 4 + q);
                    pw |= (v & 0xFFu) << (q * 8);
                    nw |= (v >> 8) << (q * 8);
                }
                pv[k] = pw;
                nx[k] = nw;
            }
        }
        if constexpr (M == CT_TIER_EUCLID) {
            const CT_GLOBAL int32_t* xp = gptr(J.pos_q16 + (uint64_t)ci * S.D);
            const int32_t xj = lane < D ? xp[lane] : 0;
            const int32_t hj = lane < D ? (int32_t)S.radix[lane] - 1 : 0;
            constexpr uint32_t TS = kTabStride;
            const uint32_t n_tab = S.max_radix * TS;
            // a uniform trip count keeps every lane active for the shuffle
            for (uint32_t e0 = 0; e0 < n_tab; e0 += 64) {
                const uint32_t e = e0 + lane;
                const uint32_t v = e / TS, j = e % TS;
                const int32_t x = __shfl(xj, (int)j, 64);
                const int64_t d = (int64_t)x - (int64_t)((v << 16) + 32768u);
                if (e < n_tab) lds_tab[e] = j < D ? (uint64_t)(d * d) : 0ull;
            }
            const uint32_t sj = lane < D ? (uint32_t)min(max(xj >> 16, 0), hj) : 0u;
#pragma unroll
            for (int k = 0; k < RW; ++k) {
                uint32_t w = 0;
#pragma unroll
                for (int q = 0; q < 4; ++q) w |= (uint32_t)__builtin_amdgcn_readlane((int)sj, k * 4 + q) << (q * 8);
                s[k] = w;
            }
            tab = lds_tab;
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
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
                const uint64_t L = lin[pos];
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
                    for (int j = 0; j < RW * 4; ++j)
                        d2 += tab[((v[j >> 2] >> ((j & 3) * 8)) & 0xFFu) * kTabStride + (uint32_t)j];
                    return ((uint64_t)tier << 62) | d2;
                } else {
                    const uint64_t L = lin[pos];
                    U4 o = ct_philox(seed, who, gen, (PUR_REPAIR_KEY << 24) | (uint32_t)((L >> 32) & 0xFFFFFFu),
                                     (uint32_t)L);
                    return ((uint64_t)tier << 62) | o.x;
                }
            }
        }
    }

    // lower bound of key() over every row inside the box [lo, hi]; where it is at least `bound`
    // (the box cannot win) any value at least `bound` may be returned
    __device__ __forceinline__ uint64_t bound_box(const uint32_t* lo32, const uint32_t* hi32, uint32_t D,
                                                  uint64_t bound) const {
        if constexpr (M == CT_INDEX_L1) {
            // per digit, the distance from c to [a, b] (a <= b) is (|c - a| + |c - b| - (b - a)) / 2,
            // and v_sad_u8 sums absolute byte differences four digits at a time
            uint32_t both = 0, span = 0;
#pragma unroll
            for (int k = 0; k < RW; ++k) {
                both = __builtin_amdgcn_sad_u8(c[k], lo32[k], both);
                both = __builtin_amdgcn_sad_u8(c[k], hi32[k], both);
                span = __builtin_amdgcn_sad_u8(hi32[k], lo32[k], span);
            }
            return (both - span) >> 1;
        }
        // Four digits per 32-bit word (SWAR): per-byte comparisons give 0x80 in the bytes where
        // they hold.  Padding digits are 0 in the candidate and in both box rows: they add nothing.
        uint32_t miss = 0, far = 0;
        bool adj_ok = true;
#pragma unroll
        for (int k = 0; k < RW; ++k) {
            const uint32_t a = lo32[k], b = hi32[k], ck = c[k];
            const uint32_t out = lt_bytes(ck, a) | lt_bytes(b, ck);          // digit outside [a, b]
            miss += __popc(out);
            if constexpr (M == CT_TIER_EUCLID || M == CT_TIER_RANDOM) {
                // more than one index away: c + 1 < a or b + 1 < c (digits are at most 254, so
                // adding 1 to every byte never carries)
                far += __popc(lt_bytes(ck + 0x01010101u, a) | lt_bytes(b + 0x01010101u, ck));
                if (!adj_is_sa) {
                    // an adjacent value inside the box for every digit outside it; "none" is 0xFF,
                    // above every box bound (radices are at most 255)
                    const uint32_t p_in = ~(lt_bytes(pv[k], a) | lt_bytes(b, pv[k]));
                    const uint32_t n_in = ~(lt_bytes(nx[k], a) | lt_bytes(b, nx[k]));
                    adj_ok &= (out & ~(p_in | n_in)) == 0u;
                }
            }
        }
        if constexpr (M == CT_HAMMING) return miss;
        else if constexpr (M == CT_HAM1_RANDOM) return miss <= 1u ? 0ull : kNoKey;
        else {
            const uint64_t tier = far == 0u ? 0ull                      // strictly adjacent rows possible
                                : (!adj_is_sa && adj_ok) ? 1ull         // adjacent rows possible
                                : miss <= 1u ? 2ull                     // Hamming-1 rows possible
                                : 3ull;
            if (tier == 3u) return kTier3;
            if constexpr (M == CT_TIER_EUCLID) {
                // the squared distance only matters for boxes whose tier can still win
                if ((tier << 62) >= bound) return tier << 62;
                // squared distance from the particle to the nearest value centre inside [a, b]:
                // the table at clamp(s_j, a_j, b_j)
                uint64_t e2 = 0;
#pragma unroll
                for (int k = 0; k < RW; ++k) {
                    const uint32_t a = lo32[k], b = hi32[k];
                    const uint32_t m_lo = byte_mask(lt_bytes(s[k], a));
                    const uint32_t t1 = (a & m_lo) | (s[k] & ~m_lo);
                    const uint32_t m_hi = byte_mask(lt_bytes(b, t1));
                    const uint32_t t = (b & m_hi) | (t1 & ~m_hi);
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        e2 += tab[((t >> (q * 8)) & 0xFFu) * kTabStride + (uint32_t)(k * 4 + q)];
                }
                return (tier << 62) | e2;
            } else {
                return tier << 62;
            }
        }
    }
};

template <int CTRL, int ROWS = 0xF>
__device__ __forceinline__ void dpp_lexmin_step(uint64_t& k, uint32_t& p) {
    const uint32_t klo = (uint32_t)__builtin_amdgcn_update_dpp((int)(uint32_t)k, (int)(uint32_t)k, CTRL, ROWS, 0xF, false);
    const uint32_t khi = (uint32_t)__builtin_amdgcn_update_dpp((int)(uint32_t)(k >> 32), (int)(uint32_t)(k >> 32), CTRL,
                                                              ROWS, 0xF, false);
    const uint32_t pq = (uint32_t)__builtin_amdgcn_update_dpp((int)p, (int)p, CTRL, ROWS, 0xF, false);
    const uint64_t kq = ((uint64_t)khi << 32) | klo;
    if (kq < k || (kq == k && pq < p)) { k = kq; p = pq; }
}

// Lexicographic (key, position) minimum over the wave, every lane gets the result: the same steps
// as wave_min_u64 on the pairs.  Every lane must be active.
__device__ __forceinline__ void wave_lexmin(uint64_t& k, uint32_t& p) {
    dpp_lexmin_step<0xB1>(k, p);
    dpp_lexmin_step<0x4E>(k, p);
    dpp_lexmin_step<0x141>(k, p);
    dpp_lexmin_step<0x140>(k, p);
    dpp_lexmin_step<0x142, 0xA>(k, p);
    dpp_lexmin_step<0x143, 0xC>(k, p);
    k = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(k >> 32), 63) << 32) |
        (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)k, 63);
    p = (uint32_t)__builtin_amdgcn_readlane((int)p, 63);
}

// rank_dir on a descriptor typed as device memory, for a wave-uniform L: lanes 0-7 read the words
// of L's 8-word block up to L's word at once, so the rank costs one round trip after the
// directory instead of one per word.
__device__ __forceinline__ uint64_t rank_g(const CT_GLOBAL DevSpace* S, uint64_t L) {
    if (L >= S->N) return S->n_valid;
    const uint64_t w = L >> 6;
    const uint32_t lane = wave_lane();
    const uint64_t q = (w & ~7ull) + (lane & 7u);
    uint32_t cnt = 0;
    if (lane < 8 && q <= w) {
        const uint64_t word = gptr(S->words)[q];
        cnt = (uint32_t)__popcll(q < w ? word : word & ((1ull << (L & 63u)) - 1ull));
    }
    const uint64_t base = gptr(S->grp_off)[w >> 6] + gptr(S->dir8)[w >> 3];
    cnt += __shfl_xor(cnt, 1, 64);
    cnt += __shfl_xor(cnt, 2, 64);
    cnt += __shfl_xor(cnt, 4, 64);
    return base + uni(cnt);
}

// One (candidate, part) item: the lexicographic (key, position) minimum over the rows of the
// part's boxes that cannot be ruled out.
//   - bk is an exclusive bound (keys below it are wanted); it starts from the 64 valid rows
//     around the candidate's place in linear-index order, and from tier 3 for the tiered
//     metrics (their fallback pass handles candidates without a tier 0-2 neighbour);
//   - boxes are visited in position order, lanes over 64 boxes at a time: a box is opened only
//     if its lower bound is below bk, one row per lane, and the rows of the next surviving box
//     load while the current one is evaluated;
//   - after each box bk drops to the smallest key found, so later boxes (higher positions) with
//     an equal bound are skipped: ties go to the lowest position.
// Always inlined: with two kernels calling it the compiler would otherwise emit a call, whose
// register convention costs the tiered metrics twice the VGPRs plus stack spills.
template <int M, int RW>
__device__ __forceinline__ void scan_item(const RepairSet& J, const DevSpace& S, const uint32_t* list, const uint64_t* list_ins,
                          uint32_t li, uint32_t part, uint32_t parts, CT_LDS uint64_t* lds_tab,
                          unsigned long long* opened) {
    const uint32_t lane = wave_lane();
    const CT_GLOBAL DevSpace* Sg = gptr(&S);
    const uint32_t ci = uni(gld(list + li));
    const uint64_t Lc = gld(list_ins + li);
    const CT_GLOBAL uint32_t* rows32 = gptr(reinterpret_cast<const uint32_t*>(Sg->rows));
    const CT_GLOBAL uint32_t* box32 = gptr(reinterpret_cast<const uint32_t*>(Sg->boxes));
    const CT_GLOBAL uint32_t* chunk32 = gptr(reinterpret_cast<const uint32_t*>(Sg->chunks));
    const uint64_t n_valid = Sg->n_valid, n_sub = Sg->n_sub, n_chunk = Sg->n_chunk;
    const uint32_t D = Sg->D;
    // A part owns some boxes of some chunks (64 aligned boxes): with GB the largest power of two
    // (at most 8) dividing `parts` and GC = parts / GB, part p = pc GB + pb owns box pb (mod GB) of
    // every chunk pc (mod GC).  The dense region around a candidate, where most boxes survive the
    // bound, is thus shared by all of its parts instead of falling to the one or two that own its
    // chunks, and a part still visits its rows in position order.
    const uint32_t gb = min(parts & (0u - parts), 8u);
    const uint32_t gc = parts / gb;
    const uint32_t pb = part % gb, pc = part / gb;
    const uint32_t lpc = 64u / gb;                  // lanes per chunk when lanes hold box bounds
    const uint64_t n_mine = pc < n_chunk ? (n_chunk - pc + gc - 1) / gc : 0;   // chunks pc, pc + GC, ...

    Cand<M, RW> C;
    C.load(J, Sg, ci, lds_tab);

    constexpr bool tiered = (M == CT_TIER_EUCLID || M == CT_TIER_RANDOM);
    uint64_t bk = tiered ? kTier3 : kNoKey;
    // the candidate's insertion position in the valid list, found when it was listed: the 64 valid
    // rows around it seed the bound
    const uint64_t ins = ((uint64_t)uni((uint32_t)(Lc >> 32)) << 32) | uni((uint32_t)Lc);
    if (ins != ~0ull) {
        const int64_t q = (int64_t)ins - 32 + (int64_t)lane;
        uint64_t k = kNoKey;
        if (q >= 0 && (uint64_t)q < n_valid) {
            uint32_t v[RW];
#pragma unroll
            for (int w = 0; w < RW; ++w) v[w] = rows32[(uint64_t)q * RW + w];
            k = C.key(S, v, (uint64_t)q, bk);
        }
        k = wave_min_u64(k);
        if (k < bk) bk = k + 1;
    }

    uint64_t mk = bk;                               // this lane's best key (exclusive until a row is found)
    uint32_t mp = kNoPos;
    uint32_t n_box = 0, n_chunk_open = 0;           // measurement only (when `opened` is given)
    for (uint64_t ck = 0; ck < n_mine; ck += 64) {
        // lanes over 64 of the part's chunks: which ones can hold a row below the bound?
        const uint64_t kc = pc + (ck + lane) * gc;
        uint64_t lc = kNoKey;
        if (ck + lane < n_mine) {
            uint32_t lo[RW], hi[RW];
#pragma unroll
            for (int w = 0; w < RW; ++w) {
                lo[w] = chunk32[kc * 2u * RW + w];
                hi[w] = chunk32[kc * 2u * RW + RW + w];
            }
            lc = C.bound_box(lo, hi, D, bk);
        }
        uint64_t mc = __ballot(lc < bk);
        while (mc) {
            // up to GB surviving chunks at a time, lowest first: lane l holds the bound of box
            // pb + GB (l mod 64/GB) of the (l div 64/GB)-th of them, so lanes are in position order
            const uint32_t grp = lane / lpc;
            const uint32_t rk = __builtin_amdgcn_mbcnt_hi((uint32_t)(mc >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mc, 0u));
            const bool take = ((mc >> lane) & 1ull) && rk < gb;
            const uint64_t taken = __ballot(take);
            const uint32_t n_grp = (uint32_t)__popcll(taken);
            mc &= ~taken;
            // lane g < n_grp receives the g-th taken chunk (the others go to lane 63, outside every
            // group that reads), and each lane reads its group's
            const uint32_t tg = (uint32_t)__builtin_amdgcn_ds_permute((int)((take ? rk : 63u) * 4u), (int)lane);
            const uint32_t my_t = (uint32_t)__builtin_amdgcn_ds_bpermute((int)(grp * 4u), (int)tg);
            n_chunk_open += n_grp;
            const uint32_t bx = (uint32_t)(pc + (ck + my_t) * gc) * 64u + pb + gb * (lane % lpc);
            uint64_t lb = kNoKey;
            if (grp < n_grp && bx < n_sub) {
                uint32_t lo[RW], hi[RW];
#pragma unroll
                for (int w = 0; w < RW; ++w) {
                    lo[w] = box32[(uint64_t)bx * 2u * RW + w];
                    hi[w] = box32[(uint64_t)bx * 2u * RW + RW + w];
                }
                lb = C.bound_box(lo, hi, D, bk);
            }
            uint64_t m = __ballot(lb < bk);
            // box of lane t, and the rows of the next surviving box loading while the current
            // one is evaluated
            auto box_of = [&](int t) { return (uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)bx, t); };
            uint32_t nv[RW];
            int tn = m ? __ffsll((long long)m) - 1 : -1;
            auto fetch = [&](int t) {
                const uint64_t q = box_of(t) * 64u + lane;
#pragma unroll
                for (int w = 0; w < RW; ++w) nv[w] = q < n_valid ? rows32[q * RW + w] : 0u;
            };
            if (tn >= 0) fetch(tn);
            while (tn >= 0) {
                const int t = tn;
                m &= ~(1ull << t);
                ++n_box;
                uint32_t v[RW];
#pragma unroll
                for (int w = 0; w < RW; ++w) v[w] = nv[w];
                tn = m ? __ffsll((long long)m) - 1 : -1;
                if (tn >= 0) fetch(tn);
                const uint64_t r = box_of(t) * 64u + lane;
                bool found = false;
                if (r < n_valid) {
                    const uint64_t k = C.key(S, v, r, mk < bk ? mk : bk);
                    if (k < mk) { mk = k; mp = (uint32_t)r; found = true; }
                }
                // the bound (the wave's least key) only moves when some lane found a smaller key
                // in this box: otherwise the minimum and the pruning below would change nothing
                if (__ballot(found)) {
                    const uint64_t wm = wave_min_u64(mk);
                    bk = wm < bk ? wm : bk;
                    if (m) {
                        m &= __ballot(lb < bk);         // drop boxes the tighter bound now rules out
                        if (tn >= 0 && !((m >> tn) & 1ull)) {
                            tn = m ? __ffsll((long long)m) - 1 : -1;
                            if (tn >= 0) fetch(tn);
                        }
                    }
                }
            }
            mc &= __ballot(lc < bk);                    // and chunks
        }
    }
    // lexicographic (key, position) minimum over the wave
    uint64_t k2 = mp == kNoPos ? kNoKey : mk;
    uint32_t p2 = mp;
    wave_lexmin(k2, p2);
    if (lane == 0) {
        J.part_key[(uint64_t)li * parts + part] = k2;
        J.part_pos[(uint64_t)li * parts + part] = p2;
        if (opened) {
            atomicAdd(opened, (unsigned long long)n_box);
            atomicAdd(opened + 1, (unsigned long long)n_chunk_open);
        }
    }
}

// HAM1_RANDOM by enumeration: the Hamming-1 neighbours of c are the configurations that change
// one parameter to another of its values; each is looked up in the validity bitmask and the
// valid ones compete with their Philox key, ties to the lowest linear index (the same minimum
// as a scan of the valid list).  One wave per candidate; lanes over (parameter, value) pairs.
__device__ __forceinline__ void ham1_item(const RepairSet& J, const DevSpace& S, uint32_t li) {
    const uint32_t lane = wave_lane();
    const uint32_t ci = uni(J.list[li]);
    const uint8_t* cr = J.rows + (uint64_t)ci * S.R;
    // linear index over the in-domain digits, and the digits outside their domain
    uint64_t Lp = 0;
    uint32_t bad = 0, bad_j = 0;
    for (uint32_t j = 0; j < S.D; ++j) {
        const uint32_t d = cr[j];
        if (d < S.radix[j]) Lp += (uint64_t)d * S.stride[j];
        else { ++bad; bad_j = j; }
    }
    const uint32_t who = J.who ? J.who[ci] : ci;
    const uint32_t gen = J.gen ? *J.gen : J.gen_value;
    uint64_t bkey = kNoKey, bL = ~0ull;
    const uint32_t n_pairs = S.val_off[S.D - 1] + S.radix[S.D - 1];
    if (bad <= 1) {
        for (uint32_t e = lane; e < n_pairs; e += 64) {
            uint32_t j = 0;
            while (j + 1 < S.D && S.val_off[j + 1] <= e) ++j;
            const uint32_t v = e - S.val_off[j];
            const uint32_t d = cr[j];
            if (v == d || (bad == 1 && j != bad_j)) continue;
            const uint64_t Lq = (d < S.radix[j] ? Lp - (uint64_t)d * S.stride[j] : Lp) + (uint64_t)v * S.stride[j];
            if (!bit_valid(S, Lq)) continue;
            const U4 o = ct_philox(J.seed, who, gen, (PUR_MUT_KEY << 24) | (uint32_t)((Lq >> 32) & 0xFFFFFFu), (uint32_t)Lq);
            if (o.x < bkey || (o.x == bkey && Lq < bL)) { bkey = o.x; bL = Lq; }
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const uint32_t klo = __shfl_xor((uint32_t)bkey, o, 64), khi = __shfl_xor((uint32_t)(bkey >> 32), o, 64);
        const uint32_t llo = __shfl_xor((uint32_t)bL, o, 64), lhi = __shfl_xor((uint32_t)(bL >> 32), o, 64);
        const uint64_t kq = ((uint64_t)khi << 32) | klo, lq = ((uint64_t)lhi << 32) | llo;
        if (kq < bkey || (kq == bkey && lq < bL)) { bkey = kq; bL = lq; }
    }
    if (lane == 0) {
        J.part_key[li] = bkey;
        J.part_pos[li] = bkey == kNoKey ? kNoPos : (uint32_t)rank_dir(S, bL);
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
                                                        const uint32_t* __restrict__ prep_off, PlanArgs pa) {
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
        const uint64_t ins = dom ? rank_dir(S, L) : ~0ull;                 // loads before any store
        const uint32_t pos = valid ? (uint32_t)ins : kNoPos;
        const bool act = J.apply == nullptr || J.apply[i];
        row_store(c, J.out_rows + (uint64_t)i * S.R, S.R);
        J.out_pos[i] = pos;
        if (act && (J.metric == CT_HAM1_RANDOM || !valid)) {
            const uint32_t k = atomicAdd(&J.count[0], 1u);
            J.list[k] = i;
            J.list_ins[k] = ins;
        }
    }
    plan_if_last(sets, n_sets, pa);
}

// The first item of this wave.  Workgroups go to the 8 XCDs in turn (block b to XCD b mod 8), so
// numbering the waves XCD by XCD makes item i, and every item after it in the grid-stride loop,
// run on XCD i mod 8.  With a multiple of 8 parts per candidate (the plan rounds to one) and
// multiples of 8 items before each candidate, item i is a part p of its candidate with
// p mod 8 = i mod 8: every candidate's part p reads the same chunks of the list, so one XCD's L2
// holds the eighth of the list its items read instead of each XCD fetching all of it.  Grids
// that are not a multiple of 8 blocks keep the plain numbering.
__device__ __forceinline__ uint32_t first_item(uint32_t wpb) {
    const uint32_t b = blockIdx.x, w = threadIdx.x >> 6;
    if (gridDim.x & 7u) return b * wpb + w;
    return 8u * (wpb * (b >> 3) + w) + (b & 7u);
}

// A scan launch that plans its own items (SelfPlan::on; at most kSelfPlanSets sets): every wave
// derives the plan of its class with lane s holding set s, in registers, instead of reading the
// offsets a one-wave plan launch wrote, and global wave 0 writes the candidate offsets and this
// class's parts that the finish reads.  The same figures as plan_wave's, one launch fewer.
struct SelfPlan {
    uint32_t on, target_items, min_sub;
};
constexpr uint32_t kSelfPlanSets = 64;

template <int M, int RW>
__global__ __launch_bounds__(kBlock) void k_repair_scan(const RepairSet* __restrict__ sets, uint32_t n_sets,
                                                        RepairPlan plan, uint32_t which, uint32_t tab_stride,
                                                        SelfPlan sp) {
    constexpr uint32_t cls = (uint32_t)M * 4u + (RW == 1 ? 0u : RW == 2 ? 1u : RW == 4 ? 2u : 3u);
    extern __shared__ uint64_t lds_tabs[];
    const uint32_t wpb = blockDim.x / 64;
    CT_LDS uint64_t* lds_tab = (CT_LDS uint64_t*)lds_tabs + (threadIdx.x >> 6) * tab_stride;
    const uint32_t* off = plan.item_off + cls * (n_sets + 1);
    uint32_t total, sp_p = 1, sp_iv = 0, sp_ex = 0;
    if (sp.on) {
        const uint32_t lane = wave_lane();
        uint32_t cls_s = kRepairClasses, cc = 0;
        if (lane < n_sets) {
            cls_s = plan_cls(sets, lane, which);
            cc = plan_count(sets, lane, which);
        }
        const uint32_t c = cls_s == cls ? cc : 0u;
        const uint32_t tot = plan_sum_u32(c);
        const uint32_t gp = tot ? max(sp.target_items / tot, 1u) : 1u;
        if (lane < n_sets) sp_p = plan_parts(sets[lane], cls_s, gp, sp.min_sub);
        const uint32_t w = c * sp_p;
        sp_iv = plan_incl_scan(w);                  // lanes past the sets repeat the total
        sp_ex = sp_iv - w;
        total = (uint32_t)__builtin_amdgcn_readlane((int)sp_iv, 63);
        if (first_item(wpb) == 0) {
            const uint32_t ic = plan_incl_scan(cc);
            if (lane < n_sets) {
                plan.cand_off[lane] = ic - cc;
                if (cls_s == cls) plan.parts[lane] = sp_p;
            }
            if (lane == 63) plan.cand_off[n_sets] = ic;
        }
    } else {
        total = off[n_sets];
    }
    unsigned long long* opened = plan.opened ? plan.opened + 2 * which : nullptr;
    const uint32_t waves = gridDim.x * wpb;
    for (uint32_t item = uni(first_item(wpb)); item < total; item += waves) {
        uint32_t s, parts, local;
        if (sp.on) {
            // the first lane whose inclusive prefix passes the item holds its set
            s = (uint32_t)(__ffsll((long long)__ballot(item < sp_iv)) - 1);
            parts = (uint32_t)__builtin_amdgcn_readlane((int)sp_p, (int)s);
            local = item - (uint32_t)__builtin_amdgcn_readlane((int)sp_ex, (int)s);
        } else {
            s = uni(find_set_wave(off, n_sets, item));
            parts = uni(plan.parts[s]);
            local = item - off[s];
        }
        const RepairSet& J = sets[s];
        const DevSpace& S = *J.S;
        const uint32_t li = local / parts, part = local % parts;
        if constexpr (M == CT_HAM1_RANDOM) {
            ham1_item(J, S, li);
        } else {
            const uint32_t* list = which ? J.fb_list : J.list;
            const uint64_t* list_ins = which ? J.fb_ins : J.list_ins;
            scan_item<M, RW>(J, S, list, list_ins, li, part, parts, lds_tab, opened);
        }
    }
}

// All scanned metrics of one row width in a single launch: the item ranges of the classes in
// `mmask` (bit m: metric m, Hamming to Alg. 3) are laid end to end and every wave takes items of
// any of them, so the latency chains of the classes overlap instead of running one launch after
// another.  Each item runs the same code as in its own class's kernel.  The ranges go in the
// order their items tend to run longest (Alg. 2's distances, the index distance, Alg. 3's keys,
// Hamming), so the longest start first, while the grid is still filling.
__device__ __forceinline__ uint32_t mix_metric(uint32_t q) {
    return q == 0 ? (uint32_t)CT_TIER_EUCLID : q == 1 ? (uint32_t)CT_INDEX_L1 : q == 2 ? (uint32_t)CT_TIER_RANDOM
                                                                                      : (uint32_t)CT_HAMMING;
}

template <int RW>
__global__ __launch_bounds__(kBlock) void k_repair_scan_mix(const RepairSet* __restrict__ sets, uint32_t n_sets,
                                                            RepairPlan plan, uint32_t which, uint32_t tab_stride,
                                                            uint32_t mmask) {
    constexpr uint32_t rwi = RW == 1 ? 0u : RW == 2 ? 1u : RW == 4 ? 2u : 3u;
    extern __shared__ uint64_t lds_tabs[];
    const uint32_t wpb = blockDim.x / 64;
    CT_LDS uint64_t* lds_tab = (CT_LDS uint64_t*)lds_tabs + (threadIdx.x >> 6) * tab_stride;
    uint32_t end[4];
    uint32_t acc = 0;
#pragma unroll
    for (uint32_t q = 0; q < 4; ++q) {
        const uint32_t m = mix_metric(q);
        if (mmask & (1u << m)) acc += plan.item_off[(m * 4u + rwi) * (n_sets + 1) + n_sets];
        end[q] = acc;
    }
    const uint32_t waves = gridDim.x * wpb;
    unsigned long long* opened = plan.opened ? plan.opened + 2 * which : nullptr;
    for (uint32_t item = uni(first_item(wpb)); item < acc; item += waves) {
        const uint32_t q = item < end[0] ? 0u : item < end[1] ? 1u : item < end[2] ? 2u : 3u;
        const uint32_t m = mix_metric(q);
        const uint32_t* off = plan.item_off + (m * 4u + rwi) * (n_sets + 1);
        const uint32_t local_item = item - (q ? end[q - 1] : 0u);
        const uint32_t s = uni(find_set_wave(off, n_sets, local_item));
        const RepairSet& J = sets[s];
        const DevSpace& S = *J.S;
        const uint32_t parts = uni(plan.parts[s]);
        const uint32_t local = local_item - off[s];
        const uint32_t li = local / parts, part = local % parts;
        const uint32_t* list = which ? J.fb_list : J.list;
        const uint64_t* list_ins = which ? J.fb_ins : J.list_ins;
        switch (m) {
        case CT_HAMMING: scan_item<CT_HAMMING, RW>(J, S, list, list_ins, li, part, parts, lds_tab, opened); break;
        case CT_INDEX_L1: scan_item<CT_INDEX_L1, RW>(J, S, list, list_ins, li, part, parts, lds_tab, opened); break;
        case CT_TIER_EUCLID: scan_item<CT_TIER_EUCLID, RW>(J, S, list, list_ins, li, part, parts, lds_tab, opened); break;
        default: scan_item<CT_TIER_RANDOM, RW>(J, S, list, list_ins, li, part, parts, lds_tab, opened); break;
        }
    }
}

// GA mutation of every flagged child in one kernel, one wave per child (the preparation, plan,
// enumeration and finish of a repair pass would be four launches): the child's row (already valid
// after the main pass) is encoded, its single-parameter changes are looked up in the validity
// bitmask, the valid ones compete with their Philox key (ties: lowest linear index), and the
// winner replaces the child.  A child without a valid single-parameter change keeps its row.
__global__ __launch_bounds__(kBlock) void k_mutate(const RepairSet* __restrict__ sets, uint32_t n_sets,
                                                   const uint32_t* __restrict__ off) {
    const uint32_t total = off[n_sets];
    const uint32_t lane = wave_lane();
    const uint32_t waves = gridDim.x * (kBlock / 64);
    for (uint32_t item = uni(blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6)); item < total; item += waves) {
        const uint32_t s = uni(find_set_wave(off, n_sets, item));
        const RepairSet& J = sets[s];
        const uint32_t ci = item - off[s];
        if (!uni(J.apply[ci])) continue;
        const CT_GLOBAL DevSpace& S = *gptr(J.S);
        // lane j < D holds digit j of the child, its radix, stride and first pair index, so the
        // per-pair lookups below are shuffles, not memory round trips
        const uint32_t D = S.D;
        const uint32_t dj = lane < D ? (uint32_t)gld(J.rows + (uint64_t)ci * S.R + lane) : 0u;
        const uint32_t rj = lane < D ? S.radix[lane] : 1u;
        const uint64_t sj = lane < D ? S.stride[lane] : 0ull;
        const uint32_t oj = lane < D ? S.val_off[lane] : 0xFFFFFFFFu;
        // linear index over the in-domain digits, and the digits outside their domain
        const bool in = lane >= D || dj < rj;
        uint64_t Lp = in && lane < D ? (uint64_t)dj * sj : 0ull;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const uint32_t lo = __shfl_xor((uint32_t)Lp, o, 64), hi = __shfl_xor((uint32_t)(Lp >> 32), o, 64);
            Lp += ((uint64_t)hi << 32) | lo;
        }
        const uint64_t out_mask = __ballot(!in);
        const uint32_t bad = (uint32_t)__popcll(out_mask);
        const uint32_t bad_j = out_mask ? (uint32_t)(__ffsll((long long)out_mask) - 1) : 0u;
        const uint32_t who = J.who ? J.who[ci] : ci;
        const uint32_t gen = J.gen ? *J.gen : J.gen_value;
        uint64_t bkey = kNoKey, bL = ~0ull;
        const uint32_t n_pairs = S.val_off[D - 1] + S.radix[D - 1];
        if (bad <= 1) {
            for (uint32_t e0 = 0; e0 < n_pairs; e0 += 64) {     // uniform trip count: shuffles need every lane
                const uint32_t e = e0 + lane;
                // parameter of pair e: the last j with val_off[j] <= e
                uint32_t j = 0;
                for (uint32_t t = 1; t < D; ++t) j += (uint32_t)__builtin_amdgcn_readlane((int)oj, (int)t) <= e ? 1u : 0u;
                const uint32_t d = (uint32_t)__shfl((int)dj, (int)j, 64);
                const uint32_t r = (uint32_t)__shfl((int)rj, (int)j, 64);
                const uint32_t off_j = (uint32_t)__shfl((int)oj, (int)j, 64);
                const uint64_t st = ((uint64_t)(uint32_t)__shfl((int)(uint32_t)(sj >> 32), (int)j, 64) << 32) |
                                    (uint32_t)__shfl((int)(uint32_t)sj, (int)j, 64);
                const uint32_t v = e - off_j;
                if (e >= n_pairs || v == d || (bad == 1 && j != bad_j)) continue;
                const uint64_t Lq = (d < r ? Lp - (uint64_t)d * st : Lp) + (uint64_t)v * st;
                if (!bit_valid(J.S[0], Lq)) continue;
                const U4 o = ct_philox(J.seed, who, gen, (PUR_MUT_KEY << 24) | (uint32_t)((Lq >> 32) & 0xFFFFFFu), (uint32_t)Lq);
                if (o.x < bkey || (o.x == bkey && Lq < bL)) { bkey = o.x; bL = Lq; }
            }
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const uint32_t klo = __shfl_xor((uint32_t)bkey, o, 64), khi = __shfl_xor((uint32_t)(bkey >> 32), o, 64);
            const uint32_t llo = __shfl_xor((uint32_t)bL, o, 64), lhi = __shfl_xor((uint32_t)(bL >> 32), o, 64);
            const uint64_t kq = ((uint64_t)khi << 32) | klo, lq = ((uint64_t)lhi << 32) | llo;
            if (kq < bkey || (kq == bkey && lq < bL)) { bkey = kq; bL = lq; }
        }
        if (bkey != kNoKey) {
            const uint32_t pos = uni((uint32_t)rank_g(gptr(J.S), bL));
            const CT_GLOBAL uint32_t* src = gptr(reinterpret_cast<const uint32_t*>(S.rows + (uint64_t)pos * S.R));
            uint32_t* dst = reinterpret_cast<uint32_t*>(J.out_rows + (uint64_t)ci * S.R);
            if (lane < S.R / 4) dst[lane] = src[lane];
            if (lane == 0) J.out_pos[ci] = pos;
        }
        if (lane == 0 && J.tally) atomicAdd(J.tally, 1ull);
    }
}

// The plan as a launch of its own (one wave).
__global__ __launch_bounds__(64) void k_repair_plan(const RepairSet* __restrict__ sets, uint32_t n_sets, uint32_t which,
                                                    RepairPlan plan, uint32_t class_mask, uint32_t target_items,
                                                    uint32_t min_sub) {
    plan_wave(sets, n_sets, which, plan, class_mask, target_items, min_sub);
}

// Reduce the parts of every candidate (one wave per candidate) and write the result.  In the main
// pass of a tiered set, candidates without a tier 0-2 neighbour go to the fallback list.
__global__ __launch_bounds__(kBlock) void k_repair_finish(const RepairSet* __restrict__ sets, uint32_t n_sets,
                                                          RepairPlan plan, uint32_t which, uint32_t count_tally,
                                                          PlanArgs pa) {
    const uint32_t total = plan.cand_off[n_sets];
    const uint32_t lane = wave_lane();
    const uint32_t waves = gridDim.x * (kBlock / 64);
    for (uint32_t item = uni(blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6)); item < total; item += waves) {
        const uint32_t s = uni(find_set_wave(plan.cand_off, n_sets, item));
        const RepairSet& J = sets[s];
        const DevSpace& S = *J.S;
        const uint32_t parts = plan.parts[s];
        const uint32_t li = item - plan.cand_off[s];
        if (which == 0 && count_tally && li == 0 && lane == 0 && J.tally)
            atomicAdd(J.tally, (unsigned long long)(plan.cand_off[s + 1] - plan.cand_off[s]));
        uint64_t bk = kNoKey;
        uint32_t bp = kNoPos;
        for (uint32_t p = lane; p < parts; p += 64) {
            const uint64_t k = J.part_key[(uint64_t)li * parts + p];
            const uint32_t q = J.part_pos[(uint64_t)li * parts + p];
            if (q != kNoPos && (k < bk || (k == bk && q < bp))) { bk = k; bp = q; }
        }
        wave_lexmin(bk, bp);
        const uint32_t ci = (which ? J.fb_list : J.list)[li];
        if (bp != kNoPos) {
            const uint32_t* src = reinterpret_cast<const uint32_t*>(S.rows + (uint64_t)bp * S.R);
            uint32_t* dst = reinterpret_cast<uint32_t*>(J.out_rows + (uint64_t)ci * S.R);
            if (lane < S.R / 4) dst[lane] = src[lane];
            if (lane == 0) J.out_pos[ci] = bp;
        } else if (which == 0 && tiered_metric(J.metric) && lane == 0) {
            const uint32_t k = atomicAdd(&J.count[1], 1u);
            J.fb_list[k] = ci;
            J.fb_ins[k] = J.list_ins[li];     // the fallback seeds its bound around the same place
        }
    }
    plan_if_last(sets, n_sets, pa);
}

// Waves of one scan launch.  Each launch of the fallback pass (which = 1) scans one class
// (Hamming at one row width), planned for about `items` items (more only when it has more
// candidates than that), so a grid beyond that would only add blocks that find no item.
uint32_t scan_waves(const RepairPasses& rp, uint32_t which) {
    return which ? std::min(rp.tune.grid_waves, rp.tune.items) : rp.tune.grid_waves;
}

// the pass's plan, with the measurement counters when they are on
RepairPlan scan_plan(const RepairPasses& rp) {
    RepairPlan p = rp.plan;
    p.opened = prof_box_counter();
    return p;
}

// The fallback pass plans inside its scans when the sets fit one wave's lanes (its scans are
// single-class launches: the fallback is Hamming only).  The few fallback candidates sit far
// from valid rows, where parts of more than 16 boxes only lengthen the pass, whatever suits the
// main pass.
bool fb_self_planned(const RepairPasses& rp) { return rp.n_sets <= kSelfPlanSets; }
uint32_t fb_min_sub(const RepairPasses& rp) { return std::min(rp.tune.min_sub, kFallbackMinSub); }

template <int M, int RW>
void launch_scan_rw(const RepairPasses& rp, uint32_t which, hipStream_t st) {
    ProfScope ps_(which ? "k_repair_scan_fb" : "k_repair_scan", st);
    // TIER_EUCLID keeps one distance table per wave in LDS
    const uint32_t stride = M == CT_TIER_EUCLID ? std::max<uint32_t>(rp.euclid_tab, 1) : 0;
    const uint32_t wpb = kScanWavesPerBlock;
    const SelfPlan sp{which == 1 && fb_self_planned(rp) ? 1u : 0u, rp.tune.items, fb_min_sub(rp)};
    hipLaunchKernelGGL((k_repair_scan<M, RW>), dim3(std::max<uint32_t>(scan_waves(rp, which) / wpb, 1)), dim3(wpb * 64),
                       (size_t)wpb * stride * 8, st,
                       rp.d_sets, rp.n_sets, scan_plan(rp), which, stride, sp);
}

template <int RW>
void launch_mix_rw(const RepairPasses& rp, uint32_t mmask, uint32_t which, hipStream_t st) {
    ProfScope ps_(which ? "k_repair_scan_fb" : "k_repair_scan", st);
    const uint32_t stride = (mmask & (1u << CT_TIER_EUCLID)) ? std::max<uint32_t>(rp.euclid_tab, 1) : 0;
    const uint32_t wpb = kScanWavesPerBlock;
    hipLaunchKernelGGL((k_repair_scan_mix<RW>), dim3(std::max<uint32_t>(scan_waves(rp, which) / wpb, 1)), dim3(wpb * 64),
                       (size_t)wpb * stride * 8, st, rp.d_sets, rp.n_sets, scan_plan(rp), which, stride, mmask);
}

void launch_mix(const RepairPasses& rp, uint32_t rwi, uint32_t mmask, uint32_t which, hipStream_t st) {
    if (rwi == 0) launch_mix_rw<1>(rp, mmask, which, st);
    else if (rwi == 1) launch_mix_rw<2>(rp, mmask, which, st);
    else if (rwi == 2) launch_mix_rw<4>(rp, mmask, which, st);
    else launch_mix_rw<8>(rp, mmask, which, st);
}

template <int M>
void launch_class_rw(const RepairPasses& rp, uint32_t rwi, uint32_t which, hipStream_t st) {
    if (rwi == 0) launch_scan_rw<M, 1>(rp, which, st);
    else if (rwi == 1) launch_scan_rw<M, 2>(rp, which, st);
    else if (rwi == 2) launch_scan_rw<M, 4>(rp, which, st);
    else launch_scan_rw<M, 8>(rp, which, st);
}

void launch_class(const RepairPasses& rp, uint32_t cls, uint32_t which, hipStream_t st) {
    switch (cls / 4u) {
    case CT_HAMMING: launch_class_rw<CT_HAMMING>(rp, cls % 4u, which, st); break;
    case CT_INDEX_L1: launch_class_rw<CT_INDEX_L1>(rp, cls % 4u, which, st); break;
    case CT_TIER_EUCLID: launch_class_rw<CT_TIER_EUCLID>(rp, cls % 4u, which, st); break;
    case CT_TIER_RANDOM: launch_class_rw<CT_TIER_RANDOM>(rp, cls % 4u, which, st); break;
    default: launch_class_rw<CT_HAM1_RANDOM>(rp, cls % 4u, which, st); break;
    }
}

// Every scan class in `mask`: one after another on st, or, with a fan and more than one class,
// each on an auxiliary stream forked from st and joined back into it (the classes touch disjoint
// sets, so they may overlap).
int launch_scans(const RepairPasses& rp, uint32_t mask, uint32_t which, hipStream_t st) {
    if (rp.tune.mode == kScanFused) {
        // per row width, the scanned metrics together; the enumerated mutation metric alone
        for (uint32_t rwi = 0; rwi < 4; ++rwi) {
            uint32_t mm = 0;
            for (uint32_t m = 0; m < (uint32_t)CT_HAM1_RANDOM; ++m)
                if (mask & (1u << (m * 4u + rwi))) mm |= 1u << m;
            if (which == 0 && __builtin_popcount(mm) > 1) {
                launch_mix(rp, rwi, mm, which, st);
            } else {
                // (the fallback pass is Hamming only; its single-class launches may plan themselves)
                for (uint32_t m2 = mm; m2; m2 &= m2 - 1u) launch_class(rp, (uint32_t)__builtin_ctz(m2) * 4u + rwi, which, st);
            }
            if (mask & (1u << ((uint32_t)CT_HAM1_RANDOM * 4u + rwi)))
                launch_class(rp, (uint32_t)CT_HAM1_RANDOM * 4u + rwi, which, st);
        }
        return CT_OK;
    }
    StreamFan* f = rp.fan;
    if (!f || !f->fork || rp.tune.mode != kScanStreams || __builtin_popcount(mask) < 2) {
        for (uint32_t cls = 0; cls < kNumClasses; ++cls)
            if (mask & (1u << cls)) launch_class(rp, cls, which, st);
        return CT_OK;
    }
    CT_HIP(hipEventRecord(f->fork, st));
    uint32_t used = 0, k = 0;
    for (uint32_t cls = 0; cls < kNumClasses; ++cls) {
        if (!(mask & (1u << cls))) continue;
        const uint32_t l = k++ % StreamFan::kLanes;
        if (!(used & (1u << l))) {
            CT_HIP(hipStreamWaitEvent(f->s[l], f->fork, 0));
            used |= 1u << l;
        }
        launch_class(rp, cls, which, f->s[l]);
    }
    for (uint32_t l = 0; l < (uint32_t)StreamFan::kLanes; ++l) {
        if (!(used & (1u << l))) continue;
        CT_HIP(hipEventRecord(f->join[l], f->s[l]));
        CT_HIP(hipStreamWaitEvent(st, f->join[l], 0));
    }
    return CT_OK;
}

uint32_t finish_grid(uint32_t n) { return std::max<uint32_t>(1, std::min<uint32_t>((n + 3) / 4, 2048)); }

}  // namespace

int fan_create(StreamFan* f) {
    // the fork and join events order work of one device: a device-scope release is enough
    const unsigned flags = hipEventDisableTiming | hipEventReleaseToDevice;
    for (int l = 0; l < StreamFan::kLanes; ++l) {
        CT_HIP(hipStreamCreateWithFlags(&f->s[l], hipStreamNonBlocking));
        CT_HIP(hipEventCreateWithFlags(&f->join[l], flags));
    }
    CT_HIP(hipEventCreateWithFlags(&f->fork, flags));
    return CT_OK;
}

void fan_destroy(StreamFan* f) {
    for (int l = 0; l < StreamFan::kLanes; ++l) {
        if (f->s[l]) (void)hipStreamDestroy(f->s[l]);
        if (f->join[l]) (void)hipEventDestroy(f->join[l]);
        f->s[l] = nullptr;
        f->join[l] = nullptr;
    }
    if (f->fork) (void)hipEventDestroy(f->fork);
    f->fork = nullptr;
}

int repair_plan_alloc(RepairPlan& p, uint32_t n_sets, std::vector<void*>& owned) {
    if (n_sets > kMaxSets) return ct_fail(CT_EINVAL, "repair: at most 4096 candidate sets per launch");
    void* a = nullptr;
    const size_t words = (size_t)(n_sets + 1) * (1 + kNumClasses) + n_sets + 1;
    CT_HIP(hipMalloc(&a, words * sizeof(uint32_t)));
    owned.push_back(a);
    uint32_t* w = static_cast<uint32_t*>(a);
    p.cand_off = w;
    p.item_off = w + (n_sets + 1);
    p.parts = w + (n_sets + 1) * (1 + kNumClasses);
    p.done = p.parts + n_sets;
    p.opened = nullptr;
    CT_HIP(hipMemset(p.done, 0, sizeof(uint32_t)));
    return CT_OK;
}

int launch_mutation(const RepairPasses& rp, hipStream_t st) {
    if (rp.n_sets == 0 || rp.total_n == 0) return CT_OK;
    ProfScope ps_("k_mutate", st);
    const uint32_t g = std::max<uint32_t>(1, std::min<uint32_t>((rp.total_n + kBlock / 64 - 1) / (kBlock / 64), 2048));
    hipLaunchKernelGGL(k_mutate, dim3(g), dim3(kBlock), 0, st, rp.d_sets, rp.n_sets, rp.d_prep_off);
    CT_HIP(hipGetLastError());
    return CT_OK;
}

int launch_repair_prep(const RepairPasses& rp, hipStream_t st) {
    if (rp.n_sets == 0 || rp.total_n == 0) return CT_OK;
    {
        ProfScope ps_("k_repair_zero", st);
        hipLaunchKernelGGL(k_repair_zero, dim3((rp.n_sets + 255) / 256), dim3(256), 0, st, rp.d_sets, rp.n_sets);
    }
    ProfScope ps_("k_repair_prep", st);
    const uint32_t g = std::max<uint32_t>(1, std::min<uint32_t>((rp.total_n + kBlock - 1) / kBlock, 4096));
    hipLaunchKernelGGL(k_repair_prep, dim3(g), dim3(kBlock), 0, st, rp.d_sets, rp.n_sets, rp.d_prep_off, PlanArgs{});
    CT_HIP(hipGetLastError());
    return CT_OK;
}

PlanArgs main_plan(const RepairPasses& rp) {
    return PlanArgs{rp.plan, rp.class_mask, rp.tune.items, rp.tune.min_sub, 0u, 1u};
}

int launch_repair_passes(const RepairPasses& rp, bool zero_counts, hipStream_t st, bool count_tally, bool prep) {
    if (rp.n_sets == 0 || rp.total_n == 0) return CT_OK;
    if (zero_counts) {
        ProfScope ps_("k_repair_zero", st);
        hipLaunchKernelGGL(k_repair_zero, dim3((rp.n_sets + 255) / 256), dim3(256), 0, st, rp.d_sets, rp.n_sets);
    }
    if (prep) {
        // the preparation's last block plans the main scans
        ProfScope ps_("k_repair_prep", st);
        const uint32_t g = std::max<uint32_t>(1, std::min<uint32_t>((rp.total_n + kBlock - 1) / kBlock, 4096));
        hipLaunchKernelGGL(k_repair_prep, dim3(g), dim3(kBlock), 0, st, rp.d_sets, rp.n_sets, rp.d_prep_off,
                           main_plan(rp));
    }
    if (int rc = launch_scans(rp, rp.class_mask, 0, st)) return rc;
    {
        ProfScope ps_("k_repair_finish", st);
        hipLaunchKernelGGL(k_repair_finish, dim3(finish_grid(rp.total_n)), dim3(kBlock), 0, st, rp.d_sets, rp.n_sets,
                           rp.plan, 0u, count_tally ? 1u : 0u, PlanArgs{});
    }
    if (rp.fb_class_mask) {
        if (!fb_self_planned(rp)) {
            // a launch of its own: the finish runs hundreds of blocks, and counting them all
            // costs more than a one-wave launch
            ProfScope ps_("k_repair_plan", st);
            hipLaunchKernelGGL(k_repair_plan, dim3(1), dim3(64), 0, st, rp.d_sets, rp.n_sets, 1u, rp.plan,
                               rp.fb_class_mask, rp.tune.items, fb_min_sub(rp));
        }
        if (int rc = launch_scans(rp, rp.fb_class_mask, 1, st)) return rc;
        {
            ProfScope ps_("k_repair_finish", st);
            hipLaunchKernelGGL(k_repair_finish, dim3(finish_grid(rp.total_n)), dim3(kBlock), 0, st, rp.d_sets,
                               rp.n_sets, rp.plan, 1u, 0u, PlanArgs{});
        }
    }
    CT_HIP(hipGetLastError());
    return CT_OK;
}
