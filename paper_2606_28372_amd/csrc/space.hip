// Search-space resolution on the GPU (Section IV-A: the whole space is
// enumerated before tuning, giving the list of valid configurations).
//
// Layout of the work: a "group" is 64 bitmask words = 4096 consecutive linear
// indices, owned by one wave.  In each of 64 steps the wave's lanes take 64
// consecutive configurations, decode them, run the constraint programs and
// ballot the results into one word, which stays in the register of lane k;
// the 64 words leave with one coalesced 512-byte store.
//
// Constraint scopes are hoisted: a program over few parameters becomes a bit
// table over its scope's value combinations (programs of one scope class
// share the AND of their tables); programs that only read the first `split`
// parameters are evaluated once per prefix (a bit table over prod_{j<split}
// r_j prefixes), a group whose prefixes are all invalid is written as zeros
// without decoding anything, and the inner programs become bit patterns per
// context of prefix values.  The valid list is then compacted in ascending
// order without atomics: per-group counts, tile sums and one scan of them,
// group offsets, and work items of at most 256 valid configurations whose
// rows are ORs of a prefix and an inner digit row; then the 64-row boxes and
// chunk boxes the repair scans prune with.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "ct_host.h"

namespace {

constexpr int kBlock = 256;            // 4 waves
constexpr int kWavesPerBlock = kBlock / 64;
constexpr int kTileGroups = 256;       // groups per scan tile
constexpr uint32_t kChunk = 256;       // valid configurations per compaction work item

__device__ __forceinline__ void load_values_lds(const DevSpace& S, int64_t* lds, uint32_t n_vals) {
    for (uint32_t i = threadIdx.x; i < n_vals; i += blockDim.x) lds[i] = S.values[i];
    __syncthreads();
}

// What evaluation and decoding read for every configuration, copied into LDS at the start of a
// kernel: the value tables, the scope tables (when they fit), the programs' table descriptors and
// the radices with their division magic numbers.  Read from the kernel argument block instead,
// each per-digit or per-program field would be a dependent scalar load inside the loops.
constexpr uint32_t kTabLdsWords = 4096;       // scope tables up to 32 KiB go to LDS
constexpr uint64_t kRowTableBytes = 16ull << 20;   // prefix / inner digit-row tables of the compaction
bool row_tables(const DevSpace& S) {
    return S.split < S.D && S.P_s * S.R <= kRowTableBytes && S.I_s * S.R <= kRowTableBytes;
}

struct LdsCtx {
    const CT_LDS int64_t* vals;
    const CT_LDS uint32_t* meta;
    const CT_LDS uint32_t* rad;
    const CT_LDS uint32_t* mm;
    const CT_LDS uint32_t* ml;
    const CT_LDS uint64_t* tabs_l;            // LDS copy of the scope tables, or null
    const CT_GLOBAL uint64_t* tabs_g;
    const CT_LDS uint32_t* rm1;               // per row word: radix - 1 of its four digits (255 past D)
    uint32_t nw;                              // row words (R / 4)
};

// Scope-table words a kernel copies into LDS (0: it reads them from device memory), and the LDS
// bytes of the context (the host sizes the launch with them)
uint32_t ctx_tab_lds(const ct_space* s) {
    const size_t vb = s->values.size() * 8;
    return s->tab_words <= kTabLdsWords && vb + s->tab_words * 8 <= 48u * 1024u ? (uint32_t)s->tab_words : 0u;
}
size_t ctx_lds_bytes(const ct_space* s) {
    return s->values.size() * 8 + (size_t)ctx_tab_lds(s) * 8 +
           (size_t)std::max<uint32_t>(s->dev.n_cons, 1) * CT_TAB_META * 4 + 3 * CT_DMAX * 4 + CT_DMAX;
}

__device__ __forceinline__ LdsCtx load_ctx(const DevSpace& S, uint32_t n_vals, uint32_t tab_words) {
    extern __shared__ int64_t lds_ctx[];
    const bool tl = tab_words != 0;
    CT_LDS int64_t* v = (CT_LDS int64_t*)lds_ctx;
    CT_LDS uint64_t* t = (CT_LDS uint64_t*)(v + n_vals);
    CT_LDS uint32_t* m = (CT_LDS uint32_t*)(t + (tl ? tab_words : 0u));
    CT_LDS uint32_t* d = m + (S.n_cons ? S.n_cons : 1u) * CT_TAB_META;
    for (uint32_t i = threadIdx.x; i < n_vals; i += blockDim.x) v[i] = S.values[i];
    if (tl)
        for (uint32_t i = threadIdx.x; i < tab_words; i += blockDim.x) t[i] = S.tabs[i];
    for (uint32_t i = threadIdx.x; i < S.n_cons * CT_TAB_META; i += blockDim.x) m[i] = S.tab_meta[i];
    CT_LDS uint32_t* rm = d + 3 * CT_DMAX;
    for (uint32_t i = threadIdx.x; i < CT_DMAX; i += blockDim.x) {
        d[i] = i < S.D ? S.radix[i] : 1u;
        d[CT_DMAX + i] = i < S.D ? S.mag_m[i] : 0u;
        d[2 * CT_DMAX + i] = i < S.D ? S.mag_l[i] : 0u;
    }
    for (uint32_t q = threadIdx.x; q < CT_DMAX / 4; q += blockDim.x) {
        uint32_t w = 0;
        for (uint32_t b = 0; b < 4; ++b) {
            const uint32_t j = 4 * q + b;
            w |= (j < S.D ? S.radix[j] - 1u : 255u) << (8 * b);
        }
        rm[q] = w;
    }
    __syncthreads();
    return LdsCtx{v, m, d, d + CT_DMAX, d + 2 * CT_DMAX, tl ? t : nullptr, gptr(S.tabs), rm, S.R / 4};
}

// digits [j0, j1) of x (x < prod_{j0<=j<j1} radix[j]), last digit fastest, from the LDS context
__device__ __forceinline__ void decode_ctx(const LdsCtx& C, uint32_t x, uint32_t j0, uint32_t j1, Row& r) {
    for (uint32_t j = j1; j-- > j0;) {
        const uint32_t q = ct_udiv(x, C.mm[j], C.ml[j]);
        r.set(j, x - q * C.rad[j]);
        x = q;
    }
}

// ct_valid with the descriptors and (when they fit) the tables in LDS; every program's scope
// parameters are read at once (up to CT_TAB_SCOPE, predicated).  kInterp = false: every program
// of the range has a table and no interpreter is compiled in.
template <bool kInterp, uint32_t RW = 0>       // RW: row words when known at compile time
__device__ __forceinline__ bool valid_ctx(const DevSpace& S, const LdsCtx& C, uint32_t c0, uint32_t c1, const Row& dig) {
    bool ok = true;
    for (uint32_t c = c0; c < c1; ++c) {
        const CT_LDS uint32_t* m = C.meta + c * CT_TAB_META;
        const uint32_t off = __builtin_amdgcn_readfirstlane(m[0]);
        if (off == CT_TAB_COVERED) continue;              // tested by another program's table
        if (!kInterp || off != ~0u) {
            // the table index sum_j digit_j * stride_j as byte dot products: strides are below
            // 2^16, low and high bytes apart, zero for parameters outside the scope
            uint32_t lo = 0, hi = 0;
#pragma unroll
            for (uint32_t q = 0; q < (RW ? RW : CT_DMAX / 4); ++q) {
                if (RW || q < C.nw) {
                    lo = __builtin_amdgcn_udot4(dig.w[q], __builtin_amdgcn_readfirstlane(m[12 + q]), lo, false);
                    hi = __builtin_amdgcn_udot4(dig.w[q], __builtin_amdgcn_readfirstlane(m[20 + q]), hi, false);
                }
            }
            const uint32_t idx = lo + (hi << 8);
            const uint64_t word = C.tabs_l ? C.tabs_l[off + (idx >> 6)] : C.tabs_g[off + (idx >> 6)];
            ok &= ((word >> (idx & 63u)) & 1ull) != 0;
        } else {
            ok &= ct_eval(S, c, c + 1, dig, (const int64_t*)C.vals);
            if (!__any(ok)) break;
        }
    }
    return ok;
}

// valid_ctx for U rows at once: each program's descriptor is read once for all of them.  Bit u of
// `okm` says whether row u is still valid; returns the updated bits.
template <bool kInterp, uint32_t RW, uint32_t U>
__device__ __forceinline__ uint32_t valid_ctx_rows(const DevSpace& S, const LdsCtx& C, uint32_t c0, uint32_t c1,
                                                   const Row (&dig)[U], uint32_t okm) {
    for (uint32_t c = c0; c < c1; ++c) {
        const CT_LDS uint32_t* m = C.meta + c * CT_TAB_META;
        const uint32_t off = __builtin_amdgcn_readfirstlane(m[0]);
        if (off == CT_TAB_COVERED) continue;              // tested by another program's table
        if (!kInterp || off != ~0u) {
            uint32_t slo[RW], shi[RW];
#pragma unroll
            for (uint32_t q = 0; q < RW; ++q) {
                slo[q] = __builtin_amdgcn_readfirstlane(m[12 + q]);
                shi[q] = __builtin_amdgcn_readfirstlane(m[20 + q]);
            }
#pragma unroll
            for (uint32_t u = 0; u < U; ++u) {
                uint32_t lo = 0, hi = 0;
#pragma unroll
                for (uint32_t q = 0; q < RW; ++q) {
                    lo = __builtin_amdgcn_udot4(dig[u].w[q], slo[q], lo, false);
                    hi = __builtin_amdgcn_udot4(dig[u].w[q], shi[q], hi, false);
                }
                const uint32_t idx = lo + (hi << 8);
                const uint64_t word = C.tabs_l ? C.tabs_l[off + (idx >> 6)] : C.tabs_g[off + (idx >> 6)];
                if (!((word >> (idx & 63u)) & 1ull)) okm &= ~(1u << u);
            }
        } else {
#pragma unroll
            for (uint32_t u = 0; u < U; ++u)
                if (!ct_eval(S, c, c + 1, dig[u], (const int64_t*)C.vals)) okm &= ~(1u << u);
        }
    }
    return okm;
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ uint32_t wave_excl_scan(uint32_t v, uint32_t lane) {
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t y = __shfl_up(x, o, 64);
        if (lane >= (uint32_t)o) x += y;
    }
    return x - v;
}

// Bits for linear indices x in [0, total) (total <= 2^32) under programs [0, c1), decoding only
// parameters [0, dlim).  Work unit: kSubWords bitmask words (64 configurations each) per wave, so
// that even small tables spread over many waves (the interpreter's instruction fetches are a
// dependent chain; other waves hide it).  Lane k keeps word k of the unit.  With group_counts,
// the valid configurations of each 4096-index group are added to its (zeroed) counter.
constexpr uint32_t kSubWords = 8;

// A program's own scope table: word w of the own tables (every tabled program owns a run of
// whole words, descriptors [n_cons, 2 n_cons)) is the ballot of the program over 64 consecutive
// combinations of its scope parameters (last one fastest), the other digits 0; combinations past
// the table's size evaluate combination 0 and are masked off.
__global__ __launch_bounds__(kBlock) void k_scope_tables(DevSpace S, uint32_t n_vals, uint64_t total_words,
                                                         uint64_t* __restrict__ tabs) {
    extern __shared__ int64_t lds_vals[];
    load_values_lds(S, lds_vals, n_vals);
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t* own = S.tab_meta + (uint64_t)S.n_cons * CT_TAB_META;
    const uint64_t stride = (uint64_t)gridDim.x * kWavesPerBlock;
    for (uint64_t w = (uint64_t)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6); w < total_words; w += stride) {
        // the program owning word w: the last one with a table starting at or before it
        uint32_t c = 0;
        for (uint32_t k = 0; k < S.n_cons; ++k) {
            const uint32_t off = own[k * CT_TAB_META];
            if (off < CT_TAB_COVERED && off <= w) c = k;
        }
        const uint32_t* m = own + c * CT_TAB_META;
        const uint64_t t0 = (w - m[0]) * 64u + lane;
        const bool in = t0 < m[2];
        uint32_t t = in ? (uint32_t)t0 : 0u;
        Row r;
#pragma unroll
        for (int q = 0; q < CT_DMAX / 4; ++q) r.w[q] = 0;
        for (uint32_t k = m[1]; k-- > 0;) {
            const uint32_t j = m[4 + k] & 31u;
            const uint32_t q = ct_udiv(t, S.mag_m[j], S.mag_l[j]);
            r.set(j, t - q * S.radix[j]);
            t = q;
        }
        const bool ok = ct_eval(S, c, c + 1, r, lds_vals) && in;
        const uint64_t b = __ballot(ok);
        if (lane == 0) tabs[w] = b;
    }
}

// Shared scope tables (words [w0, w1), after the own tables): bit t of a table is the AND of its
// programs' own-table bits at combination t of the shared scope, each found with the program's
// byte dot products.
__global__ __launch_bounds__(kBlock) void k_merge_tables(DevSpace S, uint64_t w0, uint64_t w1,
                                                         uint64_t* __restrict__ tabs) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t* own = S.tab_meta + (uint64_t)S.n_cons * CT_TAB_META;
    const uint64_t stride = (uint64_t)gridDim.x * kWavesPerBlock;
    for (uint64_t w = w0 + (uint64_t)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6); w < w1; w += stride) {
        uint32_t c = 0;
        for (uint32_t k = 0; k < S.n_cons; ++k) {
            const uint32_t off = S.tab_meta[k * CT_TAB_META];
            if (off < CT_TAB_COVERED && off >= w0 && off <= w) c = k;
        }
        const uint32_t* m = S.tab_meta + c * CT_TAB_META;
        const uint64_t t0 = (w - m[0]) * 64u + lane;
        const bool in = t0 < m[2];
        uint32_t t = in ? (uint32_t)t0 : 0u;
        Row r;
#pragma unroll
        for (int q = 0; q < CT_DMAX / 4; ++q) r.w[q] = 0;
        for (uint32_t k = m[1]; k-- > 0;) {
            const uint32_t j = m[4 + k] & 31u;
            const uint32_t q = ct_udiv(t, S.mag_m[j], S.mag_l[j]);
            r.set(j, t - q * S.radix[j]);
            t = q;
        }
        bool ok = in;
        const uint64_t members = (uint64_t)m[28] | ((uint64_t)m[29] << 32);
        for (uint64_t mm = members; mm; mm &= mm - 1ull) {
            const uint32_t* om = own + (uint32_t)__builtin_ctzll(mm) * CT_TAB_META;
            uint32_t lo = 0, hi = 0;
#pragma unroll
            for (uint32_t q = 0; q < CT_DMAX / 4; ++q) {
                if (q < S.R / 4) {
                    lo = __builtin_amdgcn_udot4(r.w[q], om[12 + q], lo, false);
                    hi = __builtin_amdgcn_udot4(r.w[q], om[20 + q], hi, false);
                }
            }
            const uint32_t idx = lo + (hi << 8);
            ok = ok && ((tabs[om[0] + (idx >> 6)] >> (idx & 63u)) & 1ull);
        }
        const uint64_t b = __ballot(ok);
        if (lane == 0) tabs[w] = b;
    }
}

// `sub` words per wave (at most 64); with pfx_ctx, also each index's context number (the mixed-
// radix number of its context digits) if it is valid, else ~0 (the prefix pass of the patterns).
template <bool TI>
__global__ __launch_bounds__(kBlock) void k_table(DevSpace S, uint64_t total, uint32_t dlim, uint32_t c1,
                                                  uint32_t n_vals, uint64_t n_words, uint64_t* __restrict__ words,
                                                  uint32_t* __restrict__ group_counts, uint32_t sub,
                                                  uint32_t* __restrict__ pfx_ctx, uint32_t tab_words) {
    const LdsCtx C = load_ctx(S, n_vals, tab_words);
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t n_units = (total + 64u * sub - 1) / (64u * sub);
    const uint64_t stride = (uint64_t)gridDim.x * kWavesPerBlock;
    for (uint64_t u = (uint64_t)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6); u < n_units; u += stride) {
        const uint64_t base = u * 64u * sub;
        uint64_t mine = 0;
        for (uint32_t k = 0; k < sub; ++k) {
            const uint64_t x = base + k * 64u + lane;
            bool ok = x < total;
            if (__any(ok)) {
                Row r;
#pragma unroll
                for (int q = 0; q < CT_DMAX / 4; ++q) r.w[q] = 0;
                decode_ctx(C, (uint32_t)(ok ? x : 0), 0, dlim, r);
                const bool in = ok;
                ok = ok && valid_ctx<!TI>(S, C, 0, c1, r);
                if (pfx_ctx && in) {
                    uint32_t ctx = 0;
                    for (uint32_t q = 0; q < S.n_cx; ++q) ctx += r.digit(S.cx[q] & 31u) * (S.cx[q] >> 5);
                    pfx_ctx[x] = ok ? ctx : ~0u;
                }
            }
            const uint64_t b = __ballot(ok);
            if (lane == k) mine = b;
        }
        const uint64_t w = u * sub + lane;
        if (lane < sub && w < n_words) words[w] = mine;
        if (group_counts) {
            const uint32_t c = wave_sum(lane < sub ? (uint32_t)__popcll(mine) : 0u);
            if (lane == 0 && c) atomicAdd(&group_counts[base / 4096u], c);
        }
    }
}

// Inner patterns: for each context c (a combination of the prefix parameters the inner programs
// read) the bits of the inner programs over every inner configuration t in [0, I_s), in pw words
// per context (the last one, past I_s, is zero).  One wave per (context, word).
template <bool TI>
__global__ __launch_bounds__(kBlock) void k_patterns(DevSpace S, uint32_t n_vals, uint64_t n_ctx, uint32_t pw,
                                                     uint64_t* __restrict__ pats, uint32_t tab_words) {
    const LdsCtx C = load_ctx(S, n_vals, tab_words);
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t total = n_ctx * pw;
    const uint64_t stride = (uint64_t)gridDim.x * kWavesPerBlock;
    for (uint64_t it = (uint64_t)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6); it < total; it += stride) {
        const uint32_t c = (uint32_t)(it / pw), wi = (uint32_t)(it % pw);
        const uint64_t t0 = (uint64_t)wi * 64u + lane;
        const bool in = t0 < S.I_s;
        Row r;
#pragma unroll
        for (int q = 0; q < CT_DMAX / 4; ++q) r.w[q] = 0;
        for (uint32_t q = 0; q < S.n_cx; ++q) {
            const uint32_t j = S.cx[q] & 31u;
            r.set(j, (c / (S.cx[q] >> 5)) % S.radix[j]);
        }
        decode_ctx(C, in ? (uint32_t)t0 : 0u, S.split, S.D, r);
        const bool ok = in && valid_ctx<!TI>(S, C, S.n_pre, S.n_cons, r);
        const uint64_t b = __ballot(ok);
        if (lane == 0) pats[it] = b;
    }
}

// Bits [off, off + len) of a pattern (len in 1..64); patterns end with a zero word.
__device__ __forceinline__ uint64_t pat_bits(const CT_GLOBAL uint64_t* pat, uint32_t off, uint32_t len) {
    const uint32_t q = off >> 6, sh = off & 63u;
    uint64_t v = pat[q] >> sh;
    if (sh && sh + len > 64u) v |= pat[q + 1] << (64u - sh);
    return len == 64u ? v : v & ((1ull << len) - 1ull);
}

// The bitmask from the patterns: lane l of a wave builds word l of kMaskUnroll groups at once
// (independent load chains, so the latency of the context and pattern loads overlaps) from the
// prefixes each word covers -- a valid prefix contributes its context's pattern, an invalid one
// zeros -- then each group's count.  Words past the space are zero.
constexpr uint32_t kMaskUnroll = 4;

__device__ __forceinline__ uint64_t pattern_word(const DevSpace& S, uint64_t L0, uint64_t p, uint32_t off,
                                                 const CT_GLOBAL uint32_t* C, const CT_GLOBAL uint64_t* P, uint32_t pw) {
    uint64_t word = 0;
    if (L0 < S.N) {
        const uint64_t Is = S.I_s;
        const uint64_t L1 = L0 + 64u < S.N ? L0 + 64u : S.N;
        uint64_t L = L0;
        while (L < L1) {
            const uint32_t len = (uint32_t)min<uint64_t>(Is - off, L1 - L);
            const uint32_t ctx = C[p];
            if (ctx != ~0u) word |= pat_bits(P + (uint64_t)ctx * pw, off, len) << (uint32_t)(L - L0);
            L += len;
            ++p;
            off = 0;
        }
    }
    return word;
}

// Only the groups that k_mask_classify listed (those spanning a valid prefix); it wrote the others
// as zeros with a count of 0.
__global__ __launch_bounds__(kBlock) void k_mask_pattern(DevSpace S, uint64_t* __restrict__ words,
                                                         uint32_t* __restrict__ group_counts,
                                                         const uint32_t* __restrict__ todo,
                                                         const uint32_t* __restrict__ n_todo,
                                                         const uint32_t* __restrict__ pfx_ctx,
                                                         const uint64_t* __restrict__ pats, uint32_t pw) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t waves = (uint64_t)gridDim.x * kWavesPerBlock;
    const uint64_t Is = S.I_s;
    const CT_GLOBAL uint64_t* P = gptr(pats);
    const CT_GLOBAL uint32_t* C = gptr(pfx_ctx);
    const uint64_t n_items = *n_todo;
    for (uint64_t i0 = (uint64_t)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6); i0 < n_items;
         i0 += waves * kMaskUnroll) {
        uint64_t w[kMaskUnroll];
        uint64_t gs[kMaskUnroll];
#pragma unroll
        for (uint32_t u = 0; u < kMaskUnroll; ++u) {
            const uint64_t it = i0 + u * waves;
            w[u] = 0;
            gs[u] = it < n_items ? todo[it] : 0;
            if (it < n_items) {
                const uint64_t g = gs[u];
                const uint64_t G0 = g * 4096u;
                const uint64_t p0 = G0 / Is;                         // wave-uniform
                const uint64_t L0 = G0 + (uint64_t)lane * 64u;
                const uint32_t rel = (uint32_t)(L0 - p0 * Is);       // < 4096 + I_s
                const uint32_t dq = ct_udiv(rel, S.Is_m, S.Is_l);
                w[u] = pattern_word(S, L0, p0 + dq, rel - dq * (uint32_t)Is, C, P, pw);
            }
        }
#pragma unroll
        for (uint32_t u = 0; u < kMaskUnroll; ++u) {
            if (i0 + u * waves < n_items) {
                const uint64_t g = gs[u];
                words[g * 64u + lane] = w[u];
                const uint32_t c = wave_sum((uint32_t)__popcll(w[u]));
                if (lane == 0) group_counts[g] = c;
            }
        }
    }
}

// Full bitmask when a prefix table exists (split < D), in two kernels.
// k_mask_classify: persistent waves take 64 groups at a time; lane l checks whether group l spans
// any valid prefix (the prefix bits it covers).  Groups that span none are written as zeros with
// one coalesced store each; the others are appended to a work list.
__global__ __launch_bounds__(kBlock) void k_mask_classify(DevSpace S, uint64_t n_groups, uint64_t n_words,
                                                          uint64_t* __restrict__ words, uint32_t* __restrict__ group_counts,
                                                          uint32_t* __restrict__ todo, uint32_t* __restrict__ n_todo) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t n_batches = (n_groups + 63u) / 64u;
    const uint64_t stride = (uint64_t)gridDim.x * kWavesPerBlock;
    for (uint64_t bt = (uint64_t)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6); bt < n_batches; bt += stride) {
        const uint64_t gl = bt * 64u + lane;
        bool need = false;
        if (gl < n_groups) {
            const uint64_t L0 = gl * 4096u;
            const uint64_t last = std::min<uint64_t>(L0 + 4095u, S.N - 1);
            const uint64_t p0 = L0 / S.I_s, p_hi = last / S.I_s;
            for (uint64_t w = p0 >> 6; w <= (p_hi >> 6) && !need; ++w) {
                uint64_t bits = S.prefix_words[w];
                if (w == (p0 >> 6)) bits &= ~0ull << (p0 & 63u);
                if (w == (p_hi >> 6) && (p_hi & 63u) != 63u) bits &= (2ull << (p_hi & 63u)) - 1ull;
                need = bits != 0;
            }
            group_counts[gl] = 0;
        }
        // the wave's groups that need the programs go to the work list with one atomic
        const uint64_t nm = __ballot(need);
        uint32_t base = 0;
        if (lane == 0 && nm) base = atomicAdd(n_todo, (uint32_t)__popcll(nm));
        base = __shfl(base, 0, 64);
        if (need) todo[base + (uint32_t)__popcll(nm & ((1ull << lane) - 1ull))] = (uint32_t)gl;
        uint64_t zero = __ballot(gl < n_groups && !need);
        while (zero) {
            const uint64_t g = bt * 64u + (uint64_t)(__ffsll((long long)zero) - 1);
            zero &= zero - 1ull;
            const uint64_t w = g * 64u + lane;
            if (w < n_words) words[w] = 0;
        }
    }
}

// k_mask_eval: work unit = kSubWords words of a listed group per wave; in each step the lanes
// take 64 consecutive configurations, skip the ones whose prefix is invalid, and run the programs
// that read inner parameters on the rest.  Counts are added to the group's counter.
template <bool TI>
__global__ __launch_bounds__(kBlock) void k_mask_eval(DevSpace S, uint32_t n_vals, uint64_t n_words,
                                                      uint64_t* __restrict__ words, uint32_t* __restrict__ group_counts,
                                                      const uint32_t* __restrict__ todo, const uint32_t* __restrict__ n_todo,
                                                      uint32_t tab_words) {
    const LdsCtx C = load_ctx(S, n_vals, tab_words);
    const uint32_t lane = threadIdx.x & 63u;
    constexpr uint32_t kUnits = 64u / kSubWords;
    const uint64_t total = (uint64_t)(*n_todo) * kUnits;
    const uint64_t stride = (uint64_t)gridDim.x * kWavesPerBlock;
    for (uint64_t it = (uint64_t)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6); it < total; it += stride) {
        const uint64_t g = todo[it / kUnits];
        const uint32_t sub = (uint32_t)(it % kUnits);
        const uint64_t L0 = g * 4096u + (uint64_t)sub * kSubWords * 64u;
        const uint64_t p0 = L0 / S.I_s;
        const uint32_t r0 = (uint32_t)(L0 - p0 * S.I_s);
        uint64_t mine = 0;
        for (uint32_t k = 0; k < kSubWords; ++k) {
            const uint32_t off = k * 64u + lane;
            const uint64_t L = L0 + off;
            const uint32_t x = r0 + off;
            const uint32_t q = ct_udiv(x, S.Is_m, S.Is_l);
            const uint32_t inner = x - q * (uint32_t)S.I_s;
            const uint64_t p = p0 + q;
            const bool inr = L < S.N;
            const uint64_t pp = inr ? p : 0u;     // p < P_s whenever L < N
            bool ok = inr && ((S.prefix_words[pp >> 6] >> (pp & 63u)) & 1ull);
            if (__any(ok)) {
                Row r;
#pragma unroll
                for (int t = 0; t < CT_DMAX / 4; ++t) r.w[t] = 0;
                decode_ctx(C, ok ? (uint32_t)p : 0u, 0, S.split, r);
                decode_ctx(C, ok ? inner : 0u, S.split, S.D, r);
                ok = ok && valid_ctx<!TI>(S, C, S.n_pre, S.n_cons, r);
            }
            const uint64_t b = __ballot(ok);
            if (lane == k) mine = b;
        }
        const uint64_t w = g * 64u + (uint64_t)sub * kSubWords + lane;
        if (lane < kSubWords && w < n_words) words[w] = mine;
        const uint32_t c = wave_sum(lane < kSubWords ? (uint32_t)__popcll(mine) : 0u);
        if (lane == 0 && c) atomicAdd(&group_counts[g], c);
    }
}

// Sums of each tile of kTileGroups group counts: valid configurations and compaction work items.
__global__ __launch_bounds__(kTileGroups) void k_tile_sums(const uint32_t* __restrict__ counts, uint64_t n_groups,
                                                           uint64_t* __restrict__ tile_sums,
                                                           uint64_t* __restrict__ tile_items) {
    __shared__ uint32_t part[2][kTileGroups / 64];
    uint64_t g = (uint64_t)blockIdx.x * kTileGroups + threadIdx.x;
    const uint32_t v = g < n_groups ? counts[g] : 0u;
    const uint32_t s = wave_sum(v), it = wave_sum((v + kChunk - 1u) / kChunk);
    if ((threadIdx.x & 63u) == 0) {
        part[0][threadIdx.x >> 6] = s;
        part[1][threadIdx.x >> 6] = it;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t t = 0, ti = 0;
        for (int i = 0; i < kTileGroups / 64; ++i) {
            t += part[0][i];
            ti += part[1][i];
        }
        tile_sums[blockIdx.x] = t;
        tile_items[blockIdx.x] = ti;
    }
}

__device__ __forceinline__ uint64_t wave_incl_scan64(uint64_t x, uint32_t lane) {
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t lo = __shfl_up((uint32_t)x, o, 64), hi = __shfl_up((uint32_t)(x >> 32), o, 64);
        if (lane >= (uint32_t)o) x += ((uint64_t)hi << 32) | lo;
    }
    return x;
}

// Exclusive scans of the tile sums and the tile work items by one block: each thread takes a run
// of kScanRun consecutive tiles (all loaded before any is added), the threads' run totals are
// scanned inside the waves and then across the waves, and each thread writes its run's offsets;
// rounds of 1,024 runs repeat while tiles remain.  Totals at [n_tiles].
constexpr uint32_t kScanRun = 8;
__global__ __launch_bounds__(1024) void k_scan_tiles(const uint64_t* __restrict__ tile_sums,
                                                     const uint64_t* __restrict__ tile_items, uint64_t n_tiles,
                                                     uint64_t* __restrict__ tile_off, uint64_t* __restrict__ item_off) {
    __shared__ uint64_t wsum[2][16];
    __shared__ uint64_t carry[2];
    const uint32_t lane = threadIdx.x & 63u, wv = threadIdx.x >> 6;
    if (threadIdx.x == 0) carry[0] = carry[1] = 0;
    __syncthreads();
    for (uint64_t b = 0; b < n_tiles; b += 1024u * kScanRun) {
        const uint64_t i0 = b + (uint64_t)threadIdx.x * kScanRun;
        uint64_t v[kScanRun], u[kScanRun];
#pragma unroll
        for (uint32_t k = 0; k < kScanRun; ++k) {
            v[k] = i0 + k < n_tiles ? tile_sums[i0 + k] : 0;
            u[k] = i0 + k < n_tiles ? tile_items[i0 + k] : 0;
        }
        uint64_t tv = 0, tu = 0;
#pragma unroll
        for (uint32_t k = 0; k < kScanRun; ++k) {
            tv += v[k];
            tu += u[k];
        }
        const uint64_t iv = wave_incl_scan64(tv, lane), iu = wave_incl_scan64(tu, lane);
        if (lane == 63) {
            wsum[0][wv] = iv;
            wsum[1][wv] = iu;
        }
        __syncthreads();
        uint64_t pv = carry[0], pu = carry[1];
        for (uint32_t k = 0; k < wv; ++k) {
            pv += wsum[0][k];
            pu += wsum[1][k];
        }
        uint64_t ov = pv + iv - tv, ou = pu + iu - tu;
#pragma unroll
        for (uint32_t k = 0; k < kScanRun; ++k) {
            if (i0 + k < n_tiles) {
                tile_off[i0 + k] = ov;
                item_off[i0 + k] = ou;
            }
            ov += v[k];
            ou += u[k];
        }
        __syncthreads();
        if (threadIdx.x == 1023) {
            carry[0] = pv + iv;
            carry[1] = pu + iu;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        tile_off[n_tiles] = carry[0];
        item_off[n_tiles] = carry[1];
    }
}

// Group offsets: one block per scan tile, one thread per group; the offset of group g is its
// tile's offset plus the counts of the tile's earlier groups.  Groups holding valid
// configurations are listed (in any order) for the compaction.
__global__ __launch_bounds__(kTileGroups) void k_group_off(const uint32_t* __restrict__ counts, uint64_t n_groups,
                                                           const uint64_t* __restrict__ tile_off,
                                                           const uint64_t* __restrict__ item_off,
                                                           uint64_t* __restrict__ grp_off,
                                                           uint64_t* __restrict__ items) {
    __shared__ uint32_t part[kTileGroups / 64];
    __shared__ uint32_t nip[kTileGroups / 64];
    const uint32_t lane = threadIdx.x & 63u, wv = threadIdx.x >> 6;
    const uint64_t g = (uint64_t)blockIdx.x * kTileGroups + threadIdx.x;
    const uint32_t c = g < n_groups ? counts[g] : 0u;
    const uint32_t nch = (c + kChunk - 1u) / kChunk;       // the group's compaction work items
    const uint32_t ex = wave_excl_scan(c, lane);
    const uint32_t iex = wave_excl_scan(nch, lane);
    if (lane == 63) {
        part[wv] = ex + c;
        nip[wv] = iex + nch;
    }
    __syncthreads();
    uint32_t before = 0, i_before = 0;
    for (uint32_t k = 0; k < wv; ++k) {
        before += part[k];
        i_before += nip[k];
    }
    if (g < n_groups) grp_off[g] = tile_off[blockIdx.x] + before + ex;
    // the group's work items (group << 5 | run of kChunk entries), at the tile's item offset
    const uint64_t at = item_off[blockIdx.x] + i_before + iex;
    for (uint32_t k = 0; k < nch; ++k) items[at + k] = (g << 5) | k;
}

// Digit rows of the numbers [0, n) over parameters [j0, j1) (the others zero): the prefix rows
// (j0 = 0) and the inner rows (j0 = split) that the compaction ORs together.
__global__ __launch_bounds__(kBlock) void k_digit_rows(DevSpace S, uint64_t n, uint32_t j0, uint32_t j1,
                                                       uint8_t* __restrict__ out) {
    for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (uint64_t)gridDim.x * blockDim.x) {
        Row r;
#pragma unroll
        for (int q = 0; q < CT_DMAX / 4; ++q) r.w[q] = 0;
        decode_range(S, (uint32_t)t, j0, j1, r);
        row_store(r, out + t * S.R, S.R);
    }
}

// Ascending valid list from the bitmask: one listed group per wave (waves loop over the list),
// at the offset the group scan gave it.  The group's set bits go through LDS in chunks of kChunk
// consecutive entries, which the lanes then write kEntryBatch at a time, the table loads of a
// batch issued together (a lane's entries would otherwise each wait for the last).  The rank
// directory's entries of empty groups are zero.  A configuration's row is its prefix row OR its
// inner row when both tables are given, else its digits are decoded.
constexpr uint32_t kEntryBatch = kChunk / 64;

// RW words of a row, loaded / stored as whole vectors (rows are RW * 4 bytes, RW * 4 aligned)
typedef uint32_t ct_u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t ct_u32x2 __attribute__((ext_vector_type(2)));
// The same as a streaming (nontemporal) load: the validity query reads each row once, and keeping
// the rows out of the caches leaves them to the constraint tables every row looks up (2^26 rows of
// 16 bytes: 300 -> 261 us)
template <uint32_t RW>
__device__ __forceinline__ void words_load_nt(const uint8_t* p, uint32_t (&w)[RW]) {
    if constexpr (RW == 1) {
        w[0] = __builtin_nontemporal_load((const CT_GLOBAL uint32_t*)p);
    } else if constexpr (RW == 2) {
        const ct_u32x2 v = __builtin_nontemporal_load((const CT_GLOBAL ct_u32x2*)p);
        w[0] = v.x; w[1] = v.y;
    } else {
#pragma unroll
        for (uint32_t h = 0; h < RW / 4; ++h) {
            const ct_u32x4 v = __builtin_nontemporal_load((const CT_GLOBAL ct_u32x4*)p + h);
            w[4 * h] = v.x; w[4 * h + 1] = v.y; w[4 * h + 2] = v.z; w[4 * h + 3] = v.w;
        }
    }
}

template <uint32_t RW>
__device__ __forceinline__ void words_load(const uint8_t* p, uint32_t (&w)[RW]) {
    if constexpr (RW == 1) {
        w[0] = *(const CT_GLOBAL uint32_t*)p;
    } else if constexpr (RW == 2) {
        const ct_u32x2 v = *(const CT_GLOBAL ct_u32x2*)p;
        w[0] = v.x; w[1] = v.y;
    } else {
#pragma unroll
        for (uint32_t h = 0; h < RW / 4; ++h) {
            const ct_u32x4 v = ((const CT_GLOBAL ct_u32x4*)p)[h];
            w[4 * h] = v.x; w[4 * h + 1] = v.y; w[4 * h + 2] = v.z; w[4 * h + 3] = v.w;
        }
    }
}
template <uint32_t RW>
__device__ __forceinline__ void words_store(uint8_t* p, const uint32_t (&w)[RW]) {
    if constexpr (RW == 1) {
        *(CT_GLOBAL uint32_t*)p = w[0];
    } else if constexpr (RW == 2) {
        *(CT_GLOBAL ct_u32x2*)p = ct_u32x2{w[0], w[1]};
    } else {
#pragma unroll
        for (uint32_t h = 0; h < RW / 4; ++h)
            ((CT_GLOBAL ct_u32x4*)p)[h] = ct_u32x4{w[4 * h], w[4 * h + 1], w[4 * h + 2], w[4 * h + 3]};
    }
}

template <uint32_t RW, bool TABLES>
__global__ __launch_bounds__(kBlock) void k_compact(DevSpace S, const uint64_t* __restrict__ words, uint64_t n_words,
                                                    const uint64_t* __restrict__ items, const uint64_t* __restrict__ n_items,
                                                    const uint64_t* __restrict__ grp_off,
                                                    uint64_t* __restrict__ lin, uint8_t* __restrict__ rows,
                                                    uint16_t* __restrict__ dir8, const uint8_t* __restrict__ prow,
                                                    const uint8_t* __restrict__ irow) {
    constexpr uint32_t R = RW * 4;
    __shared__ uint64_t emit[kWavesPerBlock][kChunk];
    __shared__ uint32_t dig3[3 * CT_DMAX];
    for (uint32_t i = threadIdx.x; i < CT_DMAX; i += blockDim.x) {
        dig3[i] = i < S.D ? S.radix[i] : 1u;
        dig3[CT_DMAX + i] = i < S.D ? S.mag_m[i] : 0u;
        dig3[2 * CT_DMAX + i] = i < S.D ? S.mag_l[i] : 0u;
    }
    __syncthreads();
    LdsCtx C{};
    C.rad = (const CT_LDS uint32_t*)dig3;
    C.mm = C.rad + CT_DMAX;
    C.ml = C.rad + 2 * CT_DMAX;
    const uint32_t lane = threadIdx.x & 63u, wv = threadIdx.x >> 6;
    const uint64_t ni = *n_items;
    for (uint64_t it = (uint64_t)blockIdx.x * kWavesPerBlock + wv; it < ni; it += (uint64_t)gridDim.x * kWavesPerBlock) {
        const uint64_t item = items[it];
        const uint64_t g = item >> 5;
        const uint32_t cs = (uint32_t)(item & 31u) * kChunk;   // the item's entries: [cs, cs + kChunk)
        const uint64_t base = grp_off[g];
        const uint64_t wi = g * 64u + lane;
        const uint64_t p0 = g * 4096u / S.I_s;                  // prefix of the group's first index
        uint64_t rem = wi < n_words ? words[wi] : 0ull;
        const uint32_t c = (uint32_t)__popcll(rem);
        const uint32_t excl = wave_excl_scan(c, lane);
        const uint32_t total = wave_sum(c);
        // rank directory: offset of each 8-word block inside the group (the group's first item)
        if (cs == 0 && (lane & 7u) == 0 && wi < n_words) dir8[wi >> 3] = (uint16_t)excl;
        uint32_t e = excl;                       // group-local index of the lane's next bit
        while (rem && e < cs) {                  // the lane's bits before the item
            rem &= rem - 1ull;
            ++e;
        }
        {
            const uint32_t ce = cs + kChunk;
            while (rem && e < ce) {
                const uint32_t b = (uint32_t)__ffsll((long long)rem) - 1u;
                rem &= rem - 1ull;
                emit[wv][e - cs] = wi * 64u + b;
                ++e;
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            const uint32_t n = std::min<uint32_t>(kChunk, total - cs);
            uint64_t L[kEntryBatch];
            uint32_t r[kEntryBatch][RW];
#pragma unroll
            for (uint32_t k = 0; k < kEntryBatch; ++k) {
                const uint32_t i = k * 64u + lane;
                const bool act = i < n;
                L[k] = act ? emit[wv][i] : 0ull;
                // digits from the prefix and inner parts, relative to the group's first prefix
                // (L - p0 I_s < 4096 + I_s: 32-bit division by the inner size's magic number)
                const uint32_t rel = (uint32_t)(L[k] - p0 * S.I_s);
                const uint32_t dq = act ? ct_udiv(rel, S.Is_m, S.Is_l) : 0u;
                const uint32_t inner = act ? rel - dq * (uint32_t)S.I_s : 0u;
                if constexpr (TABLES) {
                    uint32_t a[RW], b[RW];
                    words_load<RW>(prow + (p0 + dq) * R, a);
                    words_load<RW>(irow + (uint64_t)inner * R, b);
#pragma unroll
                    for (uint32_t q = 0; q < RW; ++q) r[k][q] = a[q] | b[q];
                } else {
                    Row rr;
#pragma unroll
                    for (int q = 0; q < CT_DMAX / 4; ++q) rr.w[q] = 0;
                    decode_ctx(C, (uint32_t)(p0 + dq), 0, S.split, rr);
                    decode_ctx(C, inner, S.split, S.D, rr);
#pragma unroll
                    for (uint32_t q = 0; q < RW; ++q) r[k][q] = rr.w[q];
                }
            }
#pragma unroll
            for (uint32_t k = 0; k < kEntryBatch; ++k) {
                const uint32_t i = k * 64u + lane;
                if (i < n) {
                    lin[base + cs + i] = L[k];
                    words_store<RW>(rows + (base + cs + i) * R, r[k]);
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
    }
}

// Two 16-bit lanes of a word (the even and the odd bytes of four packed digits, spread out) for
// packed minimum / maximum.
typedef unsigned short ct_us2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ ct_us2 as_us2(uint32_t x) { return __builtin_bit_cast(ct_us2, x); }
__device__ __forceinline__ uint32_t as_u32(ct_us2 x) { return __builtin_bit_cast(uint32_t, x); }

// Lane permutations inside rows of 16 lanes (data-parallel primitives, no LDS round trip): swap
// neighbours, swap pairs, mirror each half-row, mirror the row.  Min/max over these four steps
// leaves every lane of a row with the row's extremum.
template <int CTRL>
__device__ __forceinline__ uint32_t dpp(uint32_t x) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)x, (int)x, CTRL, 0xF, 0xF, false);
}
constexpr int kDppXor1 = 0xB1, kDppXor2 = 0x4E, kDppHalfMirror = 0x141, kDppMirror = 0x140;

// packed 16-bit minimum / maximum of a value over groups of `span` lanes (8, 16, 32 or 64; every
// lane gets its group's result)
template <bool MAX>
__device__ __forceinline__ ct_us2 group_ext(ct_us2 v, uint32_t span) {
    auto f = [](ct_us2 a, ct_us2 b) { return MAX ? __builtin_elementwise_max(a, b) : __builtin_elementwise_min(a, b); };
    v = f(v, as_us2(dpp<kDppXor1>(as_u32(v))));
    v = f(v, as_us2(dpp<kDppXor2>(as_u32(v))));
    v = f(v, as_us2(dpp<kDppHalfMirror>(as_u32(v))));
    if (span >= 16) v = f(v, as_us2(dpp<kDppMirror>(as_u32(v))));
    if (span >= 32) v = f(v, as_us2((uint32_t)__shfl_xor((int)as_u32(v), 16, 64)));
    if (span >= 64) v = f(v, as_us2((uint32_t)__shfl_xor((int)as_u32(v), 32, 64)));
    return v;
}

// Per-byte minimum / maximum over the wave of four packed digits, on the even and the odd bytes
// as two packed 16-bit pairs (one v_pk_min_u16 / v_pk_max_u16 per step instead of a byte
// emulation).
__device__ __forceinline__ void wave_byte_minmax(uint32_t w, uint32_t& lo, uint32_t& hi) {
    const uint32_t m = 0x00FF00FFu;
    ct_us2 le = as_us2(w & m), lo2 = as_us2((w >> 8) & m), he = le, ho = lo2;
    le = group_ext<false>(le, 64);
    lo2 = group_ext<false>(lo2, 64);
    he = group_ext<true>(he, 64);
    ho = group_ext<true>(ho, 64);
    lo = as_u32(le) | (as_u32(lo2) << 8);
    hi = as_u32(he) | (as_u32(ho) << 8);
}

// Per 64-row block of the valid list (a box), the smallest and the largest value index of every
// parameter (a bounding box used to prune repair scans), four digits per word; and which value
// indices of each parameter occur in the list (for the "adjacent" neighbour rule).  Persistent
// waves take one box after another.  Presence of a parameter with at most 32 values is one bit
// per value in a per-lane mask OR-ed over every row the lane sees, reduced once at the end; a
// wider parameter's values are marked per box, one distinct value per round, in LDS.  The masks
// are OR-ed into present[D][8], skipping the atomic when the bits are there already.
template <uint32_t RW, uint32_t DB>
__global__ __launch_bounds__(kBlock) void k_boxes(DevSpace S, uint32_t* __restrict__ boxes32,
                                                  uint32_t* __restrict__ present) {
    constexpr uint32_t kSlices = 64u / RW;               // rows of a box reduced by one lane: RW
    __shared__ uint32_t pres[CT_DMAX * 8];
    __shared__ uint32_t tiles[kWavesPerBlock][64 * RW];
    for (uint32_t i = threadIdx.x; i < CT_DMAX * 8; i += blockDim.x) pres[i] = 0;
    __syncthreads();
    const uint32_t lane = threadIdx.x & 63u;
    CT_LDS uint32_t* tile = (CT_LDS uint32_t*)tiles[threadIdx.x >> 6];
    const CT_GLOBAL uint32_t* rows32 = gptr(reinterpret_cast<const uint32_t*>(S.rows));
    const bool wide = S.max_radix > 32;
    // parameters whose presence goes through the per-lane masks (at most 32 values; DB >= D)
    uint32_t small = 0;
    for (uint32_t j = 0; j < S.D; ++j) small |= S.radix[j] <= 32u ? 1u << j : 0u;
    uint32_t m[DB];
#pragma unroll
    for (uint32_t j = 0; j < DB; ++j) m[j] = 0;
    const uint64_t waves = (uint64_t)gridDim.x * kWavesPerBlock;
    // the next box's rows load while the current box is reduced (past the end: the box's first row)
    auto box_row = [&](uint64_t sb, uint32_t (&w)[RW]) {
        const uint64_t v = sb * 64u + lane;
        const CT_GLOBAL uint32_t* src = rows32 + (v < S.n_valid ? v : sb * 64u) * RW;
#pragma unroll
        for (uint32_t q = 0; q < RW; ++q) w[q] = src[q];
    };
    const uint32_t q = lane / kSlices, sl = lane % kSlices;
    const uint32_t m8 = 0x00FF00FFu;
    uint64_t sb = (uint64_t)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
    uint32_t rn[RW];
    if (sb < S.n_sub) box_row(sb, rn);
    for (; sb < S.n_sub; sb += waves) {
        const bool in = sb * 64u + lane < S.n_valid;
        uint32_t r[RW];
#pragma unroll
        for (uint32_t k = 0; k < RW; ++k) r[k] = rn[k];
        if (sb + waves < S.n_sub) box_row(sb + waves, rn);
        // The box's 64 rows go through LDS so that lane (q, s) -- word q, slice s of RW rows --
        // reduces RW rows of one word on its own; the slices then combine within groups of
        // 64 / RW lanes (row permutations, plus shuffles across rows when RW < 4).
#pragma unroll
        for (uint32_t k = 0; k < RW; ++k) tile[lane * RW + k] = r[k];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const uint32_t w0 = tile[sl * RW * RW + q];
        ct_us2 le = as_us2(w0 & m8), lo2 = as_us2((w0 >> 8) & m8), he = le, ho = lo2;
#pragma unroll
        for (uint32_t t = 1; t < RW; ++t) {
            const uint32_t w = tile[(sl * RW + t) * RW + q];
            const ct_us2 e = as_us2(w & m8), o = as_us2((w >> 8) & m8);
            le = __builtin_elementwise_min(le, e);
            lo2 = __builtin_elementwise_min(lo2, o);
            he = __builtin_elementwise_max(he, e);
            ho = __builtin_elementwise_max(ho, o);
        }
        le = group_ext<false>(le, kSlices);
        lo2 = group_ext<false>(lo2, kSlices);
        he = group_ext<true>(he, kSlices);
        ho = group_ext<true>(ho, kSlices);
        if (sl == 0) {
            boxes32[sb * 2u * RW + q] = as_u32(le) | (as_u32(lo2) << 8);
            boxes32[sb * 2u * RW + RW + q] = as_u32(he) | (as_u32(ho) << 8);
        }
        // presence of each value of the small parameters, one bit per value in the lane's masks
#pragma unroll
        for (uint32_t j = 0; j < DB; ++j)
            if ((small >> j) & 1u) m[j] |= in ? 1u << ((r[j >> 2] >> ((j & 3u) * 8u)) & 0xFFu) : 0u;
        if (wide) {
            Row rr;
#pragma unroll
            for (uint32_t k = 0; k < CT_DMAX / 4; ++k) rr.w[k] = k < RW ? r[k] : 0u;
            for (uint32_t j = 0; j < S.D; ++j) {
                if (S.radix[j] <= 32u) continue;
                const uint32_t d = rr.digit(j);
                uint64_t left = __ballot(in);
                while (left) {
                    const uint32_t src = (uint32_t)(__ffsll((long long)left) - 1);
                    const uint32_t val = (uint32_t)__shfl((int)d, (int)src, 64);
                    if (lane == src) atomicOr(&pres[j * 8u + (val >> 5)], 1u << (val & 31u));
                    left &= ~__ballot(d == val);
                }
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
#pragma unroll
    for (uint32_t j = 0; j < DB; ++j) {
        if ((small >> j) & 1u) {
            uint32_t x = m[j];
            x |= dpp<kDppXor1>(x);
            x |= dpp<kDppXor2>(x);
            x |= dpp<kDppHalfMirror>(x);
            x |= dpp<kDppMirror>(x);
            x |= (uint32_t)__shfl_xor((int)x, 16, 64);
            x |= (uint32_t)__shfl_xor((int)x, 32, 64);
            if (lane == 0 && x) atomicOr(&pres[j * 8u], x);
        }
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < S.D * 8u; i += blockDim.x) {
        const uint32_t mk = pres[i];
        if (mk && (__hip_atomic_load(&present[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & mk) != mk)
            atomicOr(&present[i], mk);
    }
}

// Per 64 boxes (4096 rows), the smallest box minimum and the largest box maximum of every
// parameter: the level above the boxes, so a scan can rule out 64 boxes with one bound.
__global__ __launch_bounds__(kBlock) void k_chunks(DevSpace S, uint8_t* __restrict__ chunks) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t ck = (uint64_t)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
    if (ck >= S.n_chunk) return;
    const uint64_t b = ck * 64u + lane;
    const uint64_t src = (b < S.n_sub ? b : ck * 64u) * 2u * S.R;
    Row lo_r, hi_r;
    row_load(lo_r, S.boxes + src, S.R);
    row_load(hi_r, S.boxes + src + S.R, S.R);
    const uint32_t nw = S.R / 4;
    uint32_t outw = 0;
#pragma unroll
    for (uint32_t q = 0; q < CT_DMAX / 4; ++q) {
        if (q < nw) {
            uint32_t lo, hi, lo2, hi2;
            wave_byte_minmax(lo_r.w[q], lo, hi2);          // the minimum of the boxes' minima
            wave_byte_minmax(hi_r.w[q], lo2, hi);          // the maximum of their maxima
            if (lane == q) outw = lo;
            if (lane == nw + q) outw = hi;
        }
    }
    if (lane < 2 * nw) reinterpret_cast<uint32_t*>(chunks + ck * 2u * S.R)[lane] = outw;
}

// The nearest present value index below / above every index of every parameter ("adjacent"
// neighbour rule; 0xFF: none), after OR-ing the boxes kernel's per-block presence words.  One
// block of 1024 threads: four threads per presence word split the blocks between them.
__global__ __launch_bounds__(1024) void k_prevnext(uint32_t D, const uint32_t* __restrict__ partial, uint32_t n_part,
                                                   uint8_t* __restrict__ pn) {
    __shared__ uint32_t part4[4][CT_DMAX * 8];
    __shared__ uint32_t pres[CT_DMAX * 8];
    const uint32_t nwd = D * 8u;
    {
        const uint32_t i = threadIdx.x & 255u, k = threadIdx.x >> 8;
        uint32_t v = 0;
        if (i < nwd)
            for (uint32_t b = k; b < n_part; b += 4) v |= partial[(uint64_t)b * nwd + i];
        part4[k][i] = v;
    }
    __syncthreads();
    if (threadIdx.x < 256) pres[threadIdx.x] = part4[0][threadIdx.x] | part4[1][threadIdx.x] | part4[2][threadIdx.x] | part4[3][threadIdx.x];
    __syncthreads();
    for (uint32_t t = threadIdx.x; t < D * 256u; t += blockDim.x) {
        const uint32_t j = t >> 8, k = t & 255u, kw = k >> 5, kb = k & 31u;
        uint32_t prev = 0xFF, next = 0xFF;
        for (int w = (int)kw; w >= 0; --w) {
            uint32_t m = pres[j * 8u + (uint32_t)w];
            if ((uint32_t)w == kw) m &= (1u << kb) - 1u;
            if (m) { prev = (uint32_t)w * 32u + 31u - (uint32_t)__clz(m); break; }
        }
        for (uint32_t w = kw; w < 8; ++w) {
            uint32_t m = pres[j * 8u + w];
            if (w == kw) m &= kb == 31u ? 0u : ~((2u << kb) - 1u);
            if (m) { next = w * 32u + (uint32_t)__ffs(m) - 1u; break; }
        }
        pn[t * 2 + 0] = (uint8_t)prev;
        pn[t * 2 + 1] = (uint8_t)next;
    }
}

// Validity of caller rows: kRowsPerThread rows per thread and round (their loads in flight
// together), persistent blocks (the evaluation context goes to LDS once per block).
constexpr uint32_t kRowsPerThread = 4;
template <bool TI, uint32_t RW>
__global__ __launch_bounds__(kBlock) void k_valid_rows(DevSpace S, uint32_t n_vals, const uint8_t* __restrict__ rows,
                                                       uint64_t n, uint8_t* __restrict__ out, uint32_t tab_words) {
    const LdsCtx C = load_ctx(S, n_vals, tab_words);
    uint32_t rmq[RW];
#pragma unroll
    for (uint32_t q = 0; q < RW; ++q) rmq[q] = __builtin_amdgcn_readfirstlane(C.rm1[q]);
    const uint64_t step = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i0 = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i0 < n; i0 += step * kRowsPerThread) {
        Row r[kRowsPerThread];
#pragma unroll
        for (uint32_t u = 0; u < kRowsPerThread; ++u) {
            const uint64_t i = i0 + u * step;
            uint32_t w[RW];
            if (i < n) words_load_nt<RW>(rows + i * (RW * 4u), w);
            else
                for (uint32_t q = 0; q < RW; ++q) w[q] = 0;
#pragma unroll
            for (uint32_t q = 0; q < CT_DMAX / 4; ++q) r[u].w[q] = q < RW ? w[q] : 0u;
        }
        uint32_t okm = 0;
#pragma unroll
        for (uint32_t u = 0; u < kRowsPerThread; ++u) {
            // every digit below its radix, four at a time: in 16-bit lanes of the even and the odd
            // bytes, 0x100 + (radix - 1) - digit keeps bit 8 exactly when digit < radix
            bool ok = i0 + u * step < n;
#pragma unroll
            for (uint32_t q = 0; q < RW; ++q) {
                const uint32_t te = ((rmq[q] & 0x00FF00FFu) | 0x01000100u) - (r[u].w[q] & 0x00FF00FFu);
                const uint32_t to = (((rmq[q] >> 8) & 0x00FF00FFu) | 0x01000100u) - ((r[u].w[q] >> 8) & 0x00FF00FFu);
                ok &= ((te & to & 0x01000100u) == 0x01000100u);
            }
            if (!ok) {
#pragma unroll
                for (int q = 0; q < CT_DMAX / 4; ++q) r[u].w[q] = 0;
            }
            okm |= ok ? 1u << u : 0u;
        }
        okm = valid_ctx_rows<!TI, RW, kRowsPerThread>(S, C, 0, S.n_cons, r, okm);
#pragma unroll
        for (uint32_t u = 0; u < kRowsPerThread; ++u)
            if (i0 + u * step < n) out[i0 + u * step] = (okm >> u) & 1u;
    }
}

__global__ __launch_bounds__(kBlock) void k_rank(DevSpace S, const uint8_t* __restrict__ rows, uint64_t n,
                                                 int64_t* __restrict__ pos) {
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    Row r;
    row_load(r, rows + i * S.R, S.R);
    pos[i] = row_in_domain(S, r) ? rank_of(S, row_encode(S, r)) : -1;
}

// Do programs [c0, c1) all have scope tables (so the table-only kernel variants apply)?
bool tabled(const ct_space* s, uint32_t c0, uint32_t c1) {
    for (uint32_t c = c0; c < c1; ++c)
        if (s->tab_meta[(size_t)c * CT_TAB_META] == ~0u) return false;
    return true;
}

uint32_t grid_for(uint64_t items, uint32_t per_block, uint32_t cap = 0x7FFFFFFFu) {
    uint64_t g = (items + per_block - 1) / per_block;
    if (g < 1) g = 1;
    return (uint32_t)std::min<uint64_t>(g, cap);
}

template <uint32_t RW>
void launch_compact_rw(const DevSpace& S, bool tables, const uint64_t* words, uint64_t n_words, const uint64_t* items,
                       const uint64_t* n_items, uint64_t max_items, const uint64_t* grp_off, uint64_t* lin,
                       uint8_t* rows, uint16_t* dir8, const uint8_t* prow, const uint8_t* irow, hipStream_t st) {
    const dim3 grid(grid_for(std::min<uint64_t>(max_items, 32768), kWavesPerBlock));
    if (tables)
        hipLaunchKernelGGL((k_compact<RW, true>), grid, dim3(kBlock), 0, st, S, words, n_words, items, n_items, grp_off,
                           lin, rows, dir8, prow, irow);
    else
        hipLaunchKernelGGL((k_compact<RW, false>), grid, dim3(kBlock), 0, st, S, words, n_words, items, n_items, grp_off,
                           lin, rows, dir8, prow, irow);
}

void launch_compact(const DevSpace& S, bool tables, const uint64_t* words, uint64_t n_words, const uint64_t* items,
                    const uint64_t* n_items, uint64_t max_items, const uint64_t* grp_off, uint64_t* lin, uint8_t* rows,
                    uint16_t* dir8, const uint8_t* prow, const uint8_t* irow, hipStream_t st) {
    if (S.R == 4) launch_compact_rw<1>(S, tables, words, n_words, items, n_items, max_items, grp_off, lin, rows, dir8, prow, irow, st);
    else if (S.R == 8) launch_compact_rw<2>(S, tables, words, n_words, items, n_items, max_items, grp_off, lin, rows, dir8, prow, irow, st);
    else if (S.R == 16) launch_compact_rw<4>(S, tables, words, n_words, items, n_items, max_items, grp_off, lin, rows, dir8, prow, irow, st);
    else launch_compact_rw<8>(S, tables, words, n_words, items, n_items, max_items, grp_off, lin, rows, dir8, prow, irow, st);
}

template <uint32_t RW>
void launch_boxes(const DevSpace& S, uint32_t* boxes, uint32_t* present, hipStream_t st) {
    const dim3 grid(grid_for(S.n_sub, kWavesPerBlock, 2048));
    if (S.D <= 8 && RW * 4 >= 8) hipLaunchKernelGGL((k_boxes<RW, 8>), grid, dim3(kBlock), 0, st, S, boxes, present);
    else if (S.D <= 16 && RW * 4 >= 16) hipLaunchKernelGGL((k_boxes<RW, 16>), grid, dim3(kBlock), 0, st, S, boxes, present);
    else hipLaunchKernelGGL((k_boxes<RW, RW * 4>), grid, dim3(kBlock), 0, st, S, boxes, present);
}

}  // namespace

uint64_t space_resident_bytes(const ct_space* s, uint64_t n_valid) {
    const DevSpace& S = s->dev;
    const uint64_t n_groups = (S.N + 4095u) / 4096u, n_words_alloc = n_groups * 64u;
    uint64_t b = n_words_alloc * 8u;                                      // validity bitmask
    if (S.split != S.D) b += (S.P_s + 4095u) / 4096u * 64u * 8u;          // prefix table
    const uint64_t nv = n_valid ? n_valid : 1;
    b += nv * (8u + S.R);                                                  // linear indices + rows
    b += (uint64_t)S.D * 256u * 2u;                                        // prev/next present values
    b += n_groups * 8u + (n_words_alloc / 8u) * 2u;                        // rank directory
    b += (std::max<uint64_t>((n_valid + 63u) / 64u, 1) + (n_valid + 4095u) / 4096u) * 2u * S.R;  // boxes + chunks
    b += s->values.size() * 8u + std::max<size_t>(s->code.size(), 1) * 4u + sizeof(DevSpace);
    b += s->tab_meta.size() * 4u + std::max<uint64_t>(s->tab_words, 1) * 8u;       // scope tables
    return b;
}

uint64_t space_build_scratch_bytes(const ct_space* s) {
    const uint64_t n_groups = (s->dev.N + 4095u) / 4096u;
    const uint64_t n_tiles = (n_groups + kTileGroups - 1) / kTileGroups;
    const uint64_t pw = (s->dev.I_s + 63u) / 64u + 1u;
    // counts, tiles, compaction work items (one per non-empty group; the items past those, one per
    // kChunk valid configurations, are charged with the list when the build checks its byte limit)
    return n_groups * 4u + (4u * n_tiles + 2u) * 8u + (n_groups + 2u) * 8u +
           (row_tables(s->dev) ? (s->dev.P_s + s->dev.I_s) * s->dev.R : 0u) +          // digit-row tables
           (s->n_ctx ? s->dev.P_s * 4u + s->n_ctx * pw * 8u : (n_groups + 1u) * 4u) +   // patterns or work list
           1024u * (uint64_t)s->dev.D * 32u;                                           // presence partials
}

int space_build_device(ct_space* s, hipStream_t st) {
    DevSpace& S = s->dev;
    const uint32_t n_vals = (uint32_t)s->values.size();
    const size_t lds = ctx_lds_bytes(s);
    const uint32_t tw = ctx_tab_lds(s);
    const uint64_t n_groups = (S.N + 4095u) / 4096u;
    s->n_words = (S.N + 63u) / 64u;
    const uint64_t n_words_alloc = n_groups * 64u;
    uint32_t* d_counts = nullptr;
    uint64_t* d_tiles = nullptr;
    uint64_t* d_off = nullptr;
    const uint64_t n_tiles = (n_groups + kTileGroups - 1) / kTileGroups;
    CT_HIP(hipMalloc(&s->d_words, n_words_alloc * sizeof(uint64_t)));
    CT_HIP(hipMallocAsync((void**)&d_counts, n_groups * sizeof(uint32_t), st));
    // per tile: sums (valid configurations, then work items); exclusive offsets of both
    CT_HIP(hipMallocAsync((void**)&d_tiles, 2 * n_tiles * sizeof(uint64_t), st));
    CT_HIP(hipMallocAsync((void**)&d_off, 2 * (n_tiles + 1) * sizeof(uint64_t), st));
    uint64_t* d_ioff = d_off + n_tiles + 1;
    if (s->own_words) {
        ProfScope ps_("k_scope_tables", st);
        hipLaunchKernelGGL(k_scope_tables, dim3(grid_for(s->own_words, kWavesPerBlock, 1024)), dim3(kBlock), lds, st, S,
                           n_vals, s->own_words, s->d_tabs);
    }
    if (s->tab_words > s->own_words) {
        ProfScope ps_("k_merge_tables", st);
        hipLaunchKernelGGL(k_merge_tables, dim3(grid_for(s->tab_words - s->own_words, kWavesPerBlock, 1024)), dim3(kBlock), 0,
                           st, S, s->own_words, s->tab_words, s->d_tabs);
    }

    if (S.split == S.D) {
        // the whole space is one table (only when N < 64 or every parameter has one value)
        CT_HIP(hipMemsetAsync(d_counts, 0, n_groups * sizeof(uint32_t), st));
        CT_HIP(hipMemsetAsync(s->d_words, 0, n_words_alloc * sizeof(uint64_t), st));
        const uint64_t units = (S.N + 64u * kSubWords - 1) / (64u * kSubWords);
        const dim3 grid(grid_for(units, kWavesPerBlock, 4096));
        ProfScope ps_("k_table", st);
        if (tabled(s, 0, S.n_cons))
            hipLaunchKernelGGL(k_table<true>, grid, dim3(kBlock), lds, st, S, S.N, S.D, S.n_cons, n_vals, s->n_words,
                               s->d_words, d_counts, kSubWords, (uint32_t*)nullptr, tw);
        else
            hipLaunchKernelGGL(k_table<false>, grid, dim3(kBlock), lds, st, S, S.N, S.D, S.n_cons, n_vals, s->n_words,
                               s->d_words, d_counts, kSubWords, (uint32_t*)nullptr, tw);
    } else {
        const uint64_t p_groups = (S.P_s + 4095u) / 4096u;
        CT_HIP(hipMalloc(&s->d_prefix, p_groups * 64u * sizeof(uint64_t)));
        CT_HIP(hipMemsetAsync(s->d_prefix, 0, p_groups * 64u * sizeof(uint64_t), st));
        // one word of prefixes per wave: the prefix table is small and its waves should be many
        const uint64_t units = (S.P_s + 63u) / 64u;
        uint32_t* d_pfx_ctx = nullptr;
        uint64_t* d_pats = nullptr;
        const uint32_t pw = (uint32_t)((S.I_s + 63u) / 64u + 1u);
        if (s->n_ctx) {
            CT_HIP(hipMallocAsync((void**)&d_pfx_ctx, S.P_s * sizeof(uint32_t), st));
            CT_HIP(hipMallocAsync((void**)&d_pats, s->n_ctx * pw * sizeof(uint64_t), st));
        }
        {
            const dim3 grid(grid_for(units, kWavesPerBlock, 4096));
            ProfScope ps_("k_table", st);
            if (tabled(s, 0, S.n_pre))
                hipLaunchKernelGGL(k_table<true>, grid, dim3(kBlock), lds, st, S, S.P_s, S.split, S.n_pre, n_vals,
                                   p_groups * 64u, s->d_prefix, (uint32_t*)nullptr, 1u, d_pfx_ctx, tw);
            else
                hipLaunchKernelGGL(k_table<false>, grid, dim3(kBlock), lds, st, S, S.P_s, S.split, S.n_pre, n_vals,
                                   p_groups * 64u, s->d_prefix, (uint32_t*)nullptr, 1u, d_pfx_ctx, tw);
        }
        S.prefix_words = s->d_prefix;
        // groups spanning no valid prefix are zeros (written here); the others are listed
        uint32_t* d_todo = nullptr;
        CT_HIP(hipMallocAsync((void**)&d_todo, (n_groups + 1) * sizeof(uint32_t), st));
        CT_HIP(hipMemsetAsync(d_todo + n_groups, 0, sizeof(uint32_t), st));
        { ProfScope ps_("k_mask", st); hipLaunchKernelGGL(k_mask_classify, dim3(grid_for((n_groups + 63u) / 64u, kWavesPerBlock, 2048)), dim3(kBlock), 0, st, S, n_groups,
                           s->n_words, s->d_words, d_counts, d_todo, d_todo + n_groups); }
        const bool ti = tabled(s, S.n_pre, S.n_cons);
        if (s->n_ctx) {
            {
                const dim3 grid(grid_for(s->n_ctx * pw, kWavesPerBlock, 4096));
                ProfScope ps_("k_patterns", st);
                if (ti) hipLaunchKernelGGL(k_patterns<true>, grid, dim3(kBlock), lds, st, S, n_vals, s->n_ctx, pw, d_pats, tw);
                else hipLaunchKernelGGL(k_patterns<false>, grid, dim3(kBlock), lds, st, S, n_vals, s->n_ctx, pw, d_pats, tw);
            }
            { ProfScope ps_("k_mask", st); hipLaunchKernelGGL(k_mask_pattern, dim3(grid_for(n_groups, kWavesPerBlock * kMaskUnroll, 4096)), dim3(kBlock), 0, st, S,
                               s->d_words, d_counts, d_todo, d_todo + n_groups, d_pfx_ctx, d_pats, pw); }
            CT_HIP(hipFreeAsync(d_pfx_ctx, st));
            CT_HIP(hipFreeAsync(d_pats, st));
        } else {
            const dim3 grid(grid_for(n_groups * (64u / kSubWords), kWavesPerBlock, 4096));
            ProfScope ps_("k_mask", st);
            if (ti)
                hipLaunchKernelGGL(k_mask_eval<true>, grid, dim3(kBlock), lds, st, S, n_vals, s->n_words, s->d_words,
                                   d_counts, d_todo, d_todo + n_groups, tw);
            else
                hipLaunchKernelGGL(k_mask_eval<false>, grid, dim3(kBlock), lds, st, S, n_vals, s->n_words, s->d_words,
                                   d_counts, d_todo, d_todo + n_groups, tw);
        }
        CT_HIP(hipFreeAsync(d_todo, st));
    }
    CT_HIP(hipGetLastError());
    { ProfScope ps_("k_tile_sums", st); hipLaunchKernelGGL(k_tile_sums, dim3((uint32_t)n_tiles), dim3(kTileGroups), 0, st, d_counts, n_groups, d_tiles,
                                                       d_tiles + n_tiles); }
    { ProfScope ps_("k_scan_tiles", st); hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(1024), 0, st, d_tiles, d_tiles + n_tiles, n_tiles,
                                                        d_off, d_ioff); }
    CT_HIP(hipGetLastError());
    uint64_t total = 0;
    CT_HIP(hipMemcpyAsync(&total, d_off + n_tiles, sizeof(uint64_t), hipMemcpyDeviceToHost, st));
    CT_HIP(hipStreamSynchronize(st));
    s->n_valid = total;
    S.n_valid = total;
    s->over_limit = s->byte_limit && space_resident_bytes(s, total) + total / kChunk * 8u > s->byte_limit;
    if (s->over_limit) {
        (void)hipFreeAsync(d_counts, st);
        (void)hipFreeAsync(d_tiles, st);
        (void)hipFreeAsync(d_off, st);
        (void)hipStreamSynchronize(st);
        return ct_fail(CT_ENOMEM, "space build: the resolved space exceeds the byte limit");
    }
    const uint64_t alloc_n = total ? total : 1;
    CT_HIP(hipMalloc(&s->d_lin, alloc_n * sizeof(uint64_t)));
    CT_HIP(hipMalloc(&s->d_rows, alloc_n * S.R));
    CT_HIP(hipMalloc(&s->d_prevnext, (size_t)S.D * 256 * 2));
    CT_HIP(hipMalloc(&s->d_grp_off, n_groups * sizeof(uint64_t)));
    CT_HIP(hipMalloc(&s->d_dir8, (n_words_alloc / 8) * sizeof(uint16_t)));
    S.n_sub = (total + 63u) / 64u;
    S.n_chunk = (S.n_sub + 63u) / 64u;
    // boxes, then the chunk level in the same allocation
    CT_HIP(hipMalloc(&s->d_boxes, (std::max<uint64_t>(S.n_sub, 1) + S.n_chunk) * 2u * S.R));
    {
        // group offsets (every group) and the list of groups with valid configurations
        // compaction work items: a non-empty group's runs of kChunk valid configurations
        const uint64_t max_items = std::min<uint64_t>(n_groups, total) + total / kChunk + 1;
        uint64_t* d_items = nullptr;
        CT_HIP(hipMallocAsync((void**)&d_items, max_items * sizeof(uint64_t), st));
        const uint64_t* d_nitems = d_ioff + n_tiles;          // the item total
        CT_HIP(hipMemsetAsync(s->d_dir8, 0, (n_words_alloc / 8) * sizeof(uint16_t), st));
        { ProfScope ps_("k_group_off", st); hipLaunchKernelGGL(k_group_off, dim3((uint32_t)n_tiles), dim3(kTileGroups), 0, st, d_counts,
                           n_groups, d_off, d_ioff, s->d_grp_off, d_items); }
        if (total) {
            // prefix and inner digit rows, when both tables are small, so that a valid
            // configuration's row is two loads and an OR instead of a decode
            uint8_t* d_prow = nullptr;
            uint8_t* d_irow = nullptr;
            const bool rt = row_tables(S);
            if (rt) {
                CT_HIP(hipMallocAsync((void**)&d_prow, S.P_s * S.R, st));
                CT_HIP(hipMallocAsync((void**)&d_irow, S.I_s * S.R, st));
                ProfScope ps_("k_digit_rows", st);
                hipLaunchKernelGGL(k_digit_rows, dim3(grid_for(S.P_s, kBlock, 4096)), dim3(kBlock), 0, st, S, S.P_s, 0u, S.split, d_prow);
                hipLaunchKernelGGL(k_digit_rows, dim3(grid_for(S.I_s, kBlock, 4096)), dim3(kBlock), 0, st, S, S.I_s, S.split, S.D, d_irow);
            }
            {
                ProfScope ps_("k_compact", st);
                launch_compact(S, rt, s->d_words, s->n_words, d_items, d_nitems, max_items, s->d_grp_off, s->d_lin,
                               s->d_rows, s->d_dir8, d_prow, d_irow, st);
            }
            if (rt) {
                CT_HIP(hipFreeAsync(d_prow, st));
                CT_HIP(hipFreeAsync(d_irow, st));
            }
        }
        CT_HIP(hipFreeAsync(d_items, st));
    }
    S.lin = s->d_lin;
    S.rows = s->d_rows;
    S.words = s->d_words;
    S.n_words = s->n_words;
    S.grp_off = s->d_grp_off;
    S.dir8 = s->d_dir8;
    S.boxes = s->d_boxes;
    S.chunks = s->d_boxes + std::max<uint64_t>(S.n_sub, 1) * 2u * S.R;
    {
        // boxes, chunk boxes, and the presence of every value index
        uint32_t* d_part = nullptr;
        CT_HIP(hipMallocAsync((void**)&d_part, (size_t)S.D * 8u * sizeof(uint32_t), st));
        CT_HIP(hipMemsetAsync(d_part, 0, (size_t)S.D * 8u * sizeof(uint32_t), st));
        if (total) {
            {
                ProfScope ps_("k_boxes", st);
                uint32_t* bx = (uint32_t*)s->d_boxes;
                if (S.R == 4) launch_boxes<1>(S, bx, d_part, st);
                else if (S.R == 8) launch_boxes<2>(S, bx, d_part, st);
                else if (S.R == 16) launch_boxes<4>(S, bx, d_part, st);
                else launch_boxes<8>(S, bx, d_part, st);
            }
            { ProfScope ps_("k_chunks", st); hipLaunchKernelGGL(k_chunks, dim3(grid_for(S.n_chunk, kWavesPerBlock)), dim3(kBlock), 0, st, S, s->d_boxes + std::max<uint64_t>(S.n_sub, 1) * 2u * S.R); }
        }
        { ProfScope ps_("k_prevnext", st); hipLaunchKernelGGL(k_prevnext, dim3(1), dim3(1024), 0, st, S.D, d_part, 1u, s->d_prevnext); }
        CT_HIP(hipFreeAsync(d_part, st));
    }
    S.prevnext = s->d_prevnext;
    CT_HIP(hipGetLastError());
    CT_HIP(hipFreeAsync(d_counts, st));
    CT_HIP(hipFreeAsync(d_tiles, st));
    CT_HIP(hipFreeAsync(d_off, st));
    CT_HIP(hipStreamSynchronize(st));
    return CT_OK;
}

template <uint32_t RW>
void launch_valid_rows(const ct_space* s, bool tabled_all, const uint8_t* rows, uint64_t n, uint8_t* out, hipStream_t st) {
    const dim3 grid(grid_for((n + kRowsPerThread - 1) / kRowsPerThread, kBlock, 2048));
    if (tabled_all)
        hipLaunchKernelGGL((k_valid_rows<true, RW>), grid, dim3(kBlock), ctx_lds_bytes(s), st, s->dev,
                           (uint32_t)s->values.size(), rows, n, out, ctx_tab_lds(s));
    else
        hipLaunchKernelGGL((k_valid_rows<false, RW>), grid, dim3(kBlock), ctx_lds_bytes(s), st, s->dev,
                           (uint32_t)s->values.size(), rows, n, out, ctx_tab_lds(s));
}

int launch_valid_mask(const ct_space* s, const uint8_t* rows, uint64_t n, uint8_t* out, hipStream_t st) {
    if (n == 0) return CT_OK;
    {
        ProfScope ps_("k_valid_rows", st);
        const bool ti = tabled(s, 0, s->dev.n_cons);
        if (s->dev.R == 4) launch_valid_rows<1>(s, ti, rows, n, out, st);
        else if (s->dev.R == 8) launch_valid_rows<2>(s, ti, rows, n, out, st);
        else if (s->dev.R == 16) launch_valid_rows<4>(s, ti, rows, n, out, st);
        else launch_valid_rows<8>(s, ti, rows, n, out, st);
    }
    CT_HIP(hipGetLastError());
    return CT_OK;
}

int launch_rank(const ct_space* s, const uint8_t* rows, uint64_t n, int64_t* pos, hipStream_t st) {
    if (n == 0) return CT_OK;
    { ProfScope ps_("k_rank", st); hipLaunchKernelGGL(k_rank, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, st, s->dev, rows, n, pos); }
    CT_HIP(hipGetLastError());
    return CT_OK;
}
