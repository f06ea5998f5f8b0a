// Search-space resolution on the GPU (Section IV-A: the whole space is
// enumerated before tuning, giving the list of valid configurations).
//
// Layout of the work: a "group" is 64 bitmask words = 4096 consecutive linear
// indices, owned by one wave.  In each of 64 steps the wave's lanes take 64
// consecutive configurations, decode them, run the constraint programs and
// ballot the results into one word, which stays in the register of lane k;
// the 64 words leave with one coalesced 512-byte store.
//
// Constraint scopes are hoisted: programs that only read the first `split`
// parameters are evaluated once per prefix (a bit table over prod_{j<split}
// r_j prefixes), and a group whose prefixes are all invalid is written as
// zeros without decoding anything.  The valid list is then compacted in
// ascending order: per-group counts, a two-level exclusive scan, and a
// per-wave emission stage that spreads the group's valid indices over the
// wave's lanes through LDS before decoding their digit rows.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "ct_host.h"

namespace {

constexpr int kBlock = 256;            // 4 waves
constexpr int kWavesPerBlock = kBlock / 64;
constexpr int kTileGroups = 256;       // groups per scan tile
constexpr int kEmit = 256;             // LDS entries per wave in the emission stage

__device__ __forceinline__ void load_values_lds(const DevSpace& S, int64_t* lds, uint32_t n_vals) {
    for (uint32_t i = threadIdx.x; i < n_vals; i += blockDim.x) lds[i] = S.values[i];
    __syncthreads();
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

__global__ __launch_bounds__(kBlock) void k_table(DevSpace S, uint64_t total, uint32_t dlim, uint32_t c1,
                                                  uint32_t n_vals, uint64_t n_words, uint64_t* __restrict__ words,
                                                  uint32_t* __restrict__ group_counts) {
    extern __shared__ int64_t lds_vals[];
    load_values_lds(S, lds_vals, n_vals);
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t n_units = (total + 64u * kSubWords - 1) / (64u * kSubWords);
    const uint64_t stride = (uint64_t)gridDim.x * kWavesPerBlock;
    for (uint64_t u = (uint64_t)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6); u < n_units; u += stride) {
        const uint64_t base = u * 64u * kSubWords;
        uint64_t mine = 0;
        for (uint32_t k = 0; k < kSubWords; ++k) {
            const uint64_t x = base + k * 64u + lane;
            bool ok = x < total;
            if (__any(ok)) {
                Row r;
#pragma unroll
                for (int q = 0; q < CT_DMAX / 4; ++q) r.w[q] = 0;
                decode_range(S, (uint32_t)(ok ? x : 0), 0, dlim, r);
                ok = ok && ct_eval(S, 0, c1, r, lds_vals);
            }
            const uint64_t b = __ballot(ok);
            if (lane == k) mine = b;
        }
        const uint64_t w = u * kSubWords + lane;
        if (lane < kSubWords && w < n_words) words[w] = mine;
        if (group_counts) {
            const uint32_t c = wave_sum(lane < kSubWords ? (uint32_t)__popcll(mine) : 0u);
            if (lane == 0 && c) atomicAdd(&group_counts[base / 4096u], c);
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
__global__ __launch_bounds__(kBlock) void k_mask_eval(DevSpace S, uint32_t n_vals, uint64_t n_words,
                                                      uint64_t* __restrict__ words, uint32_t* __restrict__ group_counts,
                                                      const uint32_t* __restrict__ todo, const uint32_t* __restrict__ n_todo) {
    extern __shared__ int64_t lds_vals[];
    load_values_lds(S, lds_vals, n_vals);
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
                decode_range(S, ok ? (uint32_t)p : 0u, 0, S.split, r);
                decode_range(S, ok ? inner : 0u, S.split, S.D, r);
                ok = ok && ct_eval(S, S.n_pre, S.n_cons, r, lds_vals);
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

// Sum of each tile of kTileGroups group counts.
__global__ __launch_bounds__(kTileGroups) void k_tile_sums(const uint32_t* __restrict__ counts, uint64_t n_groups,
                                                           uint64_t* __restrict__ tile_sums) {
    __shared__ uint64_t part[kTileGroups / 64];
    uint64_t g = (uint64_t)blockIdx.x * kTileGroups + threadIdx.x;
    uint32_t v = g < n_groups ? counts[g] : 0u;
    uint32_t s = wave_sum(v);
    if ((threadIdx.x & 63u) == 0) part[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t t = 0;
        for (int i = 0; i < kTileGroups / 64; ++i) t += part[i];
        tile_sums[blockIdx.x] = t;
    }
}

// Exclusive scan of the tile sums by one block; total at tile_off[n_tiles].
__global__ __launch_bounds__(1024) void k_scan_tiles(const uint64_t* __restrict__ tile_sums, uint64_t n_tiles,
                                                     uint64_t* __restrict__ tile_off) {
    __shared__ uint64_t buf[1024];
    __shared__ uint64_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (uint64_t b = 0; b < n_tiles; b += 1024) {
        uint64_t i = b + threadIdx.x;
        uint64_t v = i < n_tiles ? tile_sums[i] : 0;
        buf[threadIdx.x] = v;
        __syncthreads();
        for (int o = 1; o < 1024; o <<= 1) {
            uint64_t y = threadIdx.x >= (unsigned)o ? buf[threadIdx.x - o] : 0;
            __syncthreads();
            buf[threadIdx.x] += y;
            __syncthreads();
        }
        if (i < n_tiles) tile_off[i] = carry + buf[threadIdx.x] - v;
        __syncthreads();
        if (threadIdx.x == 1023) carry += buf[1023];
        __syncthreads();
    }
    if (threadIdx.x == 0) tile_off[n_tiles] = carry;
}

// Ascending valid list from the bitmask: one group per wave.
__global__ __launch_bounds__(kBlock) void k_compact(DevSpace S, const uint64_t* __restrict__ words, uint64_t n_words,
                                                    const uint32_t* __restrict__ counts,
                                                    const uint64_t* __restrict__ tile_off, uint64_t n_groups,
                                                    uint64_t* __restrict__ lin, uint8_t* __restrict__ rows,
                                                    uint64_t* __restrict__ grp_off, uint16_t* __restrict__ dir8) {
    __shared__ uint64_t emit[kWavesPerBlock][kEmit];
    const uint32_t lane = threadIdx.x & 63u, wv = threadIdx.x >> 6;
    const uint64_t g = (uint64_t)blockIdx.x * kWavesPerBlock + wv;
    if (g >= n_groups) return;
    const uint64_t tile = g / kTileGroups;
    // offset of this group = tile offset + counts of earlier groups in the tile
    uint32_t before = 0;
    for (uint64_t t = tile * kTileGroups + lane; t < g; t += 64) before += counts[t];
    const uint64_t base = tile_off[tile] + wave_sum(before);
    const uint64_t wi = g * 64u + lane;
    uint64_t rem = wi < n_words ? words[wi] : 0ull;
    const uint32_t c = (uint32_t)__popcll(rem);
    const uint32_t excl = wave_excl_scan(c, lane);
    const uint32_t total = wave_sum(c);
    // rank directory: offset of the group, and of each 8-word block inside it
    if (lane == 0) grp_off[g] = base;
    if ((lane & 7u) == 0 && wi < n_words) dir8[wi >> 3] = (uint16_t)excl;
    uint32_t e = excl;                       // list index (within the group) of the lane's next bit
    for (uint32_t cs = 0; cs < total; cs += kEmit) {
        const uint32_t ce = cs + kEmit;
        while (rem && e < ce) {
            uint32_t b = (uint32_t)__ffsll((long long)rem) - 1u;
            rem &= rem - 1ull;
            emit[wv][e - cs] = wi * 64u + b;
            ++e;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const uint32_t nchunk = std::min<uint32_t>(kEmit, total - cs);
        for (uint32_t i = lane; i < nchunk; i += 64) {
            const uint64_t L = emit[wv][i];
            const uint64_t pos = base + cs + i;
            Row r;
            decode_lin(S, L, r);
            lin[pos] = L;
            row_store(r, rows + pos * S.R, S.R);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

// Per 64-row block of the valid list, the smallest and the largest value
// index of every parameter (a bounding box used to prune repair scans).
__global__ __launch_bounds__(kBlock) void k_boxes(DevSpace S, uint8_t* __restrict__ boxes) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t sb = (uint64_t)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
    if (sb >= S.n_sub) return;
    const uint64_t v = sb * 64u + lane;
    const bool in = v < S.n_valid;
    Row r;
    row_load(r, S.rows + (in ? v : sb * 64u) * S.R, S.R);
    for (uint32_t j = 0; j < S.R; ++j) {
        uint32_t d = j < S.D ? r.digit(j) : 0u;
        uint32_t lo = d, hi = d;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            lo = min(lo, (uint32_t)__shfl_xor((int)lo, o, 64));
            hi = max(hi, (uint32_t)__shfl_xor((int)hi, o, 64));
        }
        if (lane == 0) {
            boxes[sb * 2u * S.R + j] = (uint8_t)lo;
            boxes[sb * 2u * S.R + S.R + j] = (uint8_t)hi;
        }
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
    for (uint32_t j = 0; j < S.R; ++j) {
        uint32_t lo = j < S.D ? lo_r.digit(j) : 0u, hi = j < S.D ? hi_r.digit(j) : 0u;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            lo = min(lo, (uint32_t)__shfl_xor((int)lo, o, 64));
            hi = max(hi, (uint32_t)__shfl_xor((int)hi, o, 64));
        }
        if (lane == 0) {
            chunks[ck * 2u * S.R + j] = (uint8_t)lo;
            chunks[ck * 2u * S.R + S.R + j] = (uint8_t)hi;
        }
    }
}

// Which value indices of each parameter occur in some solution, then the
// nearest present index below/above each index ("adjacent" neighbour rule).
__global__ __launch_bounds__(kBlock) void k_presence(DevSpace S, uint32_t* __restrict__ present /*[D][8]*/) {
    __shared__ uint32_t loc[CT_DMAX * 8];
    for (uint32_t i = threadIdx.x; i < CT_DMAX * 8; i += blockDim.x) loc[i] = 0;
    __syncthreads();
    for (uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; v < S.n_valid;
         v += (uint64_t)gridDim.x * blockDim.x) {
        Row r;
        row_load(r, S.rows + v * S.R, S.R);
        for (uint32_t j = 0; j < S.D; ++j) {
            uint32_t d = r.digit(j);
            atomicOr(&loc[j * 8 + (d >> 5)], 1u << (d & 31u));
        }
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < S.D * 8; i += blockDim.x)
        if (loc[i]) atomicOr(&present[i], loc[i]);
}

__global__ void k_prevnext(uint32_t D, const uint32_t* __restrict__ present, uint8_t* __restrict__ pn) {
    uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= D * 256u) return;
    uint32_t j = t >> 8, k = t & 255u;
    auto has = [&](uint32_t v) { return (present[j * 8 + (v >> 5)] >> (v & 31u)) & 1u; };
    uint32_t prev = 0xFF, next = 0xFF;
    for (int v = (int)k - 1; v >= 0; --v)
        if (has((uint32_t)v)) { prev = (uint32_t)v; break; }
    for (uint32_t v = k + 1; v < 256; ++v)
        if (has(v)) { next = v; break; }
    pn[t * 2 + 0] = (uint8_t)prev;
    pn[t * 2 + 1] = (uint8_t)next;
}

__global__ __launch_bounds__(kBlock) void k_valid_rows(DevSpace S, uint32_t n_vals, const uint8_t* __restrict__ rows,
                                                       uint64_t n, uint8_t* __restrict__ out) {
    extern __shared__ int64_t lds_vals[];
    load_values_lds(S, lds_vals, n_vals);
    for (uint64_t base = (uint64_t)blockIdx.x * blockDim.x; base < n; base += (uint64_t)gridDim.x * blockDim.x) {
        uint64_t i = base + threadIdx.x;
        bool in = i < n;
        Row r;
        if (in) row_load(r, rows + i * S.R, S.R);
        else
            for (int q = 0; q < CT_DMAX / 4; ++q) r.w[q] = 0;
        bool ok = in && row_in_domain(S, r);
        if (!ok) {
#pragma unroll
            for (int q = 0; q < CT_DMAX / 4; ++q) r.w[q] = 0;
        }
        ok = ct_eval(S, 0, S.n_cons, r, lds_vals) && ok;
        if (in) out[i] = ok ? 1 : 0;
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

uint32_t grid_for(uint64_t items, uint32_t per_block, uint32_t cap = 0x7FFFFFFFu) {
    uint64_t g = (items + per_block - 1) / per_block;
    if (g < 1) g = 1;
    return (uint32_t)std::min<uint64_t>(g, cap);
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
    return b;
}

uint64_t space_build_scratch_bytes(const ct_space* s) {
    const uint64_t n_groups = (s->dev.N + 4095u) / 4096u;
    const uint64_t n_tiles = (n_groups + kTileGroups - 1) / kTileGroups;
    return n_groups * 4u + (2u * n_tiles + 1u) * 8u + (uint64_t)s->dev.D * 32u;
}

int space_build_device(ct_space* s, hipStream_t st) {
    DevSpace& S = s->dev;
    const uint32_t n_vals = (uint32_t)s->values.size();
    const size_t lds = s->lds_values_bytes;
    const uint64_t n_groups = (S.N + 4095u) / 4096u;
    s->n_words = (S.N + 63u) / 64u;
    const uint64_t n_words_alloc = n_groups * 64u;
    uint32_t* d_counts = nullptr;
    uint64_t* d_tiles = nullptr;
    uint64_t* d_off = nullptr;
    const uint64_t n_tiles = (n_groups + kTileGroups - 1) / kTileGroups;
    CT_HIP(hipMalloc(&s->d_words, n_words_alloc * sizeof(uint64_t)));
    CT_HIP(hipMallocAsync((void**)&d_counts, n_groups * sizeof(uint32_t), st));
    CT_HIP(hipMallocAsync((void**)&d_tiles, n_tiles * sizeof(uint64_t), st));
    CT_HIP(hipMallocAsync((void**)&d_off, (n_tiles + 1) * sizeof(uint64_t), st));

    if (S.split == S.D) {
        // the whole space is one table (only when N < 64 or every parameter has one value)
        CT_HIP(hipMemsetAsync(d_counts, 0, n_groups * sizeof(uint32_t), st));
        CT_HIP(hipMemsetAsync(s->d_words, 0, n_words_alloc * sizeof(uint64_t), st));
        const uint64_t units = (S.N + 64u * kSubWords - 1) / (64u * kSubWords);
        { ProfScope ps_("k_table", st); hipLaunchKernelGGL(k_table, dim3(grid_for(units, kWavesPerBlock, 4096)), dim3(kBlock), lds, st, S, S.N, S.D,
                           S.n_cons, n_vals, s->n_words, s->d_words, d_counts); }
    } else {
        const uint64_t p_groups = (S.P_s + 4095u) / 4096u;
        CT_HIP(hipMalloc(&s->d_prefix, p_groups * 64u * sizeof(uint64_t)));
        CT_HIP(hipMemsetAsync(s->d_prefix, 0, p_groups * 64u * sizeof(uint64_t), st));
        const uint64_t units = (S.P_s + 64u * kSubWords - 1) / (64u * kSubWords);
        { ProfScope ps_("k_table", st); hipLaunchKernelGGL(k_table, dim3(grid_for(units, kWavesPerBlock, 4096)), dim3(kBlock), lds, st, S, S.P_s,
                           S.split, S.n_pre, n_vals, p_groups * 64u, s->d_prefix, (uint32_t*)nullptr); }
        S.prefix_words = s->d_prefix;
        uint32_t* d_todo = nullptr;
        CT_HIP(hipMallocAsync((void**)&d_todo, (n_groups + 1) * sizeof(uint32_t), st));
        CT_HIP(hipMemsetAsync(d_todo + n_groups, 0, sizeof(uint32_t), st));
        { ProfScope ps_("k_mask", st); hipLaunchKernelGGL(k_mask_classify, dim3(grid_for((n_groups + 63u) / 64u, kWavesPerBlock, 2048)), dim3(kBlock), 0, st, S, n_groups,
                           s->n_words, s->d_words, d_counts, d_todo, d_todo + n_groups); }
        { ProfScope ps_("k_mask", st); hipLaunchKernelGGL(k_mask_eval, dim3(grid_for(n_groups * (64u / kSubWords), kWavesPerBlock, 4096)), dim3(kBlock), lds, st, S, n_vals,
                           s->n_words, s->d_words, d_counts, d_todo, d_todo + n_groups); }
        CT_HIP(hipFreeAsync(d_todo, st));
    }
    CT_HIP(hipGetLastError());
    { ProfScope ps_("k_tile_sums", st); hipLaunchKernelGGL(k_tile_sums, dim3((uint32_t)n_tiles), dim3(kTileGroups), 0, st, d_counts, n_groups, d_tiles); }
    { ProfScope ps_("k_scan_tiles", st); hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(1024), 0, st, d_tiles, n_tiles, d_off); }
    CT_HIP(hipGetLastError());
    uint64_t total = 0;
    CT_HIP(hipMemcpyAsync(&total, d_off + n_tiles, sizeof(uint64_t), hipMemcpyDeviceToHost, st));
    CT_HIP(hipStreamSynchronize(st));
    s->n_valid = total;
    S.n_valid = total;
    s->over_limit = s->byte_limit && space_resident_bytes(s, total) > s->byte_limit;
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
    uint32_t* d_present = nullptr;
    CT_HIP(hipMallocAsync((void**)&d_present, (size_t)S.D * 8 * sizeof(uint32_t), st));
    CT_HIP(hipMemsetAsync(d_present, 0, (size_t)S.D * 8 * sizeof(uint32_t), st));
    CT_HIP(hipMalloc(&s->d_grp_off, n_groups * sizeof(uint64_t)));
    CT_HIP(hipMalloc(&s->d_dir8, (n_words_alloc / 8) * sizeof(uint16_t)));
    S.n_sub = (total + 63u) / 64u;
    S.n_chunk = (S.n_sub + 63u) / 64u;
    // boxes, then the chunk level in the same allocation
    CT_HIP(hipMalloc(&s->d_boxes, (std::max<uint64_t>(S.n_sub, 1) + S.n_chunk) * 2u * S.R));
    if (total) {
        { ProfScope ps_("k_compact", st); hipLaunchKernelGGL(k_compact, dim3(grid_for(n_groups, kWavesPerBlock)), dim3(kBlock), 0, st, S, s->d_words,
                           s->n_words, d_counts, d_off, n_groups, s->d_lin, s->d_rows, s->d_grp_off, s->d_dir8); }
    }
    S.lin = s->d_lin;
    S.rows = s->d_rows;
    S.words = s->d_words;
    S.n_words = s->n_words;
    S.grp_off = s->d_grp_off;
    S.dir8 = s->d_dir8;
    S.boxes = s->d_boxes;
    S.chunks = s->d_boxes + std::max<uint64_t>(S.n_sub, 1) * 2u * S.R;
    if (total) {
        { ProfScope ps_("k_boxes", st); hipLaunchKernelGGL(k_boxes, dim3(grid_for(S.n_sub, kWavesPerBlock)), dim3(kBlock), 0, st, S, s->d_boxes); }
        { ProfScope ps_("k_chunks", st); hipLaunchKernelGGL(k_chunks, dim3(grid_for(S.n_chunk, kWavesPerBlock)), dim3(kBlock), 0, st, S, s->d_boxes + std::max<uint64_t>(S.n_sub, 1) * 2u * S.R); }
    }
    if (total) {
        { ProfScope ps_("k_presence", st); hipLaunchKernelGGL(k_presence, dim3(grid_for(total, kBlock, 1024)), dim3(kBlock), 0, st, S, d_present); }
    }
    { ProfScope ps_("k_prevnext", st); hipLaunchKernelGGL(k_prevnext, dim3(grid_for(S.D * 256u, 256)), dim3(256), 0, st, S.D, d_present,
                       s->d_prevnext); }
    S.prevnext = s->d_prevnext;
    CT_HIP(hipGetLastError());
    CT_HIP(hipFreeAsync(d_present, st));
    CT_HIP(hipFreeAsync(d_counts, st));
    CT_HIP(hipFreeAsync(d_tiles, st));
    CT_HIP(hipFreeAsync(d_off, st));
    CT_HIP(hipStreamSynchronize(st));
    return CT_OK;
}

int launch_valid_mask(const ct_space* s, const uint8_t* rows, uint64_t n, uint8_t* out, hipStream_t st) {
    if (n == 0) return CT_OK;
    { ProfScope ps_("k_valid_rows", st); hipLaunchKernelGGL(k_valid_rows, dim3(grid_for(n, kBlock, 8192)), dim3(kBlock), s->lds_values_bytes, st, s->dev,
                       (uint32_t)s->values.size(), rows, n, out); }
    CT_HIP(hipGetLastError());
    return CT_OK;
}

int launch_rank(const ct_space* s, const uint8_t* rows, uint64_t n, int64_t* pos, hipStream_t st) {
    if (n == 0) return CT_OK;
    { ProfScope ps_("k_rank", st); hipLaunchKernelGGL(k_rank, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, st, s->dev, rows, n, pos); }
    CT_HIP(hipGetLastError());
    return CT_OK;
}
