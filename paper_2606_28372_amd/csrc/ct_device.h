// Device-side building blocks of libct (gfx950, wave64).
//
//  - DevSpace: everything a kernel needs to know about a resolved space,
//    passed by value as a kernel argument;
//  - exact 32-bit division by a run-time constant (round-up multiply-high
//    method, Granlund & Montgomery 1994) for mixed-radix decoding;
//  - Philox4x32-10 (Salmon et al., SC'11);
//  - the constraint-bytecode interpreter (Python integer semantics, a
//    poison bit per stack slot for "would raise").
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ct_bytecode.h"

#define CT_DMAX 32        // parameters per space
#define CT_STACK 16       // interpreter stack depth
// Scope tables: constraints that read at most CT_TAB_SCOPE parameters whose value counts
// multiply to at most CT_TAB_BITS are evaluated once per combination of those parameters into a
// bit table; a configuration then tests one bit instead of running the programs.  Programs of one
// class (prefix / inner) share a table over the union of their scopes while it stays within both
// limits: its bit is the AND of theirs.
#define CT_TAB_SCOPE 8
#define CT_TAB_BITS 65536u
#define CT_TAB_META 30    // u32 per program: word offset (~0: no table; CT_TAB_COVERED: in another
                          // program's table), scope size, table bits, 0, (stride << 5) | parameter
                          // for each scope parameter [4..11], the table strides as bytes by row
                          // word: low bytes [12..19], high [20..27] (a row's table index is two
                          // byte dot products per row word), the programs in the table [28..29]
#define CT_TAB_COVERED 0xFFFFFFFEu

struct DevSpace {
    uint32_t D;           // parameters
    uint32_t R;           // row bytes (4, 8, 16, 32)
    uint32_t n_cons;      // constraint programs
    uint32_t n_pre;       // programs [0, n_pre) only read parameters [0, split)
    uint32_t split;       // prefix parameters
    uint32_t max_radix;
    uint64_t N;           // Cartesian size
    uint64_t P_s;         // prod of prefix radices
    uint64_t I_s;         // prod of inner radices (< 2^31)
    uint32_t Is_m, Is_l;  // magic for I_s
    uint64_t n_valid;
    uint32_t radix[CT_DMAX];
    uint32_t mag_m[CT_DMAX];
    uint32_t mag_l[CT_DMAX];
    uint32_t val_off[CT_DMAX];
    uint64_t stride[CT_DMAX];
    uint32_t cons_off[CT_MAX_PROGRAMS + 1];
    const int64_t* values;      // concatenated value tables
    const uint32_t* code;       // bytecode
    const uint64_t* prefix_words;  // prefix validity bits [ceil(P_s/64)]
    uint32_t n_cx;              // context: prefix parameters read by programs [n_pre, n_cons)
    uint32_t cx[CT_DMAX];       // (stride << 5) | parameter, last context parameter fastest
    const uint32_t* tab_meta;   // [n_cons][CT_TAB_META] scope tables of the programs
    const uint64_t* tabs;       // the tables' bits
    const uint64_t* lin;        // valid list: ascending linear indices
    const uint8_t* rows;        // valid list: digit rows [n_valid][R]
    const uint8_t* prevnext;    // [D][256][2] nearest present value index below/above (0xFF: none)
    const uint64_t* words;      // validity bitmask [n_words]
    uint64_t n_words;
    const uint64_t* grp_off;    // valid configurations before each 64-word group
    const uint16_t* dir8;       // valid configurations from the group start to each 8-word block
    const uint8_t* boxes;       // per 64-row block of the valid list: min row, max row (2 * R bytes)
    uint64_t n_sub;             // number of 64-row blocks
    const uint8_t* chunks;      // per 64 boxes (4096 rows): the same min / max rows over its boxes
    uint64_t n_chunk;           // ceil(n_sub / 64)
};

// Validity of a linear index from the bitmask.
// Pointers read out of descriptor structs are generic: the compiler cannot tell device memory
// from LDS and issues flat accesses, which count against both the vector-memory and the LDS
// counters, so every cross-lane shuffle would wait for all loads in flight.  Hot loads go
// through these address-space-typed pointers instead.
#define CT_GLOBAL __attribute__((address_space(1)))
#define CT_LDS __attribute__((address_space(3)))
template <typename T>
__device__ __forceinline__ const CT_GLOBAL T* gptr(const T* p) { return (const CT_GLOBAL T*)p; }
template <typename T>
__device__ __forceinline__ T gld(const T* p) { return *(const CT_GLOBAL T*)p; }

__device__ __forceinline__ bool bit_valid(const DevSpace& S, uint64_t L) {
    return L < S.N && ((gld(S.words + (L >> 6)) >> (L & 63u)) & 1ull);
}

// Number of valid configurations with linear index below L (the rank of L when it is valid),
// from the group offsets, the 8-word directory and at most 8 word popcounts.  The word loads are
// unrolled and predicated, so they are in flight together rather than one after another.
__device__ __forceinline__ uint64_t rank_dir(const DevSpace& S, uint64_t L) {
    if (L >= S.N) return S.n_valid;
    const uint64_t w = L >> 6, q0 = w & ~7ull;
    const CT_GLOBAL uint64_t* words = gptr(S.words);
    uint64_t r = gld(S.grp_off + (w >> 6)) + gld(S.dir8 + (w >> 3));
#pragma unroll
    for (uint32_t t = 0; t < 8; ++t) {
        const uint64_t q = q0 + t;
        const uint64_t word = q <= w ? words[q] : 0ull;
        r += __popcll(q < w ? word : word & ((1ull << (L & 63u)) - 1ull));
    }
    return r;
}

// ---------------------------------------------------------------------------
// Exact q = x / d for all 32-bit x, with (m, l) precomputed for d:
//   l = ceil(log2 d), m = floor(2^32 (2^l - d) / d) + 1,
//   t = mulhi(m, x), q = (t + ((x - t) >> 1)) >> (l - 1)     (d >= 2)
// ---------------------------------------------------------------------------
__host__ __device__ inline void ct_magic(uint32_t d, uint32_t* m, uint32_t* l) {
    uint32_t ll = 0;
    while ((1ull << ll) < d) ll++;
    *l = ll;
    *m = d <= 1 ? 0u : (uint32_t)((((1ull << ll) - d) << 32) / d + 1);
}

__device__ __forceinline__ uint32_t ct_udiv(uint32_t x, uint32_t m, uint32_t l) {
    if (l == 0) return x;  // d == 1
    uint32_t t = __umulhi(m, x);
    return (t + ((x - t) >> 1)) >> (l - 1);
}

// ---------------------------------------------------------------------------
// Philox4x32-10: ten rounds of the Philox S-box network, multipliers
// 0xD2511F53 / 0xCD9E8D57, Weyl key increments 0x9E3779B9 / 0xBB67AE85.
// ---------------------------------------------------------------------------
struct U4 { uint32_t x, y, z, w; };

__device__ __forceinline__ U4 ct_philox(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3) {
    uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        uint32_t hi0 = __umulhi(0xD2511F53u, c0), lo0 = 0xD2511F53u * c0;
        uint32_t hi1 = __umulhi(0xCD9E8D57u, c2), lo1 = 0xCD9E8D57u * c2;
        uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
        k0 += 0x9E3779B9u; k1 += 0xBB67AE85u;
    }
    return U4{c0, c1, c2, c3};
}

// draw purposes (counter word 2, bits 24..31)
enum { PUR_INIT = 1, PUR_DE_PICK = 2, PUR_DE_CR = 3, PUR_PSO_R = 4, PUR_GA_SEL = 5, PUR_GA_MUT = 6,
       PUR_REPAIR_KEY = 7, PUR_MUT_KEY = 8, PUR_FF_NOISE = 9, PUR_GA_XO = 10 };

__device__ __forceinline__ uint32_t ct_below(uint32_t u, uint32_t n) {
    return (uint32_t)(((uint64_t)u * n) >> 32);
}

// ---------------------------------------------------------------------------
// Rows: digits packed as bytes, digit j in byte j.
// ---------------------------------------------------------------------------
// The words of a row are a vector value, not an array: an index known only at run time becomes a
// vector element extract/insert (register moves), where an indexed array would be placed in
// scratch memory (a memory round trip per access).
typedef uint32_t ct_u32x8 __attribute__((ext_vector_type(8)));
struct Row {
    ct_u32x8 w;
    __device__ __forceinline__ uint32_t digit(uint32_t j) const { return (w[j >> 2] >> ((j & 3u) * 8u)) & 0xFFu; }
    __device__ __forceinline__ void set(uint32_t j, uint32_t d) {
        const uint32_t q = j >> 2, sh = (j & 3u) * 8u;
        w[q] = (w[q] & ~(0xFFu << sh)) | (d << sh);
    }
};

__device__ __forceinline__ void row_load(Row& r, const uint8_t* p, uint32_t R) {
    const uint32_t* q = reinterpret_cast<const uint32_t*>(p);
#pragma unroll
    for (int k = 0; k < CT_DMAX / 4; ++k) r.w[k] = (uint32_t)k < R / 4 ? q[k] : 0u;
}

__device__ __forceinline__ void row_store(const Row& r, uint8_t* p, uint32_t R) {
    uint32_t* q = reinterpret_cast<uint32_t*>(p);
#pragma unroll
    for (int k = 0; k < CT_DMAX / 4; ++k)
        if ((uint32_t)k < R / 4) q[k] = r.w[k];
}

__device__ __forceinline__ uint64_t row_encode(const DevSpace& S, const Row& r) {
    uint64_t L = 0;
    for (uint32_t j = 0; j < S.D; ++j) L += (uint64_t)r.digit(j) * S.stride[j];
    return L;
}

__device__ __forceinline__ bool row_in_domain(const DevSpace& S, const Row& r) {
    bool ok = true;
    for (uint32_t j = 0; j < S.D; ++j) ok &= r.digit(j) < S.radix[j];
    return ok;
}

// digits [j0, j1) of x (x < prod_{j0<=j<j1} radix[j]), last digit fastest
__device__ __forceinline__ void decode_range(const DevSpace& S, uint32_t x, uint32_t j0, uint32_t j1, Row& r) {
    for (uint32_t j = j1; j-- > j0;) {
        uint32_t q = ct_udiv(x, S.mag_m[j], S.mag_l[j]);
        r.set(j, x - q * S.radix[j]);
        x = q;
    }
}

// full decode of a linear index via the (prefix, inner) split
__device__ __forceinline__ void decode_lin(const DevSpace& S, uint64_t L, Row& r) {
#pragma unroll
    for (int k = 0; k < CT_DMAX / 4; ++k) r.w[k] = 0;
    uint64_t p = L / S.I_s;
    uint32_t inner = (uint32_t)(L - p * S.I_s);
    decode_range(S, (uint32_t)p, 0, S.split, r);
    decode_range(S, inner, S.split, S.D, r);
}

// position of L in the ascending valid list, or -1
__device__ __forceinline__ int64_t rank_of(const DevSpace& S, uint64_t L) {
    uint64_t lo = 0, hi = S.n_valid;
    while (lo < hi) {
        uint64_t mid = (lo + hi) >> 1;
        if (S.lin[mid] < L) lo = mid + 1; else hi = mid;
    }
    return (lo < S.n_valid && S.lin[lo] == L) ? (int64_t)lo : -1;
}

// ---------------------------------------------------------------------------
// Constraint interpreter.  Every lane of a wave runs the same program, so the
// program counter, the opcode and the stack pointer are wave-uniform; values
// and poison bits are per lane.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int64_t ct_floordiv(int64_t a, int64_t b) {
    if (a == (int64_t)(int32_t)a && b == (int64_t)(int32_t)b && !(a == INT32_MIN && b == -1)) {
        int32_t a32 = (int32_t)a, b32 = (int32_t)b;
        int32_t q = a32 / b32, r = a32 - q * b32;
        if (r != 0 && ((r ^ b32) < 0)) q -= 1;
        return q;
    }
    int64_t q = a / b, r = a - q * b;
    if (r != 0 && ((r ^ b) < 0)) q -= 1;
    return q;
}

__device__ __forceinline__ int64_t ct_mod(int64_t a, int64_t b) {
    int64_t r;
    if (a == (int64_t)(int32_t)a && b == (int64_t)(int32_t)b && b != -1) {
        int32_t a32 = (int32_t)a, b32 = (int32_t)b;
        r = a32 % b32;
    } else {
        r = b == -1 ? 0 : a % b;
    }
    if (r != 0 && ((r ^ b) < 0)) r += b;
    return r;
}

// Evaluate programs [c0, c1) for one configuration; true iff all are truthy and none raised.
__device__ __forceinline__ bool ct_eval(const DevSpace& S, uint32_t c0, uint32_t c1, const Row& dig,
                                        const int64_t* __restrict__ vals) {
    bool ok = true;
    for (uint32_t c = c0; c < c1; ++c) {
        int64_t st[CT_STACK];
        uint32_t err = 0;
        int sp = 0;
        for (uint32_t pc = S.cons_off[c], end = S.cons_off[c + 1]; pc < end;) {
            uint32_t w = S.code[pc++];
            uint32_t op = w & 0xFFu;
            int32_t imm = (int32_t)w >> 8;
            if (op == OP_PARAM) {
                st[sp] = vals[S.val_off[imm] + dig.digit((uint32_t)imm)];
                err &= ~(1u << sp);
                ++sp;
            } else if (op == OP_CONST) {
                st[sp] = imm;
                err &= ~(1u << sp);
                ++sp;
            } else if (op == OP_CONST64) {
                uint64_t lo = S.code[pc], hi = S.code[pc + 1];
                pc += 2;
                st[sp] = (int64_t)(lo | (hi << 32));
                err &= ~(1u << sp);
                ++sp;
            } else if (op == OP_NEG) {
                st[sp - 1] = -st[sp - 1];
            } else if (op == OP_ABS) {
                st[sp - 1] = st[sp - 1] < 0 ? -st[sp - 1] : st[sp - 1];
            } else if (op == OP_NOT) {
                st[sp - 1] = st[sp - 1] == 0;
            } else {
                int64_t b = st[sp - 1], a = st[sp - 2];
                uint32_t eb = (err >> (sp - 1)) & 1u, ea = (err >> (sp - 2)) & 1u;
                uint32_t e = ea | eb;
                int64_t r = 0;
                switch (op) {
                case OP_ADD: r = a + b; break;
                case OP_SUB: r = a - b; break;
                case OP_MUL: r = a * b; break;
                case OP_FDIV: if (b == 0) e = 1; else r = ct_floordiv(a, b); break;
                case OP_MOD: if (b == 0) e = 1; else r = ct_mod(a, b); break;
                case OP_MIN: r = a < b ? a : b; break;
                case OP_MAX: r = a > b ? a : b; break;
                case OP_LT: r = a < b; break;
                case OP_LE: r = a <= b; break;
                case OP_GT: r = a > b; break;
                case OP_GE: r = a >= b; break;
                case OP_EQ: r = a == b; break;
                case OP_NE: r = a != b; break;
                case OP_AND:   // Python 'and': first operand if falsy, else the second
                    if (ea) e = 1; else if (a == 0) { r = a; e = 0; } else { r = b; e = eb; }
                    break;
                case OP_OR:    // Python 'or': first operand if truthy, else the second
                    if (ea) e = 1; else if (a != 0) { r = a; e = 0; } else { r = b; e = eb; }
                    break;
                default: e = 1; break;
                }
                --sp;
                st[sp - 1] = r;
                err = (err & ~(1u << (sp - 1))) | (e << (sp - 1));
            }
        }
        ok &= !(err & 1u) && st[0] != 0;
        if (!__any(ok)) break;
    }
    return ok;
}

// Programs [c0, c1) for one configuration: a table bit for programs with a scope table, the
// interpreter for the others.  Same result as ct_eval: a table holds the program's value for
// every combination of the parameters it reads, and no other digit can change it.  With
// kInterp = false every program of the range must have a table: the kernel then carries no
// interpreter (whose stack would put it in scratch memory).
template <bool kInterp = true>
__device__ __forceinline__ bool ct_valid(const DevSpace& S, uint32_t c0, uint32_t c1, const Row& dig,
                                         const int64_t* __restrict__ vals) {
    bool ok = true;
    for (uint32_t c = c0; c < c1; ++c) {
        const CT_GLOBAL uint32_t* m = gptr(S.tab_meta + c * CT_TAB_META);
        const uint32_t off = m[0];
        if (off == CT_TAB_COVERED) continue;              // tested by another program's table
        if (!kInterp || off != ~0u) {
            uint32_t lo = 0, hi = 0;
#pragma unroll
            for (uint32_t q = 0; q < CT_DMAX / 4; ++q) {
                if (q < S.R / 4) {
                    lo = __builtin_amdgcn_udot4(dig.w[q], m[12 + q], lo, false);
                    hi = __builtin_amdgcn_udot4(dig.w[q], m[20 + q], hi, false);
                }
            }
            const uint32_t idx = lo + (hi << 8);
            ok &= ((gld(S.tabs + off + (idx >> 6)) >> (idx & 63u)) & 1ull) != 0;
        } else {
            ok &= ct_eval(S, c, c + 1, dig, vals);
        }
        if (!__any(ok)) break;
    }
    return ok;
}
