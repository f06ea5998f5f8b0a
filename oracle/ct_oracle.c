/*
 * Reference oracle for constraint-aware evolutionary auto-tuning -- TEST
 * INFRASTRUCTURE ONLY.  Plain, slow, scalar C; no blocking, no fusion, no
 * bit tricks.  It shares no code with the GPU library and is only loaded by
 * the tests, the smoke check and the benchmark's CPU-baseline leg.
 *
 * What it computes (each function cites the passage it follows):
 *   - constraint evaluation with Python integer semantics over the oracle's
 *     own expression-tree encoding (CSP definition, Section IV-A);
 *   - full enumeration of the valid set as a bitmask and an ascending list
 *     of linear indices (Section IV-A: all configurations are determined
 *     before tuning starts);
 *   - repair / neighbour argmin scans written from the definitions (the four
 *     neighbour rules of Section IV-A, Alg. 1 Repair, Alg. 2, Alg. 3);
 *   - the Philox4x32-10 counter-based generator (Salmon et al., SC'11).
 *
 * Overflow of any 64-bit intermediate is detected and reported, never
 * wrapped: the oracle refuses to give an answer it cannot compute exactly.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------------- */
/* Expression trees (prefix encoding produced by oracle/expr.py)           */
/* ---------------------------------------------------------------------- */
enum {
    T_NUM = 1, T_PARAM = 2, T_NEG = 3, T_NOT = 5, T_ABS = 6,
    T_ADD = 10, T_SUB = 11, T_MUL = 12, T_FDIV = 13, T_MOD = 14,
    T_MIN = 20, T_MAX = 21, T_CMP = 30, T_AND = 40, T_OR = 41
};
enum { C_LT = 0, C_LE = 1, C_GT = 2, C_GE = 3, C_EQ = 4, C_NE = 5 };

static int g_overflow = 0;

int or_overflow_flag(void) { return __atomic_load_n(&g_overflow, __ATOMIC_RELAXED); }
void or_clear_overflow(void) { __atomic_store_n(&g_overflow, 0, __ATOMIC_RELAXED); }
static void flag_overflow(void) { __atomic_store_n(&g_overflow, 1, __ATOMIC_RELAXED); }

/* Pointer just past the node starting at p. */
static const int64_t* skip(const int64_t* p) {
    int64_t tag = *p++;
    switch (tag) {
    case T_NUM: case T_PARAM: return p + 1;
    case T_NEG: case T_NOT: case T_ABS: return skip(p);
    case T_ADD: case T_SUB: case T_MUL: case T_FDIV: case T_MOD: return skip(skip(p));
    case T_MIN: case T_MAX: case T_AND: case T_OR: {
        int64_t n = *p++;
        for (int64_t i = 0; i < n; i++) p = skip(p);
        return p;
    }
    case T_CMP: {
        int64_t n = *p++;            /* number of operands; n-1 operator codes follow */
        p += n - 1;
        for (int64_t i = 0; i < n; i++) p = skip(p);
        return p;
    }
    }
    abort();
}

static int cmp_op(int64_t op, int64_t a, int64_t b) {
    switch (op) {
    case C_LT: return a < b;
    case C_LE: return a <= b;
    case C_GT: return a > b;
    case C_GE: return a >= b;
    case C_EQ: return a == b;
    case C_NE: return a != b;
    }
    abort();
}

/* Python floor division and modulo (b != 0). */
static int64_t py_floordiv(int64_t a, int64_t b) {
    if (a == INT64_MIN && b == -1) { flag_overflow(); return 0; }
    int64_t q = a / b;
    if ((a % b != 0) && ((a < 0) != (b < 0))) q -= 1;
    return q;
}
static int64_t py_mod(int64_t a, int64_t b) {
    if (b == -1) return 0;
    int64_t r = a % b;
    if (r != 0 && ((r < 0) != (b < 0))) r += b;
    return r;
}

/*
 * Evaluate the node at p with Python semantics.  Returns 0 and sets *out on
 * success; returns 1 where Python would raise (division or modulo by zero).
 * Evaluation stops at the first error; 'and', 'or' and chained comparisons
 * short-circuit exactly as Python does, so an operand that Python never
 * evaluates can never raise here either.
 */
static int eval(const int64_t* p, const int64_t* pv, int64_t* out) {
    int64_t tag = p[0];
    const int64_t* q = p + 1;
    int64_t a = 0, b = 0, r = 0;
    switch (tag) {
    case T_NUM: *out = q[0]; return 0;
    case T_PARAM: *out = pv[q[0]]; return 0;
    case T_NEG:
        if (eval(q, pv, &a)) return 1;
        if (a == INT64_MIN) flag_overflow();
        *out = -a; return 0;
    case T_NOT:
        if (eval(q, pv, &a)) return 1;
        *out = (a == 0); return 0;
    case T_ABS:
        if (eval(q, pv, &a)) return 1;
        if (a == INT64_MIN) flag_overflow();
        *out = a < 0 ? -a : a; return 0;
    case T_ADD: case T_SUB: case T_MUL: case T_FDIV: case T_MOD:
        if (eval(q, pv, &a)) return 1;
        if (eval(skip(q), pv, &b)) return 1;
        switch (tag) {
        case T_ADD: if (__builtin_add_overflow(a, b, &r)) flag_overflow(); break;
        case T_SUB: if (__builtin_sub_overflow(a, b, &r)) flag_overflow(); break;
        case T_MUL: if (__builtin_mul_overflow(a, b, &r)) flag_overflow(); break;
        case T_FDIV: if (b == 0) return 1; r = py_floordiv(a, b); break;
        default: if (b == 0) return 1; r = py_mod(a, b); break;
        }
        *out = r; return 0;
    case T_MIN: case T_MAX: {
        int64_t n = q[0];
        const int64_t* c = q + 1;
        int64_t best = 0;
        for (int64_t i = 0; i < n; i++) {
            if (eval(c, pv, &a)) return 1;
            if (i == 0 || (tag == T_MIN ? a < best : a > best)) best = a;
            c = skip(c);
        }
        *out = best; return 0;
    }
    case T_AND: case T_OR: {
        /* Python: 'and' returns the first falsy operand, else the last one;
           'or' returns the first truthy operand, else the last one. */
        int64_t n = q[0];
        const int64_t* c = q + 1;
        for (int64_t i = 0; i < n; i++) {
            if (eval(c, pv, &a)) return 1;
            if (i == n - 1) break;
            if (tag == T_AND && a == 0) break;
            if (tag == T_OR && a != 0) break;
            c = skip(c);
        }
        *out = a; return 0;
    }
    case T_CMP: {
        /* a op1 b op2 c ... == (a op1 b) and (b op2 c) and ..., each operand evaluated once */
        int64_t n = q[0];
        const int64_t* ops = q + 1;
        const int64_t* c = q + n;  /* first operand */
        if (eval(c, pv, &a)) return 1;
        for (int64_t i = 1; i < n; i++) {
            c = skip(c);
            if (eval(c, pv, &b)) return 1;
            if (!cmp_op(ops[i - 1], a, b)) { *out = 0; return 0; }
            a = b;
        }
        *out = 1; return 0;
    }
    }
    abort();
}

/* ---------------------------------------------------------------------- */
/* Search space: the CSP (X, D, C) of Section IV-A                         */
/* ---------------------------------------------------------------------- */
typedef struct {
    int32_t n_params;
    const int32_t* radices;     /* |D_j| */
    const int64_t* values;      /* D_j concatenated in parameter order */
    int32_t n_cons;
    const int64_t* expr;        /* constraint trees concatenated */
    const int64_t* expr_off;    /* start of each constraint in expr */
} or_space;

/* Value offsets of each parameter inside s->values. */
static void value_offsets(const or_space* s, int64_t* off) {
    int64_t o = 0;
    for (int j = 0; j < s->n_params; j++) { off[j] = o; o += s->radices[j]; }
}

/*
 * A configuration (given by its value indices) is a solution iff every
 * constraint evaluates without raising and is truthy (Section IV-A).
 */
static int config_valid(const or_space* s, const int64_t* off, const int32_t* digits) {
    int64_t pv[64];
    for (int j = 0; j < s->n_params; j++) pv[j] = s->values[off[j] + digits[j]];
    for (int c = 0; c < s->n_cons; c++) {
        int64_t v;
        if (eval(s->expr + s->expr_off[c], pv, &v)) return 0;
        if (v == 0) return 0;
    }
    return 1;
}

/* Mixed-radix decode, last parameter fastest (itertools.product order). */
static void decode(const or_space* s, uint64_t L, int32_t* digits) {
    for (int j = s->n_params - 1; j >= 0; j--) {
        digits[j] = (int32_t)(L % (uint64_t)s->radices[j]);
        L /= (uint64_t)s->radices[j];
    }
}

static uint64_t encode(const or_space* s, const int32_t* digits) {
    uint64_t L = 0;
    for (int j = 0; j < s->n_params; j++) L = L * (uint64_t)s->radices[j] + (uint64_t)digits[j];
    return L;
}

int or_valid_digits(const or_space* s, const int32_t* digits) {
    int64_t off[64];
    value_offsets(s, off);
    return config_valid(s, off, digits);
}

/* Validity of n rows of digits (row-major n x n_params). */
void or_valid_rows(const or_space* s, const int32_t* rows, int64_t n, uint8_t* out) {
    int64_t off[64];
    value_offsets(s, off);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) out[i] = (uint8_t)config_valid(s, off, rows + i * s->n_params);
}

/*
 * Validity bitmask over linear indices [64*w0, 64*w1): bit (L mod 64) of
 * word L/64 is set iff configuration L is a solution.  Indices at or beyond
 * n_cartesian are left clear.
 */
void or_mask_words(const or_space* s, uint64_t n_cartesian, uint64_t w0, uint64_t w1, uint64_t* words) {
    int64_t off[64];
    value_offsets(s, off);
#pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t w = (int64_t)w0; w < (int64_t)w1; w++) {
        uint64_t word = 0;
        for (int b = 0; b < 64; b++) {
            uint64_t L = (uint64_t)w * 64u + (uint64_t)b;
            if (L >= n_cartesian) break;
            int32_t d[64];
            decode(s, L, d);
            if (config_valid(s, off, d)) word |= (uint64_t)1 << b;
        }
        words[w - (int64_t)w0] = word;
    }
}

/* Validity of arbitrary linear indices. */
void or_valid_lin(const or_space* s, const uint64_t* lin, int64_t n, uint8_t* out) {
    int64_t off[64];
    value_offsets(s, off);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) {
        int32_t d[64];
        decode(s, lin[i], d);
        out[i] = (uint8_t)config_valid(s, off, d);
    }
}

void or_decode_many(const or_space* s, const uint64_t* lin, int64_t n, int32_t* rows) {
    for (int64_t i = 0; i < n; i++) decode(s, lin[i], rows + i * s->n_params);
}

void or_encode_many(const or_space* s, const int32_t* rows, int64_t n, uint64_t* lin) {
    for (int64_t i = 0; i < n; i++) lin[i] = encode(s, rows + i * s->n_params);
}

/* ---------------------------------------------------------------------- */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of the    */
/* Philox S-box network with the published multipliers and Weyl key bumps. */
/* ---------------------------------------------------------------------- */
void or_philox(uint32_t k0, uint32_t k1, const uint32_t ctr[4], uint32_t out[4]) {
    const uint64_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    for (int round = 0; round < 10; round++) {
        uint64_t p0 = M0 * (uint64_t)x0;
        uint64_t p1 = M1 * (uint64_t)x2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
        k0 += W0; k1 += W1;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

void or_philox_many(uint32_t k0, uint32_t k1, const uint32_t* ctrs, int64_t n, uint32_t* outs) {
    for (int64_t i = 0; i < n; i++) or_philox(k0, k1, ctrs + 4 * i, outs + 4 * i);
}

/* ---------------------------------------------------------------------- */
/* Neighbour rules (Section IV-A) and repair argmin scans                  */
/* ---------------------------------------------------------------------- */
enum { M_HAMMING = 0, M_INDEX_L1 = 1, M_TIER_EUCLID = 2, M_TIER_RANDOM = 3, M_HAM1_RANDOM = 4 };
enum { PURPOSE_REPAIR_KEY = 7, PURPOSE_MUT_KEY = 8 };

typedef struct {
    int32_t n_params;
    int64_t n_valid;
    const int32_t* vrows;       /* n_valid x n_params value indices, ascending linear index */
    const uint64_t* vlin;       /* n_valid linear indices, ascending */
    const uint8_t* present;     /* n_params x 256: value index k of parameter j occurs in some solution */
} or_valid;

static int hamming(int D, const int32_t* c, const int32_t* v) {
    int h = 0;
    for (int j = 0; j < D; j++) h += (c[j] != v[j]);
    return h;
}

static int64_t index_l1(int D, const int32_t* c, const int32_t* v) {
    int64_t s = 0;
    for (int j = 0; j < D; j++) s += (c[j] > v[j]) ? (c[j] - v[j]) : (v[j] - c[j]);
    return s;
}

/* Strictly adjacent: every parameter identical or the previous/next value index. */
static int strictly_adjacent(int D, const int32_t* c, const int32_t* v) {
    for (int j = 0; j < D; j++) {
        int d = v[j] - c[j];
        if (d < -1 || d > 1) return 0;
    }
    return 1;
}

/* Nearest value index below / above k of parameter j that occurs in some solution (-1: none). */
static int prev_present(const or_valid* V, int j, int k) {
    for (int t = k - 1; t >= 0; t--) if (V->present[j * 256 + t]) return t;
    return -1;
}
static int next_present(const or_valid* V, int j, int k) {
    for (int t = k + 1; t < 256; t++) if (V->present[j * 256 + t]) return t;
    return -1;
}

/* Adjacent: every parameter identical, or the nearest previous/next value that occurs in a solution. */
static int adjacent(const or_valid* V, const int32_t* c, const int32_t* v) {
    for (int j = 0; j < V->n_params; j++) {
        if (v[j] == c[j]) continue;
        if (v[j] == prev_present(V, j, c[j])) continue;
        if (v[j] == next_present(V, j, c[j])) continue;
        return 0;
    }
    return 1;
}

/* First non-empty neighbour set of Alg. 2 / Alg. 3 as a tier: 0 strictly adjacent, 1 adjacent, 2 Hamming, 3 none. */
static int tier_of(const or_valid* V, const int32_t* c, const int32_t* v) {
    if (strictly_adjacent(V->n_params, c, v)) return 0;
    if (adjacent(V, c, v)) return 1;
    if (hamming(V->n_params, c, v) == 1) return 2;
    return 3;
}

static uint32_t random_key(uint32_t k0, uint32_t k1, uint32_t who, uint32_t gen, uint32_t purpose, uint64_t L) {
    uint32_t ctr[4] = {who, gen, (purpose << 24) | (uint32_t)((L >> 32) & 0xFFFFFFu), (uint32_t)L};
    uint32_t out[4];
    or_philox(k0, k1, ctr, out);
    return out[0];
}

/* Centre of value index k in Q16.16 index units: (k + 1/2) * 2^16. */
static int64_t centre_q16(int32_t k) { return (2 * (int64_t)k + 1) * 32768; }

/*
 * Argmin over the valid list of a lexicographic key (k1, k2, L) for one
 * candidate c; ties in (k1, k2) resolve to the lowest linear index because
 * the list is scanned in ascending order and only strictly smaller keys
 * replace the incumbent.  Returns the position in the valid list, or -1
 * when no valid row has a finite key (only possible for HAM1_RANDOM).
 *
 *   HAMMING      k1 = #differing parameters                       (neighbour rule "Hamming")
 *   INDEX_L1     k1 = sum |index differences|                     (rule "index-distance"; Alg. 1 Repair)
 *   TIER_EUCLID  k1 = tier, k2 = squared distance to position X    (Alg. 2) -- tier 3 ranks by Hamming
 *   TIER_RANDOM  k1 = tier, k2 = Philox draw per (candidate, L)    (Alg. 3) -- tier 3 ranks by Hamming
 *   HAM1_RANDOM  k1 = 0 for Hamming-1 rows else none, k2 = draw    (GA mutation, Section IV-D)
 */
int64_t or_argmin(const or_valid* V, const int32_t* c, int metric, const int64_t* pos_q16,
                  uint32_t k0, uint32_t k1, uint32_t who, uint32_t gen) {
    int D = V->n_params;
    int64_t best = -1;
    uint64_t best1 = 0, best2 = 0;
    for (int64_t i = 0; i < V->n_valid; i++) {
        const int32_t* v = V->vrows + i * D;
        uint64_t key1 = 0, key2 = 0;
        int t;
        switch (metric) {
        case M_HAMMING: key1 = (uint64_t)hamming(D, c, v); break;
        case M_INDEX_L1: key1 = (uint64_t)index_l1(D, c, v); break;
        case M_TIER_EUCLID:
            t = tier_of(V, c, v);
            key1 = (uint64_t)t;
            if (t < 3) {
                uint64_t s = 0;
                for (int j = 0; j < D; j++) {
                    int64_t d = pos_q16[j] - centre_q16(v[j]);
                    s += (uint64_t)(d * d);
                }
                key2 = s;
            } else {
                key2 = (uint64_t)hamming(D, c, v);
            }
            break;
        case M_TIER_RANDOM:
            t = tier_of(V, c, v);
            key1 = (uint64_t)t;
            key2 = (t < 3) ? random_key(k0, k1, who, gen, PURPOSE_REPAIR_KEY, V->vlin[i])
                           : (uint64_t)hamming(D, c, v);
            break;
        case M_HAM1_RANDOM:
            if (hamming(D, c, v) != 1) continue;
            key2 = random_key(k0, k1, who, gen, PURPOSE_MUT_KEY, V->vlin[i]);
            break;
        default: abort();
        }
        if (best < 0 || key1 < best1 || (key1 == best1 && key2 < best2)) {
            best = i; best1 = key1; best2 = key2;
        }
    }
    return best;
}

/* Many candidates at once (independent scans, one per candidate). */
void or_argmin_many(const or_valid* V, const int32_t* cands, int64_t n, int metric, const int64_t* pos_q16,
                    uint32_t k0, uint32_t k1, const uint32_t* who, uint32_t gen, int64_t* out) {
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < n; i++)
        out[i] = or_argmin(V, cands + i * V->n_params, metric,
                           pos_q16 ? pos_q16 + i * V->n_params : NULL, k0, k1, who[i], gen);
}

void or_set_num_threads(int n) {
#ifdef _OPENMP
    extern void omp_set_num_threads(int);
    omp_set_num_threads(n < 1 ? 1 : n);
#else
    (void)n;
#endif
}

int or_num_threads(void) {
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}
