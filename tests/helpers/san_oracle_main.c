/*
 * Driver that runs the oracle's C code (oracle/ct_oracle.c) in a standalone executable, so the
 * test suite can build it with AddressSanitizer and UndefinedBehaviorSanitizer (a sanitized
 * shared library could not be loaded into an unsanitized Python).  Test infrastructure only.
 *
 * Input file (int64 little endian throughout):
 *   D, radices[D], n_values, values[n_values], n_cons, n_expr, expr[n_expr], expr_off[n_cons],
 *   n_cand, cands[n_cand * D], pos_q16[n_cand * D], who[n_cand], key, gen
 * Output file: the bitmask words of the whole space, the validity of each candidate (one int64
 * each), then for metrics 0..4 the argmin position of every candidate (int64, -1 for none).
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t n_params;
    const int32_t* radices;
    const int64_t* values;
    int32_t n_cons;
    const int64_t* expr;
    const int64_t* expr_off;
} or_space;

typedef struct {
    int32_t n_params;
    int64_t n_valid;
    const int32_t* vrows;
    const uint64_t* vlin;
    const uint8_t* present;
} or_valid;

void or_mask_words(const or_space* s, uint64_t n_cartesian, uint64_t w0, uint64_t w1, uint64_t* words);
void or_valid_rows(const or_space* s, const int32_t* rows, int64_t n, uint8_t* out);
void or_decode_many(const or_space* s, const uint64_t* lin, int64_t n, int32_t* rows);
void or_argmin_many(const or_valid* V, const int32_t* cands, int64_t n, int metric, const int64_t* pos_q16,
                    uint32_t k0, uint32_t k1, const uint32_t* who, uint32_t gen, int64_t* out);

static FILE* in;

static int64_t rd(void) {
    int64_t v;
    if (fread(&v, 8, 1, in) != 1) {
        fprintf(stderr, "short input\n");
        exit(2);
    }
    return v;
}

static void* xcalloc(size_t n, size_t sz) {
    void* p = calloc(n ? n : 1, sz);
    if (!p) exit(3);
    return p;
}

int main(int argc, char** argv) {
    if (argc != 3) return 2;
    in = fopen(argv[1], "rb");
    if (!in) return 2;
    const int64_t D = rd();
    int32_t* radices = xcalloc((size_t)D, 4);
    uint64_t N = 1;
    for (int64_t j = 0; j < D; j++) {
        radices[j] = (int32_t)rd();
        N *= (uint64_t)radices[j];
    }
    const int64_t nv = rd();
    int64_t* values = xcalloc((size_t)nv, 8);
    for (int64_t k = 0; k < nv; k++) values[k] = rd();
    const int64_t n_cons = rd(), n_expr = rd();
    int64_t* expr = xcalloc((size_t)n_expr, 8);
    int64_t* expr_off = xcalloc((size_t)n_cons, 8);
    for (int64_t k = 0; k < n_expr; k++) expr[k] = rd();
    for (int64_t k = 0; k < n_cons; k++) expr_off[k] = rd();
    const int64_t n_cand = rd();
    int32_t* cands = xcalloc((size_t)(n_cand * D), 4);
    int64_t* pos = xcalloc((size_t)(n_cand * D), 8);
    uint32_t* who = xcalloc((size_t)n_cand, 4);
    for (int64_t k = 0; k < n_cand * D; k++) cands[k] = (int32_t)rd();
    for (int64_t k = 0; k < n_cand * D; k++) pos[k] = rd();
    for (int64_t k = 0; k < n_cand; k++) who[k] = (uint32_t)rd();
    const uint64_t key = (uint64_t)rd();
    const uint32_t gen = (uint32_t)rd();
    fclose(in);

    or_space s = {(int32_t)D, radices, values, (int32_t)n_cons, expr, expr_off};
    const uint64_t n_words = (N + 63) / 64;
    uint64_t* words = xcalloc((size_t)n_words, 8);
    or_mask_words(&s, N, 0, n_words, words);
    int64_t n_valid = 0;
    for (uint64_t w = 0; w < n_words; w++) n_valid += __builtin_popcountll(words[w]);
    uint64_t* vlin = xcalloc((size_t)n_valid, 8);
    int64_t k = 0;
    for (uint64_t w = 0; w < n_words; w++)
        for (int b = 0; b < 64; b++)
            if ((words[w] >> b) & 1u) vlin[k++] = w * 64 + (uint64_t)b;
    int32_t* vrows = xcalloc((size_t)(n_valid * D), 4);
    or_decode_many(&s, vlin, n_valid, vrows);
    uint8_t* present = xcalloc((size_t)(D * 256), 1);
    for (int64_t i = 0; i < n_valid; i++)
        for (int64_t j = 0; j < D; j++) present[j * 256 + vrows[i * D + j]] = 1;
    or_valid V = {(int32_t)D, n_valid, vrows, vlin, present};

    FILE* out = fopen(argv[2], "wb");
    if (!out) return 2;
    fwrite(words, 8, (size_t)n_words, out);
    uint8_t* ok = xcalloc((size_t)n_cand, 1);
    or_valid_rows(&s, cands, n_cand, ok);
    for (int64_t i = 0; i < n_cand; i++) {
        const int64_t v = ok[i];
        fwrite(&v, 8, 1, out);
    }
    int64_t* best = xcalloc((size_t)n_cand, 8);
    for (int metric = 0; metric <= 4; metric++) {
        if (n_valid) or_argmin_many(&V, cands, n_cand, metric, pos, (uint32_t)key, (uint32_t)(key >> 32), who, gen, best);
        fwrite(best, 8, (size_t)n_cand, out);
    }
    fclose(out);
    free(best); free(ok); free(present); free(vrows); free(vlin); free(words);
    free(who); free(pos); free(cands); free(expr_off); free(expr); free(values); free(radices);
    return 0;
}
