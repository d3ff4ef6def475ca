/*
 * Plain CPU oracle for the PIR Answer.  TEST INFRASTRUCTURE ONLY:
 * only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load this library.  It shares no code with the GPU path.
 *
 * What it computes follows the PIR interface of the paper (Definition 1: a
 * server turns a client query into a response derived from its local
 * database) in the single-server LWE form: the response is the database
 * matrix times the query vector over Z/2^32 (and, for the Goldberg
 * instantiation, over Z/p).  Every function is the plain
 * definition written out as loops; unsigned 32-bit arithmetic in C wraps
 * modulo 2^32, which is exactly the ring the answer lives in.  No blocking,
 * no reordering beyond the definition's sum, no intrinsics.  OpenMP splits
 * the independent output rows over threads; the per-row sums run in index
 * order.
 */
#include <stdint.h>
#include <stddef.h>
#include <stdlib.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Threads the OpenMP runtime will use for the parallel loops below. */
int oracle_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void oracle_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/*
 * Single-query Answer (the server's response to one query, Definition 1;
 * the batched form is the multi-request response of Section 5.2):
 *   a[r] = sum_{j<C} D[r][j] * q[j]  (mod 2^32)
 * D: R x C bytes, row r starting at D + r*pitch.  q: C words.  a: R words.
 */
void oracle_answer(const uint8_t* D, uint64_t R, uint64_t C, uint64_t pitch,
                   const uint32_t* q, uint32_t* a) {
    int64_t r;
#pragma omp parallel for schedule(static)
    for (r = 0; r < (int64_t)R; ++r) {
        const uint8_t* row = D + (uint64_t)r * pitch;
        uint32_t acc = 0;
        for (uint64_t j = 0; j < C; ++j) acc += (uint32_t)row[j] * q[j];
        a[r] = acc;
    }
}

/*
 * Batched Answer over selected rows:
 *   out[i][b] = sum_{j<C} D[rows[i]][j] * Q[j][b]  (mod 2^32)
 * Q: C x B words, row-major.  out: m x B words, row-major.  rows == NULL
 * means rows[i] = i.  Computing a subset of rows is what the full-size
 * checks use (each output row depends on one database row only); the
 * offline hint H = D * A is this function with Q = A and B = n.
 */
void oracle_answer_batch_rows(const uint8_t* D, uint64_t C, uint64_t pitch,
                              const uint64_t* rows, uint64_t m,
                              const uint32_t* Q, uint64_t B, uint32_t* out) {
    int64_t i;
#pragma omp parallel for schedule(static)
    for (i = 0; i < (int64_t)m; ++i) {
        uint64_t r = rows ? rows[i] : (uint64_t)i;
        const uint8_t* row = D + r * pitch;
        uint32_t* o = out + (uint64_t)i * B;
        for (uint64_t b = 0; b < B; ++b) o[b] = 0;
        for (uint64_t j = 0; j < C; ++j) {
            uint32_t d = row[j];
            const uint32_t* qj = Q + j * B;
            for (uint64_t b = 0; b < B; ++b) o[b] += d * qj[b];
        }
    }
}

/*
 * Word-by-word matrix-vector product over Z/2^32, used by the LWE client
 * (query A*s and decoding H*s):
 *   y[r] = sum_{k<n} M[r][k] * x[k]  (mod 2^32),  M: R x n words row-major.
 */
void oracle_matvec_u32(const uint32_t* M, uint64_t R, uint64_t n,
                       const uint32_t* x, uint32_t* y) {
    int64_t r;
#pragma omp parallel for schedule(static)
    for (r = 0; r < (int64_t)R; ++r) {
        const uint32_t* row = M + (uint64_t)r * n;
        uint32_t acc = 0;
        for (uint64_t k = 0; k < n; ++k) acc += row[k] * x[k];
        y[r] = acc;
    }
}

/*
 * Batched Answer over a prime field (the server product of the Goldberg /
 * FTR instantiation, Section 5.1; Algorithm 4's batched product "mod q"):
 *   out[i][b] = (sum_{j<C} D[rows[i]][j] * Q[j][b]) mod p
 * The sum is formed exactly in unsigned 128-bit integers (each term is
 * below 2^40) and reduced once.  Q: C x B words, out: m x B words,
 * rows == NULL means rows[i] = i.  Returns -1 if the accumulator buffer
 * cannot be allocated, else 0.
 */
int oracle_answer_batch_mod(const uint8_t* D, uint64_t C, uint64_t pitch,
                            const uint64_t* rows, uint64_t m, const uint32_t* Q,
                            uint64_t B, uint32_t p, uint32_t* out) {
    int failed = 0;
    int64_t i;
#pragma omp parallel for schedule(static)
    for (i = 0; i < (int64_t)m; ++i) {
        uint64_t r = rows ? rows[i] : (uint64_t)i;
        const uint8_t* row = D + r * pitch;
        unsigned __int128* acc = (unsigned __int128*)calloc(B ? B : 1, sizeof(unsigned __int128));
        if (!acc) {
#pragma omp atomic write
            failed = 1;
            continue;
        }
        for (uint64_t j = 0; j < C; ++j) {
            uint64_t d = row[j];
            const uint32_t* qj = Q + j * B;
            for (uint64_t b = 0; b < B; ++b) acc[b] += (unsigned __int128)(d * (uint64_t)qj[b]);
        }
        uint32_t* o = out + (uint64_t)i * B;
        for (uint64_t b = 0; b < B; ++b) o[b] = (uint32_t)(acc[b] % p);
        free(acc);
    }
    return failed ? -1 : 0;
}
