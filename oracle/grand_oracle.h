/*
 * grand_oracle.h -- plain CPU oracle for GRAND decoding of Gray M-QAM
 * modulated polar codewords (arXiv 2405.01808).
 *
 * TEST INFRASTRUCTURE.  This header and grand_oracle.c are called only by the
 * tests, by the smoke check and by the benchmark's CPU-baseline leg.  The
 * product library neither includes this header nor links this code, and this
 * code includes nothing of the product.
 *
 * Parity is pinned for: code-construction checks (Definition "Polar codes"),
 * Algorithm 1 (Theorem 3.1, Table II at N = 128), demapping (Definitions 3.1
 * and 3.2 against brute-force Euclidean geometry), the TEP order (brute-force
 * sort of all subsets, Corollary 3.1 count), decoding (brute-force search
 * over all codewords for N <= 16) and Algorithm 2's symbol cut-off (the
 * selection against the geometric corner distance of Definition 3.1, the
 * decode against brute force over the selected symbols' candidates).  The Gray labelling convention and the
 * Q.12 quantisation are conventions the paper does not fix (parity unpinned
 * by the paper; pinned only by the Gray-adjacency and round-trip checks).
 */
#ifndef GRAND_ORACLE_H
#define GRAND_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_OK = 0, ORC_EINVAL = -1, ORC_ENOMEM = -2 };

/* Fixed-point scale of the demapper: received coordinates in lattice units
 * are multiplied by ORC_ONE (exact in binary floating point) and rounded
 * half-to-even to an integer. */
#define ORC_ONE 4096
#define ORC_COST_MAX 32767u

/* Demap one codeword (Algorithm 2 Step 1 with Definitions 3.1 and 3.2).
 * rx: 2L floats (a_1, b_1, ...), L = ceil(N / log2 M).
 * yhat: N bytes (0/1), the hard-decision word.
 * item_cost / item_pos: per (symbol, axis) in natural order, the cost of the
 * near-neighbour flip and the codeword bit it flips; flips that land on pad
 * bits are dropped.  *n_items receives the count (<= 2L).
 * Returns ORC_OK or ORC_EINVAL. */
int orc_demap(uint32_t N, uint32_t M, const float *rx, uint8_t *yhat,
              uint32_t *item_cost, uint32_t *item_pos, uint32_t *n_items);

/* Algorithm 1 (pMult) on a dense K x N 0/1 byte matrix H and a 0/1 byte
 * vector c: r = H c^T over GF(2).  Also reports the number of parallel steps
 * (one AND step plus the XOR-halving rounds), the AND count W_H and the
 * Theorem's XOR count sum_i ceil(log2 W_H(i)).  Any pointer among steps,
 * and_gates, xor_gates may be NULL. */
int orc_pmult(uint32_t K, uint32_t N, const uint8_t *H, const uint8_t *c,
              uint8_t *r, uint32_t *steps, uint64_t *and_gates,
              uint64_t *xor_gates);

/* The first `count` test error patterns in decoding order for n items whose
 * costs are already sorted ascending (cost_sorted[r] is the cost of rank r).
 * masks_out: count x ceil(n/64) words, bit r = rank r in the pattern.
 * costs_out: count sums.  Returns the number produced (< count only when all
 * 2^n patterns are exhausted), or a negative error. */
int64_t orc_enumerate(uint32_t n, const uint32_t *cost_sorted, uint64_t count,
                      uint64_t *masks_out, uint64_t *costs_out);

/* Full decode (Algorithm 2 with the ordering, cap and abandonment readings).
 * h_rows: rows x ceil(N/64) u64, bit j of row i in word i*ceil(N/64)+j/64.
 * codeword_out: ceil(N/64) u64.  On success *abandoned_out = 0 and *q_out is
 * the 1-based rank of the accepted pattern; on abandonment the hard word is
 * returned with *q_out = min(cap, 2^n) and *abandoned_out = 1. */
int orc_decode(uint32_t N, uint32_t rows, const uint64_t *h_rows,
               const float *rx, uint32_t M, double noise_var, uint64_t cap,
               uint64_t *codeword_out, uint64_t *q_out, uint8_t *abandoned_out);

/* Algorithm 2 Steps 1-3: rank the L symbols by L(r, s) of Definition 3.1
 * (compared as d1^2 + d2^2 of the two axes' near-neighbour costs, ties by
 * symbol index) and mark the first min(S, L), the least reliable, in
 * selected[0 .. L-1] (0/1 bytes).  *n_selected receives min(S, L).
 * Returns ORC_OK, ORC_EINVAL (S = 0 or bad arguments) or ORC_ENOMEM. */
int orc_select_symbols(uint32_t N, uint32_t M, const float *rx, uint32_t S,
                       uint8_t *selected, uint32_t *n_selected);

/* orc_decode with Algorithm 2's cut-off: with cutoff = S > 0 only the items
 * of the symbols orc_select_symbols marks take part, so the patterns are the
 * 4^S combinations of those symbols' candidates (fewer when pad bits drop
 * items) in the same order, and abandonment returns q = min(cap, 2^n) over
 * the kept items.  cutoff = 0 is orc_decode. */
int orc_decode_ex(uint32_t N, uint32_t rows, const uint64_t *h_rows,
                  const float *rx, uint32_t M, double noise_var, uint64_t cap,
                  uint32_t cutoff, uint64_t *codeword_out, uint64_t *q_out,
                  uint8_t *abandoned_out);

typedef struct {
    uint32_t N, rows, M;
    uint32_t cutoff;           /* 0: full pattern space; S > 0: Algorithm 2 cut-off */
    const uint64_t *h_rows;
    const float *rx;
    double noise_var;
    uint64_t cap;
    uint64_t *codeword_out;
    uint64_t *q_out;
    uint8_t *abandoned_out;
    int32_t status;
    int32_t pad1;
    double seconds;            /* wall time of this decode */
} orc_job;

/* Decode many independent codewords on `nthreads` POSIX threads (one decode
 * per task).  Returns the number of threads actually used. */
int orc_decode_many(orc_job *jobs, uint32_t count, uint32_t nthreads);

#ifdef __cplusplus
}
#endif
#endif
