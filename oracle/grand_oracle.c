/*
 * grand_oracle.c -- plain CPU oracle for GRAND decoding of Gray M-QAM
 * modulated polar codewords (arXiv 2405.01808, Sections II and III).
 *
 * TEST INFRASTRUCTURE.  Called only by the tests, the smoke check and the
 * benchmark's CPU-baseline leg; never by the product library.  It is written
 * for clarity, not speed: bits are bytes where that is clearer, the pattern
 * search is a textbook binary heap, and every syndrome is recomputed from the
 * hard word's syndrome and the pattern's columns.
 *
 * What is computed (readings of the paper are marked "reading"):
 *
 *  Quantisation (reading: the paper states real-valued arithmetic and no
 *  precision).  Each received coordinate x (lattice units) becomes the
 *  integer xq = round_half_even(4096 x).
 *
 *  Hard decision (Definition "M-QAM": amplitudes are odd integers).  The
 *  nearest amplitude A in {-(sqrtM-1), ..., sqrtM-1}; a value exactly on a
 *  decision boundary goes to the upper cell.
 *
 *  Near-neighbour cost (Definitions 3.1 and 3.2).  With delta = xq - 4096 A,
 *  the neighbour is A + 2 sigma with sigma = +1 for delta >= 0 and -1
 *  otherwise (reading: the paper leaves Sign(0) open); if that neighbour is
 *  outside the constellation the direction is reversed (reading: the paper's
 *  edge and corner remark keeps four points per symbol).  The cost is
 *  d = 4096 - sigma delta, which is Definition 3.1's d_1 (or d_2) = 1 - |A - a|
 *  in units of 1/4096 when the neighbour lies on the side of the received
 *  value, and 1 + |A - a| after a reversal; saturated at 32767.  The
 *  horizontal, vertical and diagonal candidates of Definition 3.2 are the
 *  flips of the in-phase bit, the quadrature bit and both (reading: the
 *  diagonal's penalty is d_1 + d_2, the additive AWGN penalty).
 *
 *  Labels (reading: the paper's Fig. 1 is not in the text).  Binary
 *  reflected Gray code per axis, level 0 = most negative, in-phase bits
 *  first, most significant bit first; pad bits beyond N are dropped.
 *
 *  Order (reading: Algorithm 2 tests all patterns at once and does not say
 *  which zero-syndrome pattern wins).  Items are ranked by (cost, bit
 *  position).  A pattern T (a set of ranks) has key (sum of costs, sum of
 *  2^rank); patterns are queried in ascending key order, the empty pattern
 *  first -- most likely first, as the GRAND maximum-likelihood argument of
 *  Section II requires.
 *
 *  Stop (Algorithm 2 Step 5; reading of the missing exit: abandonment after
 *  a query cap, as in GRAND-AB of Section I).  The first pattern whose
 *  syndrome H (yhat + e)^T is zero is returned with its 1-based query count;
 *  after `cap` queries, or after all 2^n patterns, the hard word is returned
 *  with the abandon flag set.
 */
#include "grand_oracle.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

/* ------------------------------------------------------------------ */
/* Argument checks shared by the decode entry points.                  */
/* ------------------------------------------------------------------ */

static int bits_per_axis(uint32_t M)
{
    for (int m = 1; m <= 6; m++)
        if (M == (1u << (2 * m)))
            return m;
    return 0;
}

static int valid_n(uint32_t N)
{
    return N >= 2 && N <= 1024 && (N & (N - 1)) == 0;
}

/* ------------------------------------------------------------------ */
/* Demapping: Algorithm 2 Step 1, Definitions 3.1 and 3.2.             */
/* ------------------------------------------------------------------ */

/* Nearest-amplitude decision and the near-neighbour cost on one axis.
 * levels = sqrt(M).  Outputs the amplitude index (0 = most negative), the
 * neighbour's index and the cost in units of 1/ORC_ONE. */
static void demap_axis(float x, int levels, int *idx, int *nbr_idx,
                       uint32_t *cost)
{
    double scaled = (double)x * (double)ORC_ONE;   /* exact: power of two */
    int32_t xq = (int32_t)rint(scaled);             /* round half to even */
    int32_t cell = (int32_t)floor((double)xq / (2.0 * ORC_ONE));
    int32_t A = 2 * cell + 1;
    if (A > levels - 1)
        A = levels - 1;
    if (A < -(levels - 1))
        A = -(levels - 1);
    int32_t delta = xq - A * ORC_ONE;
    int32_t sigma = (delta >= 0) ? 1 : -1;
    if (A + 2 * sigma > levels - 1 || A + 2 * sigma < -(levels - 1))
        sigma = -sigma;
    int64_t d = (int64_t)ORC_ONE - (int64_t)sigma * delta;
    if (d > ORC_COST_MAX)
        d = ORC_COST_MAX;
    *idx = (A + levels - 1) / 2;
    *nbr_idx = *idx + sigma;
    *cost = (uint32_t)d;
}

static int gray(int i) { return i ^ (i >> 1); }

int orc_demap(uint32_t N, uint32_t M, const float *rx, uint8_t *yhat,
              uint32_t *item_cost, uint32_t *item_pos, uint32_t *n_items)
{
    int m = bits_per_axis(M);
    if (!m || !valid_n(N) || !rx || !yhat || !item_cost || !item_pos || !n_items)
        return ORC_EINVAL;
    int levels = 1 << m;
    uint32_t L = (N + 2 * m - 1) / (2 * m);
    uint32_t count = 0;
    for (uint32_t i = 0; i < L; i++) {
        for (int axis = 0; axis < 2; axis++) {
            float x = rx[2 * i + axis];
            if (!isfinite(x) || fabsf(x) > 32768.0f)
                return ORC_EINVAL;
            int idx, nbr;
            uint32_t cost;
            demap_axis(x, levels, &idx, &nbr, &cost);
            int g = gray(idx);
            uint32_t base = 2u * m * i + (uint32_t)m * axis;
            for (int k = 0; k < m; k++) {         /* label bit k, MSB first */
                uint32_t p = base + k;
                if (p < N)
                    yhat[p] = (uint8_t)((g >> (m - 1 - k)) & 1);
            }
            int diff = g ^ gray(nbr);             /* exactly one bit set */
            int b = 0;
            while ((diff >> b) != 1)
                b++;
            uint32_t p = base + (uint32_t)(m - 1 - b);
            if (p < N) {
                item_cost[count] = cost;
                item_pos[count] = p;
                count++;
            }
        }
    }
    *n_items = count;
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Algorithm 1: pMult.                                                 */
/* ------------------------------------------------------------------ */

int orc_pmult(uint32_t K, uint32_t N, const uint8_t *H, const uint8_t *c,
              uint8_t *r, uint32_t *steps, uint64_t *and_gates,
              uint64_t *xor_gates)
{
    if (!H || !c || !r || K == 0 || N == 0)
        return ORC_EINVAL;
    uint8_t *terms = (uint8_t *)malloc(N);
    if (!terms)
        return ORC_ENOMEM;
    uint32_t max_rounds = 0;
    uint64_t ands = 0, xors = 0;
    for (uint32_t i = 0; i < K; i++) {
        /* Step 1: one product per element of the row's support. */
        uint32_t w = 0;
        for (uint32_t j = 0; j < N; j++)
            if (H[(size_t)i * N + j])
                terms[w++] = (uint8_t)(c[j] & H[(size_t)i * N + j]);
        ands += w;
        /* Step 2, repeated: add neighbouring terms pairwise; an unpaired
         * last term is carried to the next round (reading: the printed
         * floor(W/2) would drop it; ceil(W/2) matches the Theorem's step
         * count). */
        uint32_t rounds = 0;
        while (w > 1) {
            uint32_t half = (w + 1) / 2;
            for (uint32_t k = 0; k < w / 2; k++)
                terms[k] = terms[2 * k] ^ terms[2 * k + 1];
            if (w & 1)
                terms[w / 2] = terms[w - 1];
            w = half;
            rounds++;
        }
        xors += rounds;          /* Theorem: ceil(log2 W_H(i)) per row */
        if (rounds > max_rounds)
            max_rounds = rounds;
        r[i] = (w == 1) ? terms[0] : 0;
    }
    free(terms);
    if (steps)
        *steps = 1 + max_rounds;
    if (and_gates)
        *and_gates = ands;
    if (xor_gates)
        *xor_gates = xors;
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Pattern order: a best-first search over the successor tree.        */
/* ------------------------------------------------------------------ */
/*
 * Every nonempty pattern T with largest rank j has exactly one parent: T
 * without j when j-1 is in T, otherwise T with j replaced by j-1 (and {0}
 * has the empty pattern as parent).  The children of T are therefore
 * T + {j+1} and T - {j} + {j+1}.  Costs are sorted, so a child's key is
 * larger than its parent's; popping the smallest key from a heap that starts
 * with the empty pattern visits all patterns in ascending key order.
 */

typedef struct {
    uint32_t words;     /* u64 words per pattern mask */
    uint64_t cap;       /* nodes allocated */
    uint64_t used;
    uint64_t *mask;     /* used x words */
    uint64_t *cost;
    int32_t *maxrank;   /* -1 for the empty pattern */
    uint64_t *heap;     /* node ids */
    uint64_t heap_len;
} tep_search;

static int search_init(tep_search *s, uint32_t n, uint64_t reserve)
{
    memset(s, 0, sizeof(*s));
    s->words = (n + 63) / 64;
    s->cap = reserve < 16 ? 16 : reserve;
    s->mask = (uint64_t *)calloc(s->cap * s->words, sizeof(uint64_t));
    s->cost = (uint64_t *)malloc(s->cap * sizeof(uint64_t));
    s->maxrank = (int32_t *)malloc(s->cap * sizeof(int32_t));
    s->heap = (uint64_t *)malloc(s->cap * sizeof(uint64_t));
    return (s->mask && s->cost && s->maxrank && s->heap) ? ORC_OK : ORC_ENOMEM;
}

static void search_free(tep_search *s)
{
    free(s->mask);
    free(s->cost);
    free(s->maxrank);
    free(s->heap);
}

/* a < b in (cost, colex) order; colex compares the masks as integers. */
static int key_less(const tep_search *s, uint64_t a, uint64_t b)
{
    if (s->cost[a] != s->cost[b])
        return s->cost[a] < s->cost[b];
    for (int w = (int)s->words - 1; w >= 0; w--) {
        uint64_t x = s->mask[a * s->words + w], y = s->mask[b * s->words + w];
        if (x != y)
            return x < y;
    }
    return 0;
}

static int grow(tep_search *s)
{
    uint64_t nc = s->cap * 2;
    uint64_t *mask = (uint64_t *)realloc(s->mask, nc * s->words * sizeof(uint64_t));
    if (!mask)
        return ORC_ENOMEM;
    s->mask = mask;
    uint64_t *cost = (uint64_t *)realloc(s->cost, nc * sizeof(uint64_t));
    if (!cost)
        return ORC_ENOMEM;
    s->cost = cost;
    int32_t *mr = (int32_t *)realloc(s->maxrank, nc * sizeof(int32_t));
    if (!mr)
        return ORC_ENOMEM;
    s->maxrank = mr;
    uint64_t *heap = (uint64_t *)realloc(s->heap, nc * sizeof(uint64_t));
    if (!heap)
        return ORC_ENOMEM;
    s->heap = heap;
    s->cap = nc;
    return ORC_OK;
}

/* Append a node (copying `from`'s mask when from != UINT64_MAX) and push it. */
static int push_node(tep_search *s, uint64_t from, int32_t clear_rank,
                     int32_t set_rank, uint64_t cost)
{
    if (s->used == s->cap && grow(s) != ORC_OK)
        return ORC_ENOMEM;
    uint64_t id = s->used++;
    uint64_t *m = &s->mask[id * s->words];
    if (from != UINT64_MAX)
        memcpy(m, &s->mask[from * s->words], s->words * sizeof(uint64_t));
    else
        memset(m, 0, s->words * sizeof(uint64_t));
    if (clear_rank >= 0)
        m[clear_rank / 64] &= ~(1ull << (clear_rank % 64));
    if (set_rank >= 0)
        m[set_rank / 64] |= 1ull << (set_rank % 64);
    s->cost[id] = cost;
    s->maxrank[id] = set_rank;
    /* sift up */
    uint64_t i = s->heap_len++;
    s->heap[i] = id;
    while (i > 0) {
        uint64_t p = (i - 1) / 2;
        if (!key_less(s, s->heap[i], s->heap[p]))
            break;
        uint64_t t = s->heap[i];
        s->heap[i] = s->heap[p];
        s->heap[p] = t;
        i = p;
    }
    return ORC_OK;
}

static uint64_t pop_min(tep_search *s)
{
    uint64_t top = s->heap[0];
    s->heap[0] = s->heap[--s->heap_len];
    uint64_t i = 0;
    for (;;) {
        uint64_t l = 2 * i + 1, r = l + 1, m = i;
        if (l < s->heap_len && key_less(s, s->heap[l], s->heap[m]))
            m = l;
        if (r < s->heap_len && key_less(s, s->heap[r], s->heap[m]))
            m = r;
        if (m == i)
            break;
        uint64_t t = s->heap[i];
        s->heap[i] = s->heap[m];
        s->heap[m] = t;
        i = m;
    }
    return top;
}

/* Push the children of node `id` (largest rank j) given sorted costs. */
static int push_children(tep_search *s, uint64_t id, uint32_t n,
                         const uint32_t *cost_sorted)
{
    int32_t j = s->maxrank[id];
    if (j + 1 >= (int32_t)n)
        return ORC_OK;
    uint64_t c = s->cost[id];
    int rc = push_node(s, id, -1, j + 1, c + cost_sorted[j + 1]);
    if (rc == ORC_OK && j >= 0)
        rc = push_node(s, id, j, j + 1, c - cost_sorted[j] + cost_sorted[j + 1]);
    return rc;
}

int64_t orc_enumerate(uint32_t n, const uint32_t *cost_sorted, uint64_t count,
                      uint64_t *masks_out, uint64_t *costs_out)
{
    if (!cost_sorted || !masks_out || !costs_out || n == 0)
        return ORC_EINVAL;
    for (uint32_t r = 1; r < n; r++)
        if (cost_sorted[r] < cost_sorted[r - 1])
            return ORC_EINVAL;
    tep_search s;
    if (search_init(&s, n, 2 * count + 2) != ORC_OK) {
        search_free(&s);
        return ORC_ENOMEM;
    }
    int64_t produced = 0;
    if (push_node(&s, UINT64_MAX, -1, -1, 0) != ORC_OK)
        produced = ORC_ENOMEM;
    while (produced >= 0 && (uint64_t)produced < count && s.heap_len > 0) {
        uint64_t id = pop_min(&s);
        memcpy(&masks_out[(uint64_t)produced * s.words], &s.mask[id * s.words],
               s.words * sizeof(uint64_t));
        costs_out[produced] = s.cost[id];
        produced++;
        if (push_children(&s, id, n, cost_sorted) != ORC_OK)
            produced = ORC_ENOMEM;
    }
    search_free(&s);
    return produced;
}

/* ------------------------------------------------------------------ */
/* Symbol cut-off: Algorithm 2 Steps 1-3.                              */
/* ------------------------------------------------------------------ */

int orc_select_symbols(uint32_t N, uint32_t M, const float *rx, uint32_t S,
                       uint8_t *selected, uint32_t *n_selected)
{
    int m = bits_per_axis(M);
    if (!m || !valid_n(N) || !rx || !selected || !n_selected || S == 0)
        return ORC_EINVAL;
    int levels = 1 << m;
    uint32_t L = (N + 2 * m - 1) / (2 * m);
    uint64_t *lk = (uint64_t *)malloc(L * sizeof(uint64_t));
    uint32_t *order = (uint32_t *)malloc(L * sizeof(uint32_t));
    if (!lk || !order) {
        free(lk);
        free(order);
        return ORC_ENOMEM;
    }
    /* Step 1: the symbol's reliability L(r, s) = sqrt(d1^2 + d2^2) from
     * Definition 3.1, where d1 and d2 are the two axes' near-neighbour costs
     * (pad bits do not change them).  The square root is monotone, so the
     * integer d1^2 + d2^2 orders the symbols the same way. */
    for (uint32_t i = 0; i < L; i++) {
        uint32_t c[2];
        for (int axis = 0; axis < 2; axis++) {
            float x = rx[2 * i + axis];
            if (!isfinite(x) || fabsf(x) > 32768.0f) {
                free(lk);
                free(order);
                return ORC_EINVAL;
            }
            int idx, nbr;
            demap_axis(x, levels, &idx, &nbr, &c[axis]);
        }
        lk[i] = (uint64_t)c[0] * c[0] + (uint64_t)c[1] * c[1];
    }
    /* Step 2: pSort ascending (ties by symbol index: insertion sort is
     * stable).  Step 3: keep the first S symbols, the least reliable. */
    for (uint32_t i = 0; i < L; i++) {
        uint32_t k = i;
        order[k] = i;
        while (k > 0 && lk[order[k - 1]] > lk[order[k]]) {
            uint32_t t = order[k - 1];
            order[k - 1] = order[k];
            order[k] = t;
            k--;
        }
    }
    uint32_t keep = S < L ? S : L;
    memset(selected, 0, L);
    for (uint32_t r = 0; r < keep; r++)
        selected[order[r]] = 1;
    *n_selected = keep;
    free(lk);
    free(order);
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Decode: Algorithm 2.                                                */
/* ------------------------------------------------------------------ */

int orc_decode(uint32_t N, uint32_t rows, const uint64_t *h_rows,
               const float *rx, uint32_t M, double noise_var, uint64_t cap,
               uint64_t *codeword_out, uint64_t *q_out, uint8_t *abandoned_out)
{
    return orc_decode_ex(N, rows, h_rows, rx, M, noise_var, cap, 0, codeword_out, q_out,
                         abandoned_out);
}

int orc_decode_ex(uint32_t N, uint32_t rows, const uint64_t *h_rows,
                  const float *rx, uint32_t M, double noise_var, uint64_t cap,
                  uint32_t cutoff, uint64_t *codeword_out, uint64_t *q_out,
                  uint8_t *abandoned_out)
{
    int m = bits_per_axis(M);
    if (!m || !valid_n(N) || rows == 0 || rows >= N || !h_rows || !rx ||
        !codeword_out || !q_out || !abandoned_out || cap == 0 ||
        !isfinite(noise_var) || noise_var <= 0.0)
        return ORC_EINVAL;
    uint32_t L = (N + 2 * m - 1) / (2 * m);
    for (uint32_t i = 0; i < 2 * L; i++)
        if (!isfinite(rx[i]) || fabsf(rx[i]) > 32768.0f)
            return ORC_EINVAL;
    /* noise_var scales every penalty by the same positive factor 2/sigma^2,
     * so it cannot change the order; it is only validated. */

    uint32_t words_n = (N + 63) / 64;
    int rc = ORC_ENOMEM;
    uint8_t *yhat = (uint8_t *)calloc(N, 1);
    uint32_t *icost = (uint32_t *)malloc(2 * L * sizeof(uint32_t));
    uint32_t *ipos = (uint32_t *)malloc(2 * L * sizeof(uint32_t));
    uint32_t *order = (uint32_t *)malloc(2 * L * sizeof(uint32_t));
    uint32_t *cost_sorted = (uint32_t *)malloc(2 * L * sizeof(uint32_t));
    uint8_t *H = (uint8_t *)malloc((size_t)rows * N);
    uint8_t *s0 = (uint8_t *)malloc(rows);
    uint32_t kw = (rows + 63) / 64;           /* syndrome words */
    uint64_t *col = (uint64_t *)calloc((size_t)2 * L * kw, sizeof(uint64_t));
    uint64_t *syn0 = (uint64_t *)calloc(kw, sizeof(uint64_t));
    uint64_t *syn = (uint64_t *)calloc(kw, sizeof(uint64_t));
    uint8_t *sel = (uint8_t *)calloc(L, 1);
    tep_search s;
    memset(&s, 0, sizeof(s));
    if (!yhat || !icost || !ipos || !order || !cost_sorted || !H || !s0 ||
        !col || !syn0 || !syn || !sel)
        goto out;

    uint32_t n = 0;
    rc = orc_demap(N, M, rx, yhat, icost, ipos, &n);
    if (rc != ORC_OK)
        goto out;
    if (cutoff) {
        /* Algorithm 2 Steps 1-3: only the items of the S least reliable
         * symbols take part; Step 4's pattern set is then all their
         * combinations (4^S, fewer when pad bits drop items). */
        uint32_t kept = 0, nsel = 0;
        rc = orc_select_symbols(N, M, rx, cutoff, sel, &nsel);
        if (rc != ORC_OK)
            goto out;
        for (uint32_t i = 0; i < n; i++)
            if (sel[ipos[i] / (2u * (uint32_t)m)]) {
                icost[kept] = icost[i];
                ipos[kept] = ipos[i];
                kept++;
            }
        n = kept;
    }

    /* Algorithm 2 Step 2 (reading): rank the items by (cost, position);
     * insertion sort, n <= 2L <= 2048. */
    for (uint32_t i = 0; i < n; i++) {
        uint32_t k = i;
        order[k] = i;
        while (k > 0) {
            uint32_t a = order[k - 1], b = order[k];
            if (icost[a] < icost[b] || (icost[a] == icost[b] && ipos[a] < ipos[b]))
                break;
            order[k - 1] = b;
            order[k] = a;
            k--;
        }
    }
    for (uint32_t r = 0; r < n; r++)
        cost_sorted[r] = icost[order[r]];

    /* Dense H for Algorithm 1, and the columns H[:, p] per rank. */
    for (uint32_t i = 0; i < rows; i++)
        for (uint32_t j = 0; j < N; j++)
            H[(size_t)i * N + j] =
                (uint8_t)((h_rows[(size_t)i * words_n + j / 64] >> (j % 64)) & 1);
    for (uint32_t r = 0; r < n; r++) {
        uint32_t p = ipos[order[r]];
        for (uint32_t i = 0; i < rows; i++)
            if (H[(size_t)i * N + p])
                col[(size_t)r * kw + i / 64] |= 1ull << (i % 64);
    }

    /* Syndrome of the hard word, by Algorithm 1. */
    rc = orc_pmult(rows, N, H, yhat, s0, NULL, NULL, NULL);
    if (rc != ORC_OK)
        goto out;
    for (uint32_t i = 0; i < rows; i++)
        if (s0[i])
            syn0[i / 64] |= 1ull << (i % 64);

    /* Steps 4-5: query patterns in ascending key order.  By linearity,
     * H (yhat + e)^T = H yhat^T + sum of the columns of H selected by e. */
    rc = search_init(&s, n, 1024);
    if (rc != ORC_OK)
        goto out;
    rc = push_node(&s, UINT64_MAX, -1, -1, 0);
    if (rc != ORC_OK)
        goto out;
    uint64_t q = 0;
    int found = 0;
    uint64_t hit = 0;
    while (s.heap_len > 0 && q < cap) {
        uint64_t id = pop_min(&s);
        q++;
        memcpy(syn, syn0, kw * sizeof(uint64_t));
        for (uint32_t r = 0; r < n; r++)
            if ((s.mask[id * s.words + r / 64] >> (r % 64)) & 1)
                for (uint32_t w = 0; w < kw; w++)
                    syn[w] ^= col[(size_t)r * kw + w];
        int zero = 1;
        for (uint32_t w = 0; w < kw; w++)
            if (syn[w])
                zero = 0;
        if (zero) {
            found = 1;
            hit = id;
            break;
        }
        rc = push_children(&s, id, n, cost_sorted);
        if (rc != ORC_OK)
            goto out;
    }

    memset(codeword_out, 0, words_n * sizeof(uint64_t));
    for (uint32_t j = 0; j < N; j++)
        if (yhat[j])
            codeword_out[j / 64] |= 1ull << (j % 64);
    if (found) {
        for (uint32_t r = 0; r < n; r++)
            if ((s.mask[hit * s.words + r / 64] >> (r % 64)) & 1) {
                uint32_t p = ipos[order[r]];
                codeword_out[p / 64] ^= 1ull << (p % 64);
            }
    }
    *q_out = q;
    *abandoned_out = (uint8_t)(found ? 0 : 1);
    rc = ORC_OK;

out:
    search_free(&s);
    free(yhat);
    free(icost);
    free(ipos);
    free(order);
    free(cost_sorted);
    free(H);
    free(s0);
    free(col);
    free(syn0);
    free(syn);
    free(sel);
    return rc;
}

/* ------------------------------------------------------------------ */
/* Many decodes on a thread pool.                                      */
/* ------------------------------------------------------------------ */

typedef struct {
    orc_job *jobs;
    uint32_t count;
    uint32_t next;
    pthread_mutex_t lock;
} pool_state;

static double now_s(void)
{
    struct timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

static void *pool_worker(void *arg)
{
    pool_state *ps = (pool_state *)arg;
    for (;;) {
        pthread_mutex_lock(&ps->lock);
        uint32_t i = ps->next++;
        pthread_mutex_unlock(&ps->lock);
        if (i >= ps->count)
            break;
        orc_job *j = &ps->jobs[i];
        double t0 = now_s();
        j->status = orc_decode_ex(j->N, j->rows, j->h_rows, j->rx, j->M, j->noise_var,
                                  j->cap, j->cutoff, j->codeword_out, j->q_out,
                                  j->abandoned_out);
        j->seconds = now_s() - t0;
    }
    return NULL;
}

int orc_decode_many(orc_job *jobs, uint32_t count, uint32_t nthreads)
{
    if (nthreads < 1)
        nthreads = 1;
    if (nthreads > 256)
        nthreads = 256;
    if (nthreads > count && count > 0)
        nthreads = count;
    pool_state ps;
    ps.jobs = jobs;
    ps.count = count;
    ps.next = 0;
    pthread_mutex_init(&ps.lock, NULL);
    pthread_t th[256];
    uint32_t started = 0;
    for (uint32_t t = 1; t < nthreads; t++)
        if (pthread_create(&th[started], NULL, pool_worker, &ps) == 0)
            started++;
    pool_worker(&ps);
    for (uint32_t t = 0; t < started; t++)
        pthread_join(th[t], NULL);
    pthread_mutex_destroy(&ps.lock);
    return (int)(started + 1);
}
