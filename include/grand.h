/*
 * grand.h -- C ABI of the MI355X (gfx950) GRAND decoder for Gray M-QAM
 * modulated polar codewords (arXiv 2405.01808).
 *
 * The decoder follows Algorithm 2 of Section III: per-symbol likelihoods and
 * near-neighbour candidates (Definitions 3.1 and 3.2), test error patterns
 * queried from most to least likely, the syndrome H (yhat + e)^T evaluated
 * for each pattern (Algorithm 1 for the hard word, column updates for the
 * patterns), stopping at the first zero syndrome.  The paper leaves the loop
 * without an exit; this library abandons after a query cap, as GRAND-AB does
 * (Section I), and reports the abandonment in a flag, not as an error.
 *
 * Conventions fixed by this library (the paper does not fix them):
 *   - received coordinates are in odd-integer lattice units (Section II,
 *     Definition "M-QAM": values divided by d of Eq. 2);
 *   - each coordinate is quantised to round_half_even(4096 x); every cost is
 *     an integer in units of 1/4096, saturated at 32767;
 *   - Gray labels: binary reflected per axis, level 0 = most negative
 *     amplitude, in-phase bits first, most significant bit first; bits of the
 *     last symbol beyond N are pad bits and are never flipped;
 *   - patterns are queried in ascending (sum of costs, colex order of item
 *     ranks), items being ranked by (cost, bit position);
 *   - the query count q is the 1-based rank of the accepted pattern in that
 *     order (the hard word itself is query 1).
 *
 * All functions return GRAND_OK (0) or a negative error code.  On error the
 * outputs are left untouched.  Functions may be called from several host
 * threads; calls that share a stream are serialised by the caller.
 */
#ifndef GRAND_H
#define GRAND_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    GRAND_OK = 0,
    GRAND_EINVAL = -1,    /* bad argument (null pointer, size, M, cap, noise variance, rx value) */
    GRAND_ENOMEM = -2,    /* host or device allocation failed */
    GRAND_EDEVICE = -3,   /* a HIP runtime call failed; see grand_last_error() */
    GRAND_EBUSY = -4,     /* server admission refused (memory budget or slot table full) */
    GRAND_ECAPACITY = -5, /* a decode needed more high-subset store than configured */
    GRAND_ENOTFOUND = -6  /* server: no such request, or nothing completed */
};

/* Largest supported block length and query cap. */
#define GRAND_MAX_N 1024u
#define GRAND_MAX_CAP (1ull << 40)

/* Human-readable text for an error code (static storage). */
const char *grand_strerror(int err);

/* Detail of the last error raised on the calling host thread ("" if none). */
const char *grand_last_error(void);

/* Select the HIP device used by this thread's subsequent calls and
 * initialise the library on it.  Optional: every call initialises the
 * current device on first use. */
int grand_init(int device);

/* ------------------------------------------------------------------ */
/* Codes                                                               */
/* ------------------------------------------------------------------ */

typedef struct grand_code grand_code;

/* Create a decoder handle for the code with parity-check matrix H
 * (Definition "Polar codes", Section II: H is (N - K) x N with
 * G_I H^T = 0; any matrix is accepted, the decoder only tests H x^T = 0).
 *   n      block length N, a power of two, 2 <= n <= 1024;
 *   rows   number of rows of H, 1 <= rows < n (rows <= 512);
 *   h_rows host pointer, rows x ceil(n/64) uint64 words, row-major; bit j of
 *          row i is bit (j % 64) of word i*ceil(n/64) + j/64.  Bits at
 *          j >= n must be zero.
 * The library copies H (row-packed for Algorithm 1 and column-packed for
 * the pattern updates) to the current device; the caller keeps ownership of
 * h_rows.  The handle is immutable and may be shared between threads. */
int grand_code_create(uint32_t n, uint32_t rows, const uint64_t *h_rows,
                      grand_code **out);
void grand_code_destroy(grand_code *code);
uint32_t grand_code_n(const grand_code *code);
uint32_t grand_code_rows(const grand_code *code);

/* ------------------------------------------------------------------ */
/* One decode, host buffers, synchronous (Algorithm 2 for one word).   */
/* ------------------------------------------------------------------ */

/* rx         host pointer, 2L floats (a_1, b_1, a_2, b_2, ...), L =
 *            ceil(n / log2 M); each finite with |x| <= 32768;
 * M          4, 16, 64, 256, 1024 or 4096;
 * noise_var  per-dimension noise variance in lattice units, finite and > 0.
 *            It scales every penalty alike, so it cannot change the order
 *            of the patterns; it is validated only;
 * query_cap  1 <= cap <= GRAND_MAX_CAP;
 * codeword_out host pointer, ceil(n/64) uint64 words (bit order as h_rows);
 * queries_out, abandoned_out host pointers.
 * On success with abandoned = 0 the codeword satisfies H x^T = 0 and q is
 * the query count; with abandoned = 1 the hard-decision word is returned
 * and q = min(cap, 2^(number of candidate flips)). */
int grand_decode(const grand_code *code, const float *rx, uint32_t M,
                 float noise_var, uint64_t query_cap, uint64_t *codeword_out,
                 uint64_t *queries_out, uint8_t *abandoned_out);

/* grand_decode with Algorithm 2's symbol cut-off (Steps 1-3 and Section IV,
 * where S = 8).  The L symbols are ranked by Definition 3.1's reliability
 * L(r, s) = sqrt(d1^2 + d2^2) (compared as d1^2 + d2^2 of the two axes'
 * near-neighbour costs, ties by symbol index), and only the flips of the
 * first min(S, L) -- the least reliable -- take part: the patterns are the
 * 4^S combinations of their candidates (fewer when pad bits drop flips), in
 * the same order as grand_decode, and a search that finds no codeword
 * abandons with q = min(query_cap, 2^n) over the kept flips.
 * cutoff_symbols = 0, or >= L, is grand_decode.  Same arguments, ownership
 * and errors as grand_decode. */
int grand_decode_ex(const grand_code *code, const float *rx, uint32_t M,
                    float noise_var, uint64_t query_cap, uint32_t cutoff_symbols,
                    uint64_t *codeword_out, uint64_t *queries_out, uint8_t *abandoned_out);

/* ------------------------------------------------------------------ */
/* Many decodes, device buffers, asynchronous on a HIP stream.         */
/* ------------------------------------------------------------------ */

/* Per-codeword metadata lives in host memory (it drives the launch plan:
 * codewords are grouped into (n, M) buckets, each with its own tuned launch
 * shape); bulk data lives in device memory. */
typedef struct {
    uint32_t count;                /* number of codewords */
    uint32_t n_codes;              /* entries in codes[] */
    const grand_code *const *codes;/* host array of code handles */
    const uint32_t *code_index;    /* host [count]: codes[code_index[i]] decodes word i */
    const uint32_t *M;             /* host [count] */
    const uint64_t *query_cap;     /* host [count] */
    const float *noise_var;        /* host [count] (validated only) */
    const uint64_t *rx_offset;     /* host [count]: float offset of word i's 2L values in rx */
    const float *rx;               /* device */
    uint64_t *codeword_out;        /* device [count * 16] uint64: word i at i*16, ceil(n/64) used */
    uint64_t *queries_out;         /* device [count] */
    uint8_t *abandoned_out;        /* device [count] */
    int32_t *status_out;           /* device [count]: GRAND_OK, GRAND_EINVAL (bad rx values)
                                      or GRAND_ECAPACITY; may be NULL.  A word that fails
                                      (any nonzero status) gets q = 0, abandoned = 1 and
                                      an all-zero codeword, so the failure shows without
                                      status_out (a decode never yields q = 0) */
    uint64_t *checks_out;          /* device [count]: syndrome checks actually performed
                                      (>= q; includes speculative checks); may be NULL */
    uint32_t cutoff_symbols;       /* Algorithm 2's cut-off S for every word: 0 searches the
                                      full pattern space; S > 0 keeps only the flips of the
                                      S least reliable symbols (Steps 1-3), as in
                                      grand_decode_ex */
    uint32_t launch_mode;          /* GRAND_LAUNCH_AUTO: one launch per (n, M) bucket when some
                                      bucket fills the device alone, else one merged launch;
                                      GRAND_LAUNCH_MERGED: one launch for every word;
                                      GRAND_LAUNCH_BUCKETS: one launch per (n, M) bucket, each
                                      with that bucket's tuning.  Results do not depend on it */
    uint64_t rx_count;             /* floats in rx (> 0): every word's 2L values,
                                      rx_offset[i] .. rx_offset[i] + 2L - 1, must lie
                                      below it, or the call fails with GRAND_EINVAL */
} grand_batch;

enum { GRAND_LAUNCH_AUTO = 0, GRAND_LAUNCH_MERGED = 1, GRAND_LAUNCH_BUCKETS = 2 };

/* Algorithm 2 (Section III) for every codeword of the batch, each word
 * decoded exactly as grand_decode decodes it (grand_decode_ex with the
 * batch's cutoff_symbols).
 * Enqueue the decode of every codeword of the batch on `stream` (a
 * hipStream_t; NULL = the default stream) and return.  Outputs are valid
 * once the stream has completed.  Host-side validation errors are returned
 * directly and nothing is enqueued.  The host arrays are read during the
 * call only: the library builds the batch's job table from them and copies
 * it to device memory it keeps per stream.  A call whose table is identical
 * to the one last copied for the same stream (the same batch launched
 * again) uses that copy instead of copying it again. */
int grand_decode_batch(const grand_batch *batch, void *stream);

/* ------------------------------------------------------------------ */
/* Many decodes without any allocation                                 */
/* ------------------------------------------------------------------ */

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the batch
 * decode of grand_decode_batch, with the same arguments, validation, errors
 * and outputs (bit-identical results), that allocates nothing.  Its work
 * counter, per-word tables and high-subset node stores live in one static
 * device array of GRAND_NOALLOC_SCRATCH_BYTES that every device the library
 * runs on holds until the process ends.
 *   - at most GRAND_NOALLOC_MAX_WORDS codewords and GRAND_NOALLOC_MAX_CODES
 *     codes per call (larger batches: GRAND_EINVAL, nothing enqueued);
 *   - the words run as one launch in the caller's order (whatever
 *     launch_mode asks), with node stores of
 *     16384 nodes per workgroup (the default store holds 65536): a word that
 *     cannot reach its answer or cap within them reports GRAND_ECAPACITY in
 *     status_out (q = 0, abandoned = 1).  (Measured largest stores: 10690
 *     nodes over the 8192 words of the N = 128 16-QAM batch, 27171 over
 *     8192 words of the uneven N = 64..512 mix, up to 65256 for N = 1024
 *     256-QAM at cap 2^20.);
 *   - the per-word host arrays are copied to the device before the call
 *     returns, so the call waits for work already queued on `stream` (it
 *     cannot be recorded into a HIP graph);
 *   - every call on a device shares that device's array, and the last call
 *     leaves its contents there: calls whose launches overlap on one device
 *     (on different streams or threads) race and give wrong results.  Issue
 *     them on one stream, or order them.
 * grand_init takes the array's device address; otherwise the first call on
 * a device does. */
#define GRAND_NOALLOC_SCRATCH_BYTES (512ull << 20)
#define GRAND_NOALLOC_MAX_WORDS 65536u
#define GRAND_NOALLOC_MAX_CODES 64u
int grand_decode_batch_noalloc(const grand_batch *batch, void *stream);

/* ------------------------------------------------------------------ */
/* Batch graphs (for callers that decode batches of one fixed shape    */
/* over and over, e.g. a receiver's frames: one call per batch)        */
/* ------------------------------------------------------------------ */

/* Algorithm 2 for every codeword of a batch, recorded once and replayed.
 * grand_graph_create validates and plans `batch` exactly as
 * grand_decode_batch does, copies its job table to the device, and records
 * the launches as a HIP graph.  Each launch in the graph is preceded by a
 * kernel that zeroes its work counter, so every replay starts from the same
 * state.  The host arrays of `batch` are read only during the call.  The
 * graph keeps the batch's device pointers (rx and the outputs) and the codes'
 * device matrices: the caller keeps them alive until grand_graph_destroy and
 * may rewrite rx between launches.  grand_graph_launch enqueues one replay on
 * `stream` (a hipStream_t; NULL = the default stream).  Each replay writes
 * what grand_decode_batch would write for the rx it finds.  Replays of one
 * graph must not overlap: issue them on one stream, or order them.
 * Errors: GRAND_EINVAL (null pointer, empty or invalid batch), GRAND_ENOMEM,
 * GRAND_EDEVICE. */
typedef struct grand_graph grand_graph;
int grand_graph_create(const grand_batch *batch, grand_graph **out);
int grand_graph_launch(grand_graph *graph, void *stream);
void grand_graph_destroy(grand_graph *graph);

/* ------------------------------------------------------------------ */
/* Launch-shape tuning                                                 */
/* ------------------------------------------------------------------ */

typedef struct {
    uint32_t low_bits;     /* b: the b cheapest flips form the sorted low table
                              (0..13, and 2^b <= 8 * block) */
    uint32_t block;        /* threads per workgroup (64..1024, multiple of 64).  A
                              launch with at most one word per compute unit that
                              keeps the default 256 runs 1024-thread workgroups
                              instead */
    uint32_t first_band;   /* patterns aimed at by the first cost band (>= 1) */
    uint32_t band_growth;  /* each later band aims at growth x the patterns
                              checked so far (2..64) */
    uint32_t node_cap;     /* high-subset store entries per workgroup, held in
                              device memory, 16 bytes each (64..2^21) */
    uint32_t grid_per_cu;  /* resident workgroups per compute unit for batches */
} grand_tuning;

/* Tuning used for codes of length n and modulation M (defaults are built
 * in; grand_tuning_set overrides one (n, M) bucket, n = 0 or M = 0 acting as
 * a wildcard). */
int grand_tuning_get(uint32_t n, uint32_t M, grand_tuning *out);
int grand_tuning_set(uint32_t n, uint32_t M, const grand_tuning *t);


/* ------------------------------------------------------------------ */
/* Serving: continuously batched decoding of a request stream          */
/* ------------------------------------------------------------------ */

/* A server admits requests (Algorithm 2 decodes, one codeword each, each as
 * grand_decode decodes it) as they
 * arrive, within a slot count and a device-memory budget, and keeps several
 * HIP streams ("lanes") busy.  Whenever a lane is free, every admitted
 * request not yet on the device (up to max_batch) is written into the lane's
 * coherent pinned buffers and decoded as one launch, heaviest first.  The
 * kernel reads the requests in place and writes each result back with a
 * completion flag, so grand_server_poll returns a request as soon as its own
 * decode has ended, not when its launch has.  Launches on different lanes
 * overlap on the device while new requests keep being admitted.  A request's
 * result is bit-identical to grand_decode of the same input, whatever else
 * is in flight.  Server calls are serialised internally and may come from
 * several host threads.
 *   GRAND_SERVE_LANES      the mode described above (the only one available);
 *   GRAND_SERVE_PERSISTENT reserved: grand_server_create returns GRAND_EINVAL. */
enum { GRAND_SERVE_LANES = 0, GRAND_SERVE_PERSISTENT = 1 };
typedef struct grand_server grand_server;

typedef struct {
    uint32_t max_inflight;     /* admitted, not yet returned requests (1..2^20) */
    uint32_t lanes;            /* streams used concurrently (1..32); HIP maps them
                                  onto GPU_MAX_HW_QUEUES hardware queues */
    uint32_t max_batch;        /* requests per launch (1..65536) */
    uint32_t mode;             /* GRAND_SERVE_LANES or GRAND_SERVE_PERSISTENT */
    uint64_t memory_budget;    /* device bytes reserved for admitted requests;
                                  each reserves grand_request_bytes(n, M) */
    uint32_t wide_lanes;       /* 0, or the number of the lanes (< lanes) that serve only
                                  long words, 2L >= GRAND_WIDE_ITEMS received values
                                  (e.g. N = 512 and 1024 with QPSK, N = 1024 with 16-QAM):
                                  each such request gets one 1024-thread workgroup, a
                                  whole compute unit, and the other lanes take the rest */
    uint32_t pad;              /* must be 0 */
} grand_server_config;

#define GRAND_WIDE_ITEMS 512u

typedef struct {
    uint64_t request_id;
    uint64_t codeword[16];     /* ceil(n/64) words used */
    uint64_t queries;
    uint64_t checks;           /* syndrome checks performed (>= queries unless abandoned) */
    int32_t status;            /* GRAND_OK or a per-request error (GRAND_ECAPACITY) */
    uint8_t abandoned;
    uint8_t pad[3];
    double arrival_s;          /* trace replays: scheduled arrival; otherwise = submit_s */
    double submit_s;           /* host steady-clock seconds when admitted */
    double complete_s;         /* host steady-clock seconds when completion was observed */
} grand_result;

/* Device bytes one request of length n and modulation M reserves while
 * admitted (its received values, outputs and one high-subset store). */
uint64_t grand_request_bytes(uint32_t n, uint32_t M);

int grand_server_create(const grand_server_config *cfg, grand_server **out);
/* Waits for work on the device, then releases everything. */
void grand_server_destroy(grand_server *server);

/* Admit one request: one Algorithm 2 decode (Section III) of one codeword,
 * with the same result as grand_decode of the same input.  rx (2L floats,
 * host) is copied.  Returns GRAND_EBUSY,
 * leaving no state, when the slot count or the memory budget would be
 * exceeded; GRAND_EINVAL for bad arguments (as grand_decode). */
int grand_server_submit(grand_server *server, const grand_code *code, const float *rx,
                        uint32_t M, float noise_var, uint64_t query_cap,
                        uint64_t *request_id);

/* Withdraw an admitted request that has not been launched yet
 * (GRAND_ENOTFOUND otherwise); its slot and memory are released. */
int grand_server_cancel(grand_server *server, uint64_t request_id);

/* Launch admitted requests on free lanes and collect finished ones, without
 * blocking: up to max_out results are written to out (host) and their count
 * to *n_out. */
int grand_server_poll(grand_server *server, grand_result *out, uint32_t max_out,
                      uint32_t *n_out);

/* Requests admitted but not launched, on the device, and bytes reserved. */
int grand_server_stats(grand_server *server, uint64_t *pending, uint64_t *running,
                       uint64_t *memory_in_use);

/* One request of a recorded arrival stream. */
typedef struct {
    uint32_t code_index;       /* into codes[] */
    uint32_t M;
    uint64_t query_cap;
    uint64_t rx_offset;        /* float offset into rx (host) */
    float noise_var;
    float pad;
    double arrival_s;          /* seconds after the start of the replay, ascending */
} grand_trace_req;

/* Replay an arrival stream in real time through the server: each request is
 * submitted at its arrival time (later if admission refuses), and the host
 * polls until every request has completed.  rx (host) holds rx_count floats;
 * request i reads 2L of them from reqs[i].rx_offset on, and a request whose
 * code index, M or values fall outside is rejected with GRAND_EINVAL before
 * the replay starts.  results[i] belongs to reqs[i]; its latency is
 * complete_s - arrival_s.  *wall_s receives the replay's duration. */
int grand_server_run_trace(grand_server *server, const grand_code *const *codes,
                           uint32_t n_codes, const grand_trace_req *reqs, uint32_t count,
                           const float *rx, uint64_t rx_count, grand_result *results,
                           double *wall_s);

/* The same stream decoded one request per grand_decode call (one launch and
 * one synchronisation per request), in arrival order: the baseline the
 * server is compared with.  Same arguments and validation as
 * grand_server_run_trace. */
int grand_plain_run_trace(const grand_code *const *codes, uint32_t n_codes,
                          const grand_trace_req *reqs, uint32_t count, const float *rx,
                          uint64_t rx_count, grand_result *results, double *wall_s);

/* Test hook for callers that exercise failure handling: the next `count`
 * server launches (process-wide) fail as if the launch call had failed.  Each
 * such launch returns its requests as results with status GRAND_EDEVICE, and
 * the grand_server_poll call that attempted it returns GRAND_EDEVICE; the
 * server stays usable.  0 disarms it. */
void grand_debug_fail_launches(uint32_t count);

/* Measured peak of the decode kernel's roofline: the 32-bit bitwise
 * throughput of the current device (the incremental syndrome of Algorithm 2,
 * Step 5, is column XORs, one v_xor_b32 per 32 syndrome bits).  Runs one
 * warm-up and one timed launch of a probe kernel in which every lane issues
 * `steps` x 8 dependent-free v_xor_b32 over 8 workgroups of 256 threads per
 * compute unit, synchronously on the null stream, and stores the achieved
 * lane-operations per second (and the timed launch's seconds, if `seconds`
 * is not null).  `steps` must be a positive multiple of 8, at most 2^20.  Allocates and
 * frees a small device buffer.  Returns 0, GRAND_EINVAL for bad arguments,
 * GRAND_ENOMEM or GRAND_EDEVICE. */
int grand_probe_xor_rate(uint32_t steps, double *lane_ops_per_s, double *seconds);

/* Algorithm 1 (pMult, Section III) and its Theorem on a batch of vectors:
 * syndromes[i] = H x_i^T over GF(2) for the code's H, one full product per
 * vector (the packed rows in LDS; per row the AND with the vector, the XOR
 * fold of the products and their parity, which is the Theorem's addition
 * tree over the row's support).
 *   x          device, count x ceil(n/64) uint64 (bit order as h_rows; bits
 *              past n must be zero);
 *   syndromes  device, count x ceil(rows/64) uint64: bit r of vector i's
 *              syndrome is bit r % 64 of syndromes[i * ceil(rows/64) + r/64];
 *   stream     hipStream_t (NULL = the default stream); asynchronous.
 * Returns GRAND_OK, GRAND_EINVAL (null pointer with count > 0) or
 * GRAND_EDEVICE (also when the code lives on another device). */
int grand_pmult(const grand_code *code, const uint64_t *x, uint32_t count, uint64_t *syndromes,
                void *stream);

/* Baseline for the incremental syndrome: the paper's Step 5 model, one full
 * Algorithm 1 product s = H (yhat + e)^T per test error pattern (bit-packed
 * rows of `code` in LDS; per row an AND with the word, an XOR fold and a
 * parity), with no pattern generation, ordering or early exit.  Runs
 * `words` x `patterns` checks: word w is words_dev[w] (device, ceil(n/64)
 * uint64 each: e.g. the hard decisions of received words), or, when
 * words_dev is NULL, a hash-generated word (bit i of 32-bit word k is bit i
 * of hash(w, k), with hash(a, b) = f(a * 0x9E3779B1 ^ (b + 0x7F4A7C15) *
 * 0x85EBCA77) and f(h) = ((h ^ h >> 15) * 0x2C1B3C6D) ^ (... >> 12), bits
 * past n cleared); pattern p flips bit j of p at position j * n / 16,
 * j < 16.  One warm-up launch, one timed launch, synchronously on the null
 * stream; stores the checks per second and (if not null) the number of zero
 * syndromes found.  patterns <= 65536 and words x patterns <= 2^32.
 * Allocates and frees a small device buffer.  Returns 0, GRAND_EINVAL,
 * GRAND_ENOMEM or GRAND_EDEVICE (also when the code lives on another
 * device). */
int grand_probe_dense_pmult(const grand_code *code, const uint64_t *words_dev, uint32_t words,
                            uint32_t patterns, double *checks_per_s, uint64_t *zero_syndromes);

#ifdef __cplusplus
}
#endif
#endif
