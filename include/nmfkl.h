/*
 * nmfkl.h -- C ABI of the MI355X (gfx950) library for nonnegative matrix factorisation with
 * KL divergence by randomized coordinate descent (Nguyen & Ho, arXiv 1604.04026).
 *
 * Problem (Section 1, eq. 1): V (n x m, nonnegative, sparse) ~ W^T F with W (r x n) and
 * F (r x m) nonnegative, minimising D(V || W^T F) plus the optional L1/L2 terms of eq. 2.
 * Alg. 1 alternates two independent families of subproblems (eq. 3): one per column of V
 * (update F with W fixed) and one per row of V (update W with F fixed); each is solved by
 * Alg. 2, a pass of projected Newton steps over the r coordinates in a random order shared
 * by every column and row of the outer iteration, with first and second derivatives
 * (eq. 6) reduced over the nonzeros of the column/row plus precomputed factor sums.
 *
 * Conventions
 *  - Every function returns an int status: NMFKL_OK (0) or a negative NMFKL_E_* code.  No
 *    C++ exception and no abort crosses the ABI.  nmfkl_last_error() gives a message.
 *  - Arguments are validated before any state changes; on error the handle is unchanged.
 *  - Layout: V is given twice, as CSC (columns = the m instances) and CSR (rows = the n
 *    features), with int64 pointers, int32 indices strictly increasing inside each
 *    column/row, and float32 values (finite, >= 0).  Both factors are stored point-major,
 *    row-major float32: W as n x r (row i = the r-vector of feature i, i.e. the paper's W
 *    transposed) and F as m x r (row j = instance j, the paper's F transposed).
 *  - Pointers marked (device) are device memory owned by the caller; they must stay valid
 *    until the handle is destroyed.  The library allocates only its own scratch and frees
 *    it in the matching destroy call.  Host pointers are read during the call only.
 *  - All device work is enqueued on the caller's HIP stream (passed as void*; NULL means
 *    the default stream).  Only functions that return host values synchronise that stream.
 *    An out-of-core handle also copies V chunks on an internal stream ordered against the
 *    caller's stream with events; a batch captures its graph on a private stream and
 *    replays it on the caller's stream; the fold-in server runs its lanes on streams it owns.
 *    Device-side failures surface at the next synchronising call.
 *  - Precision: values, factors and the derivative sums are float32; the model values at
 *    the nonzeros (W_i . F_j, kept between halves), the factor column sums and the
 *    objective are float64.
 *  - A handle is not thread-safe: calls on one handle must not overlap.
 */
#ifndef NMFKL_H
#define NMFKL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define NMFKL_OK 0
#define NMFKL_E_INVAL (-1)       /* invalid argument or malformed input (nothing changed) */
#define NMFKL_E_NOMEM (-2)       /* device or host allocation failed / admission refused */
#define NMFKL_E_DEVICE (-3)      /* HIP runtime error or device-side failure */
#define NMFKL_E_NONFINITE (-4)   /* a factor holds a NaN/Inf (detected at a synchronising call) */
#define NMFKL_E_BUSY (-5)        /* no free slot (serving) */
#define NMFKL_E_UNSUPPORTED (-6) /* valid request outside the library's limits */

#define NMFKL_R_MAX 128          /* largest supported rank r */

/* Method parameters.  Fill with nmfkl_params_default() and override fields. */
typedef struct nmfkl_params {
    double alpha_W;  /* eq. 2 alpha_1: L2 weight on W (default 0) */
    double alpha_F;  /* eq. 2 alpha_2: L2 weight on F (default 0) */
    double beta_W;   /* eq. 2 beta_1: L1 weight on W (default 0) */
    double beta_F;   /* eq. 2 beta_2: L1 weight on F (default 0) */
    double eps_log;  /* smoothing added to the model inside log and denominators, Alg. 2 output line (1e-10) */
    double eps_g;    /* relative gradient threshold of Alg. 2's while-test (1e-5) */
    double eps_x;    /* step-size break ratio of Alg. 2, Section 3 value 0.1 */
    int32_t t_max;   /* Newton steps per coordinate (16) */
    int32_t j_max;   /* halvings of a decreasing step rejected by the descent guard (8) */
    int32_t literal_break; /* 1: break test on the signed step as printed (ablation), 0: on |step| */
    int32_t guard;   /* 1: descent guard on decreasing steps (default), 0: plain projected Newton */
    uint64_t seed;   /* Philox key of the coordinate orders (0) */
    int32_t foldin_max_passes; /* fold-in: passes at most (200) */
    double foldin_tol;         /* fold-in: stop when the KL decrease <= tol * KL (1e-5) */
    int32_t refresh_model;     /* 0 (default): the model values at the nonzeros (float64) are carried
                                  from one half-sweep to the next and recomputed only for the first
                                  half-sweep or after nmfkl_invalidate_model; 1: recomputed from W and
                                  F at the start of every nmfkl_sweep_F (unless nmfkl_objective just
                                  did).  Identical in exact arithmetic; the carried values move by the
                                  increments the stored float32 factors actually took, so they differ
                                  from fresh products only by float64 rounding */
    int32_t collect_stats;     /* 1: count derivative evaluations / steps / guard events (slower) */
    int32_t collect_timings;   /* 1: bracket every launch group with HIP events (nmfkl_get_timings) */
    int32_t tuning;            /* implementation choices that do not change results; bit 0: batched
                                  (lookahead) derivative sums also for segments of 257..1024 nonzeros;
                                  bit 1 (batches): blocks ordered problem by problem rather than by
                                  segment length across problems; bit 2: only the lane groups of 4 and
                                  8 nonzeros per lane (power-of-two bin capacities), not those of 3,
                                  5 and 6 between them */
    int32_t bin_shift;         /* mapping of segments of <= 1024 nonzeros to lanes (0..3, default 0):
                                  a segment of L nonzeros runs on the smallest lane group that holds
                                  L << bin_shift nonzeros (8 x 3 or 4, 16 x 3 or 4, 32 x 3 or 4, 64 x 3,
                                  4, 5, 6 or 8, 256 x 3 or 4; segments of 1025..2048 always take
                                  256 x 8).  Changes
                                  the summation order of eq. 6's sums, hence results in the last
                                  bits; results are identical for identical bin_shift */
    int32_t tile_bf16;         /* 0 (default): the fixed factor of a half-sweep is read in float32;
                                  1: its permuted copy is stored in bfloat16 (round to nearest
                                  even) and every half-sweep solves its subproblems for the rounded
                                  factor: each column/row computes its model values from the rounded
                                  tiles first (Alg. 2's first step), and the derivative sums, column
                                  sums and model increments use the rounded values (arithmetic stays
                                  float32 / float64).  Halves the bytes of each tile gather; results
                                  differ from float32 tiles by the rounding (about 2^-9 relative per
                                  factor entry) */
    int32_t out_of_core;       /* 0 (default): V's CSC/CSR arrays are device memory.  1: they are host
                                  memory (pinned, e.g. hipHostMalloc, for overlapped copies) and every
                                  half-sweep streams them through two device staging buffers in
                                  chunks of whole columns/rows, copying the next chunk while the
                                  current one is swept; no model values are kept (each column/row
                                  computes them from the tiles, Alg. 2's first step).  W and F stay
                                  device memory.  Not available for batches */
    int64_t ooc_chunk_nnz;     /* out_of_core: nonzeros per chunk (0: 1 << 25); a chunk grows to hold
                                  a longer column/row */
} nmfkl_params;

typedef struct nmfkl_problem {
    int32_t n, m, r;           /* V is n x m, rank r (1 <= r <= NMFKL_R_MAX) */
    int64_t nnz;               /* number of stored entries (same in both copies) */
    /* the six V arrays are host memory instead when params.out_of_core = 1 */
    const int64_t* csc_ptr;    /* (device) m+1 */
    const int32_t* csc_idx;    /* (device) nnz row ids */
    const float* csc_val;      /* (device) nnz */
    const int64_t* csr_ptr;    /* (device) n+1 */
    const int32_t* csr_idx;    /* (device) nnz column ids */
    const float* csr_val;      /* (device) nnz */
    float* W;                  /* (device) n x r, in/out */
    float* F;                  /* (device) m x r, in/out */
} nmfkl_problem;

typedef struct nmfkl_stats {
    int64_t coords;    /* coordinate visits */
    int64_t evals;     /* derivative evaluations (eq. 6 reductions) */
    int64_t steps;     /* accepted Newton steps */
    int64_t halvings;  /* descent-guard halvings */
    int64_t rejects;   /* steps abandoned by the guard */
    int64_t tmax_hits; /* coordinates stopped by t_max */
    int64_t zeros_W;   /* exact zeros in W at the call (n x r entries), the sparsity of the
                          paper's Table 2; -1 from nmfkl_model_get_stats */
    int64_t zeros_F;   /* exact zeros in F at the call (m x r entries); -1 from nmfkl_model_get_stats */
} nmfkl_stats;

/* Launch groups timed when params.collect_timings is set. */
#define NMFKL_T_SUMS_F 0   /* F-half: order, permuted copy of W and its float64 column sums */
#define NMFKL_T_FUSED_F 1  /* F-half: the binned launch over columns of <= 2048 nonzeros */
#define NMFKL_T_LONG_F 2   /* F-half: the cooperative launch over longer columns */
#define NMFKL_T_SUMS_W 3   /* W-half: order, permuted copy of F and its column sums */
#define NMFKL_T_FUSED_W 4  /* W-half: the binned launch over rows of <= 2048 nonzeros */
#define NMFKL_T_LONG_W 5   /* W-half: the cooperative launch over longer rows */
#define NMFKL_T_MODEL 6    /* model values at the nonzeros from W and F (+ eq. 1 terms) */
#define NMFKL_T_TERMS 7    /* eq. 1 terms from the carried model values (nmfkl_objective_carried) */
#define NMFKL_NUM_TIMED 8

typedef struct nmfkl_kernel_timing {
    double ms_total;      /* summed HIP-event time of the timed launches */
    int64_t launches;     /* number of timed launch groups */
    double gather_bytes;  /* algorithmic bytes of one launch group under the gather model:
                             per nonzero 4 (index) + 4 (value) + 4r (the fixed factor's row),
                             per segment 8 (pointer) + 8r (x read and written); for the model
                             pass per nonzero 4 + 4 + 4r + 8 (model written) + per column 4r;
                             for the carried terms per nonzero 8 (model) + 4 (value) */
    double updates;       /* coordinate updates of one launch group: nonzeros x r */
} nmfkl_kernel_timing;

typedef struct nmfkl_timings {
    nmfkl_kernel_timing k[NMFKL_NUM_TIMED];
} nmfkl_timings;

typedef struct nmfkl_handle nmfkl_handle;
typedef struct nmfkl_model nmfkl_model;

/* Defaults listed field by field above. */
int nmfkl_params_default(nmfkl_params* p);

/* The coordinate order of outer iteration t (Alg. 1: "a randomized ordered set of
 * {1..r}", here 0-based): a Fisher-Yates shuffle of 0..r-1 driven by Philox-4x64-10 with
 * key (seed, 0) and counter (b, t, stream, 0), b = 0, 1, ...; word w picks
 * j = floor(w * (i + 1) / 2^64) for i = r-1 down to 1.  Stream 0 is the sweeps, stream 1
 * the fold-in passes.  ids: host array of r int32.  Host only, no device work. */
int nmfkl_permutation(uint64_t seed, uint64_t t, uint64_t stream, int32_t r, int32_t* ids);

/* Create a handle over a problem.  Validates the shapes (host) and then, on the device,
 * the CSC/CSR structure (pointer monotonicity and ends, index ranges and strict order,
 * values finite and >= 0, CSR equal to the transpose of CSC) and W, F finite and >= 0;
 * synchronises the stream once.  Builds the nnz bins, the CSC<->CSR position maps and the
 * scratch buffers.  With params.out_of_core the structure and values are validated on the
 * host (the transpose by per-row counts and an order-independent checksum of the entries),
 * the bins are built per chunk and no maps or model values are allocated.  Errors:
 * NMFKL_E_INVAL (shape/structure/value), NMFKL_E_NOMEM, NMFKL_E_DEVICE, NMFKL_E_UNSUPPORTED
 * (a column or row of more nonzeros than the cooperative launch holds at once: 10,240 per
 * compute unit, about 2.6M on a 256-unit device).  On error *out is NULL. */
int nmfkl_create(const nmfkl_problem* prob, const nmfkl_params* p, void* hip_stream,
                 nmfkl_handle** out);

/* Alg. 1, first half of outer iteration t: sumW = W 1 (float64), then Alg. 2 on every
 * column j of V with A = W, x = F_j, (alpha_F, beta_F) and the order of iteration t.
 * Updates F in place.  Asynchronous.  t >= 0. */
int nmfkl_sweep_F(nmfkl_handle* h, int32_t t);

/* Alg. 1, second half of outer iteration t: sumF = F 1 (float64), then Alg. 2 on every
 * row i of V with A = F, x = W_i, (alpha_W, beta_W) and the same order.  Updates W in
 * place.  Asynchronous.  t >= 0. */
int nmfkl_sweep_W(nmfkl_handle* h, int32_t t);

/* eq. 1, D(V || W^T F) in float64 for the current W, F: the per-nonzero terms
 * v log(v/M) - v with M = W_i . F_j, plus sum(W^T F) = sumW . sumF.  Synchronises.
 * +inf if some nonzero has M = 0; NMFKL_E_NONFINITE if a factor holds NaN/Inf. */
int nmfkl_objective(nmfkl_handle* h, double* D_out);

/* eq. 1 for the current W, F using the model values the handle carries between halves
 * (no pass over the factors): sum over the nonzeros of v log(v/M) - v, plus sumW . sumF.
 * Differs from nmfkl_objective by the float32 rounding of factor updates accumulated in the
 * carried values (about 1e-7 relative after tens of sweeps).  Synchronises.  Falls back to
 * nmfkl_objective when no model is carried yet. */
int nmfkl_objective_carried(nmfkl_handle* h, double* D_out);

/* nmfkl_objective_carried in two steps, so that a loop can keep the device busy: enqueue
 * computes eq. 1 on the handle's stream and copies the result into the handle's pinned
 * host memory without synchronising; read synchronises the stream and returns the value of
 * the last enqueue (with the same checks and error codes as nmfkl_objective_carried).  A
 * later enqueue replaces the pending value.  read without an enqueue since the last read
 * returns NMFKL_E_INVAL. */
int nmfkl_objective_enqueue(nmfkl_handle* h);
int nmfkl_objective_read(nmfkl_handle* h, double* D_out);

/* Tell the handle that the caller changed W or F outside the library: the model values
 * the handle carries between halves are recomputed before the next half-sweep. */
int nmfkl_invalidate_model(nmfkl_handle* h);

/* Counters accumulated since creation (all zero unless params.collect_stats), and the exact
 * zeros of W and F at the call (always).  Synchronises. */
int nmfkl_get_stats(nmfkl_handle* h, nmfkl_stats* out);

/* Accumulated event times since creation or the last reset (all zero unless
 * params.collect_timings).  Synchronises. */
int nmfkl_get_timings(nmfkl_handle* h, nmfkl_timings* out);

/* Zero the accumulated timings.  Synchronises. */
int nmfkl_reset_timings(nmfkl_handle* h);

/* Free the library's scratch.  Synchronises the stream first. */
int nmfkl_destroy(nmfkl_handle* h);

/* Message of the last failed call on h (h may be NULL: the last failure of a create). */
const char* nmfkl_last_error(const nmfkl_handle* h);

/* ---------------------------------------------------------------- batched problems
 * Many independent factorisations (Alg. 1 on each; problems share nothing, as the columns
 * and rows of one problem do in eq. 3) advanced together: every launch of a half-sweep
 * covers all problems (the permuted copies and factor sums of every problem in one launch,
 * the segments of every problem binned into one set of sweep launches), and the launches of
 * a run of sweeps are captured once in a HIP graph and replayed.  A problem's results are
 * identical to those of a handle over the same problem with the same parameters (same
 * bin_shift) running the same sweeps. */
typedef struct nmfkl_batch nmfkl_batch;

typedef struct nmfkl_batch_info {
    int32_t nprob;
    int32_t bin_shift;          /* mapping in use (nmfkl_params.bin_shift) */
    int32_t tuning;             /* nmfkl_params.tuning in use */
    int32_t graph_cooperative;  /* 1: graphs hold cooperative launches; 0: ordinary launches of
                                   grids within the co-resident capacity; -1: no graph yet */
    int32_t fused_blocks[2];    /* blocks of the binned launch: F-half, W-half */
    int32_t long_parts[2];      /* parts (blocks' worth of work) of the cooperative launch */
    int32_t long_rounds[2];     /* cooperative launches per half (0 or 1) */
    int64_t nnz_total;
} nmfkl_batch_info;

/* Create a batch over nprob problems (host array of nmfkl_problem whose pointers are device
 * memory owned by the caller, valid until nmfkl_batch_destroy).  Each problem is validated
 * as by nmfkl_create (errors name the problem).  One params for all problems.  Synchronises.
 * Errors: NMFKL_E_INVAL, NMFKL_E_NOMEM, NMFKL_E_DEVICE, NMFKL_E_UNSUPPORTED.  On error *out
 * is NULL and nmfkl_batch_last_error(NULL) gives the message. */
int nmfkl_batch_create(int32_t nprob, const nmfkl_problem* probs, const nmfkl_params* p, void* hip_stream,
                       nmfkl_batch** out);

/* Outer iterations t0, ..., t0 + nsweeps - 1 of Alg. 1 (F-half then W-half) on every problem,
 * as one graph launch on the batch's stream (the graph for this nsweeps is captured on first
 * use and reused).  Asynchronous.  t0 >= 0, 1 <= nsweeps <= 100000. */
int nmfkl_batch_run(nmfkl_batch* b, int32_t t0, int32_t nsweeps);

/* eq. 1 of every problem (nprob doubles, host), from the carried model values as
 * nmfkl_objective_carried.  Synchronises; reports a failed cross-block wait as
 * NMFKL_E_DEVICE. */
int nmfkl_batch_objective(nmfkl_batch* b, double* D_out);

/* Autotuner: times one outer iteration (iteration t) under each candidate mapping
 * (bin_shift 0..2, tuning bits 0, 1 and 2 off/on) on the batch, restoring W, F and the model values after
 * every trial, and keeps the fastest.  The factors are unchanged on return.  chosen (host,
 * may be NULL) receives the parameters now in use, with which nmfkl_create reproduces the
 * batch's results.  Synchronises. */
int nmfkl_batch_tune(nmfkl_batch* b, int32_t t, nmfkl_params* chosen);

int nmfkl_batch_get_info(nmfkl_batch* b, nmfkl_batch_info* out);
const char* nmfkl_batch_last_error(const nmfkl_batch* b);

/* Synchronises the stream, then frees the batch's scratch (not the problems' memory). */
int nmfkl_batch_destroy(nmfkl_batch* b);

/* ---------------------------------------------------------------- fold-in (W fixed)
 * Fold-in solves Alg. 1's F-half for new columns of V with a trained W held fixed (the
 * columns are independent subproblems, eq. 3): a document's x starts at the mass-matched
 * constant sum(v) / sum(sumW) in every coordinate; pass p runs Alg. 2 once with the order
 * of Philox stream 1, counter p (nmfkl_permutation(seed, p, 1, r)); the document stops after
 * the first pass whose decrease of KL(v || W^T x) = sum_l (v_l log(v_l / [W^T x]_l) - v_l)
 * + sumW . x is <= foldin_tol * KL, or after foldin_max_passes passes.  Uses alpha_F,
 * beta_F and the inner-loop parameters of nmfkl_params.  A document's result does not
 * depend on the other documents processed with it.  Documents of up to 5120 distinct words
 * are supported (NMFKL_E_UNSUPPORTED beyond). */
typedef struct nmfkl_result {
    uint64_t req_id;
    int32_t passes;     /* passes run (0 unless status is NMFKL_OK) */
    int32_t status;     /* NMFKL_OK: folded in; NMFKL_RESULT_EXPIRED: not launched within its
                           time limit; NMFKL_RESULT_CANCELLED: withdrawn by nmfkl_server_cancel
                           (kl and f are 0 then) */
    double kl;          /* final KL of the document */
    double t_submit;    /* steady-clock seconds at submit (nmfkl_server_now's clock) */
    double t_done;      /* steady-clock seconds when the host observed completion */
} nmfkl_result;

#define NMFKL_RESULT_EXPIRED 1
#define NMFKL_RESULT_CANCELLED 2

typedef struct nmfkl_server nmfkl_server;

/* A resident model: W (device, n x r point-major, caller-owned, unchanged while the model
 * lives).  Validates W on the device (finite, >= 0; synchronises), computes its float64
 * column and row sums and the pass orders. */
int nmfkl_model_create(const float* W, int32_t n, int32_t r, const nmfkl_params* p, void* hip_stream,
                       nmfkl_model** out);

/* Fold in ndocs documents given in CSC form (device: doc_ptr[ndocs+1] int64, word_idx int32
 * strictly increasing per document, counts float32 finite >= 0).  Outputs (device):
 * F_out ndocs x r, passes_out, kl_out.  Validates on the device and synchronises the
 * model's stream before returning. */
int nmfkl_foldin(nmfkl_model* m, int32_t ndocs, const int64_t* doc_ptr, const int32_t* word_idx,
                 const float* counts, float* F_out, int32_t* passes_out, double* kl_out);

/* nmfkl_foldin for callers that cannot allocate memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): the same arguments, kernels and results
 * as nmfkl_foldin, but the call allocates nothing on the device or the host heap.  Its
 * scratch (the validation flags and the documents grouped by kernel variant, 64 KiB) is one
 * static device array per GPU, held until the process ends; the document pointers are
 * checked and grouped on the device.  Limit: at most 16384 documents per call
 * (NMFKL_E_UNSUPPORTED beyond); other errors as nmfkl_foldin (NMFKL_E_INVAL for malformed
 * documents, NMFKL_E_UNSUPPORTED for a document above 5120 distinct words).  The model's
 * stream must belong to the current device.  Synchronises the model's stream (twice: to
 * read the checks, and before returning).  Every call on one GPU shares that GPU's
 * scratch: calls that overlap on one GPU (from several host threads) race and must be
 * serialised by the caller. */
int nmfkl_foldin_noalloc(nmfkl_model* m, int32_t ndocs, const int64_t* doc_ptr, const int32_t* word_idx,
                         const float* counts, float* F_out, int32_t* passes_out, double* kl_out);

/* Counters of the fold-in kernels (params.collect_stats).  Synchronises. */
int nmfkl_model_get_stats(nmfkl_model* m, nmfkl_stats* out);
const char* nmfkl_model_last_error(const nmfkl_model* m);
int nmfkl_model_destroy(nmfkl_model* m);

/* Continuously batched fold-in server over a model.  `lanes` streams each run one batch of
 * up to lane_docs documents at a time; whenever a lane is free, nmfkl_server_poll launches
 * the oldest waiting documents on it, so documents that arrive while others are on the GPU
 * start without waiting for them.  Each document is returned as soon as it has converged:
 * the kernels write its result into host-coherent memory and then mark it done, so a
 * document does not wait for the slowest one of its batch.  Admission: the words of all
 * submitted and unreturned documents stay within mem_budget_bytes (8 bytes per word), and
 * at most max_queued documents wait for a lane (0: no limit). */
int nmfkl_server_create(nmfkl_model* m, int64_t mem_budget_bytes, int32_t lanes, int32_t lane_docs,
                        int32_t max_queued, nmfkl_server** out);

/* Submit one document (host arrays, copied before returning).  timeout_s > 0: if it has not
 * been launched timeout_s seconds after submission it is not launched and the first
 * nmfkl_server_poll after that returns it with status NMFKL_RESULT_EXPIRED, also while every
 * lane is busy (<= 0: no limit).  NMFKL_E_BUSY: max_queued documents are waiting (retry
 * later); NMFKL_E_NOMEM: the memory budget is full now (retry later); NMFKL_E_INVAL:
 * malformed; NMFKL_E_UNSUPPORTED: too long. */
int nmfkl_server_submit(nmfkl_server* s, uint64_t req_id, int32_t L, const int32_t* word_idx,
                        const float* counts, double timeout_s);

/* Withdraw a document that is still waiting for a lane: it is returned by a later poll with
 * status NMFKL_RESULT_CANCELLED.  NMFKL_E_INVAL if no waiting document has this id (already
 * launched, returned or unknown; a launched document runs to the end). */
int nmfkl_server_cancel(nmfkl_server* s, uint64_t req_id);

/* Non-blocking: collect finished documents, launch waiting documents on free lanes, and
 * return up to max_results finished documents (out[k] and f_out[k*r .. k*r+r)). */
int nmfkl_server_poll(nmfkl_server* s, int32_t max_results, nmfkl_result* out, float* f_out,
                      int32_t* n_out);

/* The server's clock (steady-clock seconds, as in t_submit and t_done). */
int nmfkl_server_now(double* t_out);

/* Documents submitted and not yet returned by poll, and words held against the budget. */
int nmfkl_server_pending(nmfkl_server* s, int64_t* queued, int64_t* in_flight_words);
const char* nmfkl_server_last_error(const nmfkl_server* s);

/* Waits for the lanes, then frees the server (not the model). */
int nmfkl_server_destroy(nmfkl_server* s);

#ifdef __cplusplus
}
#endif

#endif /* NMFKL_H */
