/*
 * gabp_svm.h -- C ABI of the MI355X (gfx950) GaBP SVM solver.
 *
 * Method: Bickson, Yom-Tov, Dolev, "A Gaussian Belief Propagation Solver for
 * Large Scale Support Vector Machines" (arXiv 0810.1648).
 *
 * Problem statement (section "Classification Using Support Vector
 * Machines"): a training set {(x_i, y_i)}, i = 1..N, x_i in R^m,
 * y_i in {-1, +1}, a kernel K and a cost C go in; the Lagrange multipliers
 * h = alpha and the decision function sign(sum_i alpha_i y_i K(x_i, x) + b)
 * come out.  Following section "Proposed Solution of SVM Solver Based on
 * GaBP", the solver drops the box and equality constraints and returns the
 * mean of p(h) ~ exp(-1/2 h'Ah + h'1), i.e. alpha = A^-1 1 with
 * A = Y K' Y + W: K' = K + lambda^2 (bias augmentation), W the diagonal
 * weighting of subsection "GaBP Algorithm Convergence".  alpha is computed
 * by synchronous sweeps of Algorithm 2 (section "Algorithm Optimization"):
 * every node broadcasts its aggregate precision and mean, and every
 * message is that aggregate minus the recipient's own term.
 *
 * Conventions for every call:
 *   - No exception crosses the ABI; every call returns a gabp_status.
 *   - The caller owns every buffer it passes.  Host inputs are copied before
 *     the call returns; device inputs (mem = GABP_MEM_DEVICE) are read on the
 *     given HIP stream and must stay valid until the call returns.
 *   - A handle owns all device memory it allocates and frees it in
 *     gabp_svm_destroy or when the next solve needs a different plan.
 *   - One thread at a time per handle; distinct handles are independent.
 *   - There is no CPU fallback: without a usable gfx950 device every
 *     compute call fails with GABP_E_DEVICE.
 */
#ifndef GABP_SVM_H
#define GABP_SVM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GABP_ABI_VERSION 9

/* Opaque solver handle; owns every device buffer it allocates. */
typedef struct gabp_svm gabp_svm;

typedef enum gabp_status {
    GABP_OK = 0,
    GABP_E_INVALID = 1,        /* bad argument; nothing was computed */
    GABP_E_NOMEM = 2,          /* plan does not fit the device-memory budget */
    GABP_E_NOT_CONVERGED = 3,  /* max_sweeps reached; alpha = last iterate */
    GABP_E_DIVERGED = 4,       /* a cavity precision P~_i - P_ji <= 0, or a
                                  non-finite value: alpha is undefined */
    GABP_E_DEVICE = 5,         /* HIP runtime error or no usable device */
    GABP_E_STATE = 6,          /* call not valid in the handle's state */
    GABP_E_BUFSIZE = 7         /* destination buffer too small */
} gabp_status;

/* Kernel K(x, z).  RBF: exp(-gamma ||x - z||^2), the kernel of every
 * experiment in section "Experimental Results".  PRECOMPUTED: the caller
 * passes the N x N matrix K' itself (gabp_svm_solve_kernel).  RBF_SPARSE:
 * the RBF kernel sparsified by a threshold, the route to millions of points
 * that the closing discussion names: only the pairs with
 * exp(-gamma ||x_i - x_j||^2) >= sparse_tau are kept (K'_ij = K_ij +
 * lambda^2 on them, 0 elsewhere); GaBP runs on that graph with the pair
 * records stored per edge (gabp_svm_solve; FP32 or MIXED, SYNC schedule). */
typedef enum gabp_kernel {
    GABP_KERNEL_RBF = 0, GABP_KERNEL_PRECOMPUTED = 2, GABP_KERNEL_RBF_SPARSE = 3
} gabp_kernel;

/* Diagonal weighting (subsection "GaBP Algorithm Convergence"), with
 * r_i = sum_{j != i} |K'_ij|:
 *   NONE:             A_ii = K'_ii
 *   SOFTMARGIN:       A_ii = K'_ii + 1/C            (2-norm soft margin)
 *   DOMINANT_ROW:     A_ii = max(K'_ii + 1/C, (1 + delta) r_i)   [default]
 *   DOMINANT_UNIFORM: A_ii = K'_ii + max_k (max(K'_kk + 1/C, (1+delta) r_k) - K'_kk) */
typedef enum gabp_diag {
    GABP_DIAG_NONE = 0,
    GABP_DIAG_SOFTMARGIN = 1,
    GABP_DIAG_DOMINANT_ROW = 2,
    GABP_DIAG_DOMINANT_UNIFORM = 3
} gabp_diag;

/* Box constraint 0 <= alpha <= C (eq. cons1).  The paper drops it; NONE
 * reports alpha as solved, CLIP_OUTPUT reports clip(alpha, 0, C) without
 * touching the sweep.  PROJECT (not the paper's method) restores it inside
 * the sweep: after every aggregate step the belief mean of each node is
 * clipped to [0, C] and the node broadcasts P~ times the clipped mean; the
 * fixed point is the optimum of the box-constrained dual QP (verified
 * against the QP).  PROJECT is not available in the server. */
typedef enum gabp_box {
    GABP_BOX_NONE = 0, GABP_BOX_CLIP_OUTPUT = 1, GABP_BOX_PROJECT = 2
} gabp_box;

/* Arithmetic of the sweep.
 *   FP64:  FP64 kernel entries, messages, aggregates.
 *   FP32:  FP32 kernel entries (FP32 MFMA Gram), messages and aggregates.
 *   MIXED: BF16 MFMA Gram with FP32 accumulation, FP32 stored messages,
 *          FP64 aggregates and FP64 cavity denominators P~_i - P_ji. */
typedef enum gabp_prec { GABP_PREC_FP64 = 0, GABP_PREC_FP32 = 1, GABP_PREC_MIXED = 2 } gabp_prec;

/* Kernel-matrix storage: MATERIALISE keeps K' (upper triangle) in device
 * memory; RECOMPUTE rebuilds each tile of K' from the features in every
 * sweep.  AUTO materialises when it fits the budget. */
typedef enum gabp_kstore {
    GABP_KSTORE_AUTO = 0, GABP_KSTORE_MATERIALISE = 1, GABP_KSTORE_RECOMPUTE = 2
} gabp_kstore;

/* Edge (message) state: STORED keeps both directions of every pair's
 * messages in device memory; STATELESS rebuilds them each sweep from a
 * short history of aggregates (exact while the sweep count <= depth, a
 * truncation with bound (max|A_ij| / min Q)^depth after). */
typedef enum gabp_edge { GABP_EDGE_AUTO = 0, GABP_EDGE_STORED = 1, GABP_EDGE_STATELESS = 2 } gabp_edge;

/* Gram of the MIXED path, always BF16 MFMA with FP32 accumulation:
 *   BF16:   one product of x rounded to BF16 (features perturbed by <= 2^-9
 *           relative);
 *   BF16X3: x = hi + lo, products hi*hi + hi*lo + lo*hi (about 2^-17);
 *   BF16X6: x = hi + lo + lo2, the six products whose order is >= 2^-18
 *           (about 2^-26, FP32-Gram accuracy).  AUTO = BF16X6. */
typedef enum gabp_gram {
    GABP_GRAM_AUTO = 0, GABP_GRAM_BF16 = 1, GABP_GRAM_BF16X3 = 2, GABP_GRAM_BF16X6 = 3
} gabp_gram;

/* Message schedule (Algorithm 2 leaves it open; section "Convergence in
 * Asynchronous Settings" reports faster convergence without global rounds):
 *   SYNC:    every message of sweep t from the values of sweep t-1;
 *   GROUPED: the points are split into sched_groups ordered groups of whole
 *            256-point blocks; a sweep visits the groups in order and each
 *            visit recomputes every message into the group from the current
 *            aggregates, then refreshes the group's aggregates (block
 *            Gauss-Seidel).  Same fixed point, far fewer sweeps. */
typedef enum gabp_sched { GABP_SCHED_SYNC = 0, GABP_SCHED_GROUPED = 1 } gabp_sched;

/* Where the caller's buffers live. */
typedef enum gabp_mem { GABP_MEM_HOST = 0, GABP_MEM_DEVICE = 1 } gabp_mem;

/* Stop reason of the last solve (GABP_Q_REASON). */
typedef enum gabp_reason {
    GABP_REASON_NONE = 0, GABP_REASON_CONVERGED = 1, GABP_REASON_MAX_SWEEPS = 2,
    GABP_REASON_DIVERGED = 3, GABP_REASON_STAGNATED = 4
} gabp_reason;

typedef struct gabp_svm_params {
    uint32_t struct_size;      /* sizeof(gabp_svm_params), for ABI checks */
    int32_t kernel;            /* gabp_kernel */
    double gamma;              /* RBF width, > 0 */
    double C;                  /* > 0: 1/C enters the diagonal weighting */
    double lambda_aug;         /* bias augmentation lambda; < 0 means 1/N.
                                  lambda^2 is added to every RBF entry */
    int32_t diag_mode;         /* gabp_diag, default DOMINANT_ROW */
    double diag_delta;         /* dominance margin, default 0.1 */
    int32_t box_mode;          /* gabp_box, default NONE */
    double sv_tau;             /* support vector iff alpha_i > sv_tau (0) */
    double tol_abs, tol_rel;   /* stop when ||alpha^t - alpha^(t-1)||_inf <=
                                  tol_abs + tol_rel ||alpha^t||_inf */
    int32_t max_sweeps;        /* >= 1 */
    int32_t check_every;       /* host polls the device status every k sweeps */
    int32_t stagnation_window; /* stop when the change has not decreased for
                                  this many sweeps and is <= stagnation_rel
                                  ||alpha||_inf (precision floor); 0 = off */
    double stagnation_rel;
    int32_t precision;         /* gabp_prec, default MIXED */
    int32_t kstore;            /* gabp_kstore */
    int32_t edge_state;        /* gabp_edge */
    int32_t gram;              /* gabp_gram (MIXED only) */
    int32_t stateless_depth;   /* STATELESS unroll depth 1..8; 0 = from the
                                  contraction bound rho.  AUTO takes the
                                  stateless form only at a depth <= 8 whose
                                  truncation (about (1.25 rho)^depth) stays
                                  below the message precision, and returns
                                  GABP_E_NOMEM when neither that nor the
                                  stored records fit.  STATELESS with depth 0
                                  takes min(that depth, 8) and returns
                                  GABP_E_INVALID without a bound
                                  (1.25 rho >= 1).  A depth below the bound's
                                  runs the truncated recursion and is flagged
                                  (gabp_plan.stateless_bounded = 0) */
    int32_t device;            /* HIP device ordinal */
    uint64_t hbm_budget_bytes; /* 0 = 90% of the device's free memory */
    int32_t time_sweeps;       /* 1: bracket every sweep kernel with HIP
                                  events (GABP_Q_TIMINGS.sweep_kernel_ms) */
    int32_t schedule;          /* gabp_sched, default SYNC */
    int32_t sched_groups;      /* GROUPED: number of node groups (whole
                                  256-point blocks, at most the block
                                  count); 0 = 16 */
    int32_t sparse_edges_hint; /* RBF_SPARSE: expected number of kept pairs,
                                  >= 0; it sizes the edge list that the
                                  build's single pass over the tiles fills
                                  (0 = estimated from every 32nd tile).  A
                                  hint below the true number costs a second
                                  pass; the graph is the same either way */
    double sparse_tau;         /* RBF_SPARSE: kernel threshold in (0, 1] */
    int32_t tile_chunk;        /* synchronous stateless sweeps over the K'
                                  plane with FP32 partial sums (FP32, or MIXED
                                  with series reciprocals; one level, two with
                                  series reciprocals, three with series form
                                  3): 0 = 2 x 2 chunks of tiles per workgroup
                                  when there are at least 4,096 chunks, else
                                  one tile; 1 = one tile per workgroup; 2 =
                                  2 x 2 chunks at any size.  Other plans take
                                  one tile per workgroup (gabp_plan.tile_chunk
                                  reports the choice) */
} gabp_svm_params;

/* Per-phase device times of the last solve, in milliseconds (HIP events on
 * the solve's stream). */
typedef struct gabp_timings {
    double stage_ms;           /* feature staging (and H2D copies) */
    double kbuild_ms;          /* K' build (materialised) or none */
    double diag_ms;            /* row sums + diagonal weighting + init */
    double sweep_loop_ms;      /* all sweeps + finalize + status polls */
    double sweep_kernel_ms;    /* sum over sweep-kernel launches (time_sweeps) */
    int64_t sweep_launches;    /* sweep-kernel launches that did work */
    double d2h_ms;             /* alpha download (host output) */
    double total_ms;           /* whole solve call, host wall clock */
    double predict_kernel_ms;  /* last gabp_svm_predict: time of the decision-
                                  function kernel launches (time_sweeps) */
    int64_t predict_queries;   /* queries of that call */
} gabp_timings;

/* The memory plan chosen for the last solve. */
typedef struct gabp_plan {
    int32_t precision, kstore, edge_state, gram;
    int32_t tile;              /* tile edge T (pairs are processed in T x T tiles) */
    int32_t stateless_depth;
    int64_t n_blocks;          /* ceil(N / T) */
    int64_t n_tiles;           /* n_blocks (n_blocks + 1) / 2 */
    uint64_t device_bytes;     /* device memory held by the handle */
    uint64_t alg_bytes_per_sweep; /* algorithmic HBM bytes of one sweep:
                                     N(N-1)/2 pairs x bytes per pair */
    double alg_bytes_per_pair;
    double stateless_rho;      /* a-priori bound on |A_ij| / Q_ij over every
                                  sweep (computed before sweep 1); the truncation
                                  of the message recursion is bounded by about
                                  rho^stateless_depth */
    int32_t series_reciprocal; /* stateless reciprocals of the cavity
                                  precisions: 0 exact; 1 / 2 by the series
                                  around 1/P~ with a one- / two-term top
                                  level (one term at the lower levels);
                                  3 one-term top level, 1/P~ alone at the
                                  lower levels (depth >= 3, rho^3 below
                                  the message precision) */
    int32_t sched_groups;      /* groups of the GROUPED schedule; 0 = SYNC */
    int64_t n_edges;           /* RBF_SPARSE: kept pairs (graph edges); else 0 */
    int32_t stateless_bounded; /* 1: stored records, or a stateless depth at
                                  least the one the contraction bound asks
                                  for (the truncation stays below the message
                                  precision); 0: an explicit stateless_depth
                                  below it (a truncated recursion) */
    int32_t tile_chunk;        /* synchronous sweep: 2 = one workgroup per
                                  2 x 2 chunk of tiles, whose row and column
                                  sums are added over the chunk before they
                                  are stored (FP32 partial sums; one level,
                                  two with series reciprocals, three with
                                  series form 3); 1 = one tile per workgroup;
                                  0 = the sparsified kernel (no tiles) */
    int32_t recompute_aug;     /* K' recomputed per band: 1 = each entry from
                                  the Gram of augmented rows (x, |x|^2, 1) and
                                  (c x, -c/2, -c/2 |x|^2), which is the
                                  exponent itself (BF16 splits with m + 2 <=
                                  m_pad); 0 = from the plain Gram and the norms,
                                  or K' materialised */
    int32_t reserved;
} gabp_plan;

/* Query selectors for gabp_svm_query: dst type and size in brackets. */
enum {
    GABP_Q_N = 0,          /* [int64_t] N of the last solve */
    GABP_Q_ALPHA = 1,      /* [double N] alpha (box handling applied) */
    GABP_Q_PTILDE = 2,     /* [double N] aggregate precisions P~ (Alg. 2, "Infer") */
    GABP_Q_ADIAG = 3,      /* [double N] weighted diagonal A_ii */
    GABP_Q_BIAS = 4,       /* [double] b = lambda^2 sum_i alpha_i y_i */
    GABP_Q_SV_MASK = 5,    /* [uint8_t N] 1 iff alpha_i > sv_tau */
    GABP_Q_SV_COUNT = 6,   /* [int64_t] */
    GABP_Q_SWEEPS = 7,     /* [int32_t] completed sweeps */
    GABP_Q_DELTA = 8,      /* [double] last ||alpha^t - alpha^(t-1)||_inf */
    GABP_Q_STATUS = 9,     /* [int32_t] gabp_status of the last solve */
    GABP_Q_TIMINGS = 10,   /* [gabp_timings] */
    GABP_Q_TRACE = 11,     /* [double sweeps] change per sweep, t = 1..sweeps */
    GABP_Q_PLAN = 12,      /* [gabp_plan] */
    GABP_Q_REASON = 13,    /* [int32_t] gabp_reason */
    GABP_Q_EDGES = 14,     /* [int64_t 2 x n_edges] RBF_SPARSE: kept pairs
                              (i, j), i < j, in lexicographic order */
    GABP_Q_RESIDUAL_BOUND = 15 /* [double 3] a-posteriori certificate of a
                              dense solve (subsection "GaBP Algorithm
                              Convergence": the weighted diagonal makes A
                              strictly diagonally dominant):
                              [0] ||1 - A alpha||_inf over all N rows,
                              [1] min_i (A_ii - sum_{j != i} |A_ij|),
                              [2] Varah's bound [0] / [1] on
                              ||alpha - A^-1 1||_inf (+inf unless [1] > 0),
                              with A the device's own system (its K') and
                              alpha before output clipping.  Formed by one
                              pass over K' on the first query after a solve
                              (default stream); GABP_E_STATE for sparsified
                              solves */
};

/* Fills *p with the defaults: RBF, gamma 1, C 1, lambda 1/N, DOMINANT_ROW
 * with delta 0.1, no box, tol_abs 0, tol_rel 1e-7, max_sweeps 1000,
 * check_every 8, stagnation window 10 at 1e-5, MIXED, AUTO storage,
 * device 0. */
void gabp_svm_params_default(gabp_svm_params *p);

/* Creates a solver handle on params->device.  Validates the parameters
 * (GABP_E_INVALID), binds the device (GABP_E_DEVICE).  *out receives the
 * handle (NULL on error). */
gabp_status gabp_svm_create(const gabp_svm_params *params, gabp_svm **out);

/* Solves the SVM of section "Proposed Solution of SVM Solver Based on GaBP"
 * for the training set X (N x m float32, row-major) with labels y (N
 * float32, each exactly +1 or -1).  mem tells whether X and y are host or
 * device pointers; stream is a hipStream_t (NULL = the default stream) on
 * which all device work runs.  Blocks until the sweeps stop.
 * Returns GABP_OK (converged or stagnated at the precision floor),
 * GABP_E_NOT_CONVERGED (alpha = last iterate, queryable),
 * GABP_E_DIVERGED, GABP_E_INVALID (N < 1, m < 1, non-finite X, y not +-1,
 * checked before any device work), GABP_E_NOMEM, GABP_E_DEVICE. */
gabp_status gabp_svm_solve(gabp_svm *h, const float *X, const float *y,
                           int64_t N, int64_t m, int32_t mem, void *stream);

/* Same solve for a caller-supplied symmetric kernel matrix K' (N x N
 * float64, row-major; only the upper triangle and the diagonal are read),
 * used as is: lambda_aug is not added.  The diagonal weighting and labels
 * apply as in gabp_svm_solve, so with y = +1 and GABP_DIAG_NONE this solves
 * K' alpha = 1 for any symmetric K'.  Requires kernel = PRECOMPUTED and a
 * materialised plan.  Used to test the sweep on chosen matrices. */
gabp_status gabp_svm_solve_kernel(gabp_svm *h, const double *K, const float *y,
                                  int64_t N, int32_t mem, void *stream);

/* Copies the quantity `what` (GABP_Q_*) of the last solve into dst, which
 * holds `bytes` bytes of host memory.  GABP_E_BUFSIZE if too small,
 * GABP_E_STATE if no solve has run, GABP_E_INVALID for an unknown selector. */
gabp_status gabp_svm_query(const gabp_svm *h, int32_t what, void *dst, size_t bytes);

/* Entries K'_{ij} of the materialised kernel matrix of the last solve, for
 * the `n` index pairs (rows[k], cols[k]) (host int64 arrays, i != j), as
 * float64 into out (host).  GABP_E_STATE unless K' is materialised. */
gabp_status gabp_svm_kernel_entries(const gabp_svm *h, const int64_t *rows,
                                    const int64_t *cols, int64_t n, double *out);

/* Decision function of section "Classification Using Support Vector
 * Machines" with the bias carried by the augmentation:
 * f(x) = sum_i alpha_i y_i (K(x_i, x) + lambda^2) for the nq query points
 * Xq (nq x m float32, row-major; m of the last solve); f_out receives nq
 * float64 values; the class is sign(f) with sign(0) = +1.  mem applies to
 * Xq and f_out alike.  Dense RBF solves only (GABP_E_STATE otherwise). */
gabp_status gabp_svm_predict(gabp_svm *h, const float *Xq, int64_t nq,
                             double *f_out, int32_t mem, void *stream);

/* The decision function of gabp_svm_predict, allocating nothing: for callers
 * that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc).  Xq (nq x m float32,
 * row-major) and f_out (nq float64) are DEVICE pointers; the call only
 * enqueues work on `stream` (NULL = default stream) and returns, so f_out is
 * ready once that stream's work completes.  Weights, partial sums and staged
 * queries live in one scratch array of GABP_PREDICT_SCRATCH_BYTES per device,
 * held until the process ends and shared by every call on that device: calls
 * that overlap on one device (other streams, other threads or handles) race
 * on it and must be serialised by the caller.  Every scratch byte a call
 * reads is written earlier in the same call.  GABP_E_NOMEM (with the bytes
 * needed in gabp_svm_last_error) when one call's working set exceeds the
 * array -- about 3 * 128 * m_pad bytes per 128 queries plus 8 bytes per
 * training point and per (query, training chunk) partial sum;
 * GABP_E_STATE without a finished dense RBF solve. */
#define GABP_PREDICT_SCRATCH_BYTES (64u << 20)
gabp_status gabp_svm_predict_noalloc(gabp_svm *h, const float *Xq, int64_t nq,
                                     double *f_out, void *stream);

/* Frees the handle and everything it holds.  NULL is ignored. */
void gabp_svm_destroy(gabp_svm *h);

/* Static description of a status code. */
const char *gabp_status_string(int32_t status);

/* Message of the last failed call on h (empty if none); valid until the
 * next call on h. */
const char *gabp_svm_last_error(const gabp_svm *h);

/* GABP_ABI_VERSION of the library. */
int32_t gabp_abi_version(void);


/* ------------------------------------------------------------------------
 * Serving: continuous batching of many solves on one device.
 *
 * Not part of the paper (which solves one problem at a time); this is the
 * served form of the same sweep.  A background thread admits queued
 * requests in FIFO order (with a bounded bypass for smaller requests) when
 * their device footprint fits the server's memory arena and a slot is free,
 * keeps their K' tiles and pair-record messages resident, and advances all
 * active requests together: each step is one persistent sweep launch over
 * the union of their tiles, one batched finalize and one batched stop rule.
 * Requests join and leave at step boundaries.  Each request has its own
 * partial sums and fixed reduction order, so its alpha is bitwise the same
 * whether it runs alone or in a mix.  Served plans materialise K'; the edge
 * state (stored pair records or stateless) is chosen per request by the same
 * rule as gabp_svm_solve, and requests of the same precision and level count
 * share a launch.  A request with the GROUPED schedule advances one group
 * visit per step (its stop rule runs after the visit of its last group),
 * with the groups and lists of gabp_svm_solve, so its alpha is bitwise that
 * of the single grouped solve.
 * ------------------------------------------------------------------------ */
typedef struct gabp_server gabp_server;

typedef struct gabp_server_params {
    uint32_t struct_size;      /* sizeof(gabp_server_params) */
    int32_t device;            /* HIP device ordinal */
    uint64_t arena_bytes;      /* device memory arena for all requests;
                                  0 = 80% of the free device memory */
    int32_t max_active;        /* slots: requests resident at once (<= 1024) */
    int32_t steps_per_poll;    /* sweeps launched between status read-backs */
    int32_t max_bypass;        /* smaller requests admitted ahead of a queue
                                  head that does not fit, before the head
                                  blocks admission */
    int32_t reserved;
} gabp_server_params;

/* Outcome of one request (gabp_server_result). */
typedef struct gabp_request_info {
    int32_t status;            /* gabp_status of the solve */
    int32_t reason;            /* gabp_reason */
    int32_t sweeps;
    int32_t stateless_levels;  /* 0: stored pair records; >= 1: stateless levels */
    int64_t N;
    double latency_ms;         /* completion - submission (host clock) */
    double queue_ms;           /* admission - submission */
    double device_bytes;       /* footprint held while active */
} gabp_request_info;

/* Aggregate statistics over the requests completed so far. */
typedef struct gabp_server_stats {
    int64_t submitted, completed, failed;
    double p50_ms, p99_ms, mean_ms, max_ms;   /* latency percentiles */
    double mean_queue_ms;
    double throughput_per_s;   /* completed / (last completion - first submission) */
    double mean_active;        /* active requests per step, averaged over steps */
    int64_t max_active_seen;
    int64_t steps;             /* batched steps launched */
} gabp_server_stats;

/* Fills *p with defaults: device 0, arena 0 (80% of free memory),
 * max_active 64, steps_per_poll 2, max_bypass 8. */
void gabp_server_params_default(gabp_server_params *p);

/* Creates a server, allocates its arena and starts its scheduler thread.
 * GABP_E_INVALID for bad parameters, GABP_E_DEVICE without a gfx950
 * device, GABP_E_NOMEM if the arena cannot be allocated. */
gabp_status gabp_server_create(const gabp_server_params *params, gabp_server **out);

/* Queues one solve: X (N x m float32, row-major, host), y (N float32, +-1,
 * host) and the solver parameters (RBF kernel, K' materialised, SYNC or
 * GROUPED schedule, no box projection).  Inputs are copied before the call
 * returns.  *ticket identifies
 * the request.  GABP_E_INVALID for bad inputs or parameters, GABP_E_NOMEM if
 * the request can never fit the arena. */
gabp_status gabp_server_submit(gabp_server *srv, const float *X, const float *y, int64_t N,
                               int64_t m, const gabp_svm_params *params, uint64_t *ticket);

/* *done = 1 once the request finished (successfully or not). */
gabp_status gabp_server_poll(gabp_server *srv, uint64_t ticket, int32_t *done);

/* Blocks until the request finished or timeout_s elapsed (< 0: no limit);
 * GABP_E_STATE on time-out. */
gabp_status gabp_server_wait(gabp_server *srv, uint64_t ticket, double timeout_s);

/* Copies the finished request's alpha (N float64, box handling applied) to
 * alpha (host, `bytes` long; NULL skips it) and its outcome to *info (NULL
 * skips it).  GABP_E_STATE if not finished, GABP_E_BUFSIZE if too small. */
gabp_status gabp_server_result(gabp_server *srv, uint64_t ticket, double *alpha, size_t bytes,
                               gabp_request_info *info);

/* Latency / throughput statistics of the completed requests. */
gabp_status gabp_server_stats_get(gabp_server *srv, gabp_server_stats *out);

/* Stops the scheduler (active and queued requests are abandoned) and frees
 * everything.  NULL is ignored. */
void gabp_server_destroy(gabp_server *srv);

#ifdef __cplusplus
}
#endif

#endif /* GABP_SVM_H */
