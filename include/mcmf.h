/*
 * mcmf.h -- C ABI of the MI355X library for the row/column-sampling Monte
 * Carlo estimator of power-series matrix functions on sparse graphs.
 *
 * Method: Guidotti, Acebron and Monteiro, "A fast Monte Carlo algorithm for
 * evaluating matrix functions with application in complex networks".
 * For f(sA) = sum_{k=0}^{K} c_k (sA)^k over the adjacency matrix A of a
 * graph (Section 2.2, Eq. power_series, with the inverse-temperature scale
 * s of the parametric form f(gamma A)) the library computes
 *
 *   - subgraph centrality  diag(f(sA))        (Section 3.3, RandFunmDiag,
 *                                               Eq. rand_funm_formula_diag)
 *   - total communicability / action f(sA) v  (Section 3.4, Algorithm 3,
 *                                               Eq. rand_funm_action_formula;
 *                                               v = 1 gives Eq. total_comm)
 *
 * on one AMD Instinct MI355X (gfx950).  The exact part H = c0 I + c1 sA
 * (Corollary 1) is computed exactly; the rest, U = sum_{k>=2} c_k (sA)^k, is
 * estimated from random walks on the Markov chain of Definition 1 (ii),
 * t_ij = |a_ij| / sum_k |a_ik|, with weights W^(k) = W^(k-1) a/t (Lemma 2).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Pointers.  Every array argument may be host memory or device memory of the
 * current HIP device; the library detects which.  The caller owns every
 * array it passes; the library never keeps a caller pointer after a call
 * returns (mcmf_graph_create copies the CSR into device memory).
 *
 * Walks.  K is the highest power kept.  Each start row k gets exactly
 * n_walks walks; a walk records the states t = 0..K-2 (K-1 states, K-2
 * transitions), so the expectation of the estimate is exactly the series
 * truncated at K.  The transition out of step t of walk w from start row k
 * draws Philox4x32-10 (Salmon et al., SC'11) at counter (k, w, t,
 * request_id) with key (low, high 32-bit word of seed) and uses
 * u = X1 * 2^32 + X0.  An unweighted row picks entry floor(u * deg / 2^64);
 * a weighted row picks the first entry j with u53 * rowabs < cum_j
 * (u53 = (u >> 11) * 2^-53, running sums of |a| taken left to right).
 * Identical (graph, seed, request_id, n_walks, K) therefore give identical
 * walks, whatever row subset, stream or batch they run in.
 *
 * Errors.  Every call returns a status.  On any status other than MCMF_OK
 * the output arrays are left untouched (a failure inside the GPU work of an
 * asynchronous call is reported by the next synchronising call instead).
 * mcmf_last_error() gives a readable message for the calling thread.
 *
 * Streams.  opts->stream == NULL: the call uses the graph's own stream and
 * returns when the outputs are complete.  A non-NULL hipStream_t with every
 * array in device memory and stats == NULL makes the call asynchronous and
 * ordered on that stream; otherwise it synchronises before returning.
 *
 * Thread safety.  Graphs are immutable after creation; concurrent calls on
 * one graph are allowed.  Destroying a graph while a call on it is running
 * is undefined.
 */
#ifndef MCMF_H
#define MCMF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MCMF_VERSION_MAJOR 1
#define MCMF_VERSION_MINOR 1

typedef struct mcmf_graph mcmf_graph; /* opaque; owns its device copy of A */

typedef enum {
    MCMF_OK = 0,
    MCMF_E_ARG = 1,           /* bad scalar or pointer argument */
    MCMF_E_CSR = 2,           /* malformed CSR arrays */
    MCMF_E_NOT_SYMMETRIC = 3, /* diag needs A = A^T (C_i = R_i) */
    MCMF_E_NOMEM = 4,         /* device memory or the byte budget exhausted */
    MCMF_E_DEVICE = 5,        /* HIP runtime error or no usable device */
    MCMF_E_UNSUPPORTED = 6    /* valid request outside what the library handles */
} mcmf_status;

/* Function family: coefficients c_k of f(x) = sum_k c_k x^k (Eq. power_series). */
typedef enum {
    MCMF_FN_EXP = 0,       /* c_0 = 1, c_k = c_{k-1} / k (exponential) */
    MCMF_FN_RESOLVENT = 1, /* c_k = 1: (I - sA)^-1 (Katz centrality, Section 4.5) */
    MCMF_FN_COEFFS = 2     /* caller-supplied c_0 .. c_{n_coeffs-1} */
} mcmf_fn_kind;

typedef struct {
    int32_t kind;          /* mcmf_fn_kind */
    double scale;          /* s: the estimate is of f(sA); must be finite */
    const double *coeffs;  /* MCMF_FN_COEFFS only: host array, n_coeffs >= K+1 */
    int32_t n_coeffs;
} mcmf_fn;

/* Flags for mcmf_graph_create. */
#define MCMF_SYMMETRIC 1u /* caller states A = A^T; required by mcmf_diag */
#define MCMF_VALIDATE 2u  /* check the CSR arrays (and, with MCMF_SYMMETRIC, symmetry) */
#define MCMF_DIGRAPH 4u   /* A is a directed graph: store B = [[0, A], [A^T, 0]] (Section 4,
                             Eq. digraph_sym), 2n x 2n and symmetric; rows 0..n-1 of B
                             are A's rows (out-edges), rows n..2n-1 its columns (in-edges) */

/* Precision of the walk weights.  MCMF_PRECISION_FP32_WEIGHTS keeps W, the
 * per-step factor s*sum|a| and each per-step contribution (c_{t+2} W r_l for
 * the action, c_{t+2} W for the diagonal) in FP32; every sum over steps, walks
 * and the gather stays FP64.  Walk paths are identical to the FP64 mode, so
 * the difference from FP64 is rounding only.  Step t's weight carries at
 * most 2t roundings (factor and product) and a term two or three more, so
 *     |x_fp32 - x_fp64| <= 2 K * 2^-24 * sum |terms|
 * per output (to first order, ignoring FP32 underflow of terms below 1e-38),
 * where sum |terms| is the sum of the absolute values of the walk terms
 * behind that output (the Monte Carlo part itself when A, v >= 0).
 * FP32 weights must stay below 3.4e38 in magnitude: functions whose weights
 * grow (s * sum|a| > 1 over many steps) overflow to inf in this mode. */
#define MCMF_PRECISION_FP64 0
#define MCMF_PRECISION_FP32_WEIGHTS 1

/* Allocation of walks over the start rows.  MCMF_ALLOC_PER_ROW: n_walks
 * walks from every start row.  MCMF_ALLOC_NORM (Definition 1 (i), Eq.
 * initial_prob, with N_i = N_s P(l0 = i) of Algorithms 2-3): n_walks is the
 * total N_s; start row k gets N_k = round(N_s ||C_k||_2 / sum over the start
 * rows of ||C||_2) walks, rounding half away from zero.  N_k may be 0: such a
 * row starts no walk and adds nothing to Q (diag) or q (action), so an output
 * row whose whole neighbourhood got no walk is exactly c0 + c1 s a_ii (diag)
 * or c0 v_i + c1 (sAv)_i (action), the small-N_s regime of Section 4.1.
 * MCMF_ALLOC_NORM_MIN1 is the same with at least one walk per start row (a
 * variant of this library, not the paper's: every start row's term is then
 * estimated).  Column norms: for a graph created with MCMF_SYMMETRIC,
 * ||C_k|| = ||R_k|| summed along row k in stored order; otherwise
 * (unweighted graphs only) ||C_k||^2 is the number of entries in column k.
 * The total is summed over the start rows in ascending order, on the host.
 * mcmf_diag and mcmf_action only (not mcmf_batch). */
#define MCMF_ALLOC_PER_ROW 0
#define MCMF_ALLOC_NORM 1
#define MCMF_ALLOC_NORM_MIN1 2

typedef struct {
    uint64_t seed;          /* RNG key */
    uint32_t request_id;    /* fourth Philox counter word; same id => same walks */
    int32_t precision;      /* MCMF_PRECISION_* */
    double weight_cutoff;   /* Wc > 0: a walk stops before step t once |W_t| <= Wc
                               (Eq. weight_cutoff with W^(0) = 1); 0 = off */
    void *stream;           /* hipStream_t or NULL */
    uint64_t *path_digest;  /* optional out, n entries: per start row k the wrapping
                               sum over its walks of FNV-1a over the 32-bit words of
                               the recorded states; 0 for rows that start no walk */
    double *q_out;          /* optional out (mcmf_action only), n entries: q_k of
                               Algorithm 3 per start row, 0 elsewhere */
    int32_t *walks_out;     /* optional out, n entries: walks started from each row
                               (0 for rows that start none) */
    int32_t allocation;     /* MCMF_ALLOC_* */
    uint32_t reserved[5];   /* must be zero */
} mcmf_opts;

typedef struct {
    uint64_t start_rows;    /* rows that started walks */
    uint64_t walks;         /* walks started (start_rows * n_walks per row) */
    uint64_t walk_steps;    /* recorded walk states (K-1 per full walk) */
    uint64_t gather_probes; /* mcmf_diag: column entries the gather probed (hub rows summed
                               by the walks are not probed) */
    double ms_setup;        /* marks, start set, temporaries */
    double ms_spmv;         /* r = sA v and the final assembly (action);
                               the final assembly of the diagonal (diag) */
    double ms_walk;         /* walk kernels */
    double ms_gather;       /* Q_k build + column gather + scatter (diag) */
    double ms_total;        /* whole call, device time */
} mcmf_stats;

/*
 * mcmf_graph_create -- copy a CSR matrix into device memory and build the
 * per-row metadata the walks need (Section 2.1, Eq. adj_matrix; the
 * transition matrix T of Definition 1 (ii) is implied by the rows and never
 * stored for unweighted graphs).
 *
 *   n        number of rows/columns, 0 <= n < 2^31
 *   row_ptr  int64[n+1], row_ptr[0] = 0, non-decreasing; nnz = row_ptr[n] < 2^32
 *   col_idx  int32[nnz], 0 <= col < n (order within a row is kept: it is the
 *            order the sampler's cumulative sums run in)
 *   values   double[nnz], finite; NULL means every stored entry is 1
 *   flags    MCMF_SYMMETRIC | MCMF_VALIDATE, or MCMF_DIGRAPH (| MCMF_VALIDATE)
 *   out      receives the handle; set only on MCMF_OK
 *
 * With MCMF_DIGRAPH the graph is B = [[0, A], [A^T, 0]]: n and nnz of the
 * handle are 2n and 2 nnz, B is symmetric (mcmf_diag allowed).  Row i < n of
 * B holds A's row i with columns shifted by n, in A's order; row n + j holds
 * column j of A: the rows i with a_ij != 0, ascending, with the values a_ij.
 * B is assembled on the host (A is read back first if it is in device
 * memory); columns are always range-checked there (MCMF_E_CSR).  Requires
 * n < 2^30 and 2 nnz < 2^32.
 *
 * Errors: MCMF_E_ARG (null out, n out of range, null arrays with nnz > 0),
 * MCMF_E_CSR (with MCMF_VALIDATE: row_ptr[0] != 0, decreasing row_ptr, a
 * column out of range, a non-finite value; without it only row_ptr[0] and
 * row_ptr[n] are checked), MCMF_E_NOT_SYMMETRIC (MCMF_VALIDATE |
 * MCMF_SYMMETRIC and A != A^T, or unsorted rows, which that check needs),
 * MCMF_E_UNSUPPORTED (nnz >= 2^32), MCMF_E_NOMEM, MCMF_E_DEVICE.
 */
mcmf_status mcmf_graph_create(int64_t n, const int64_t *row_ptr, const int32_t *col_idx,
                              const double *values, uint32_t flags, mcmf_graph **out);

/* ------------------------------------------------------------------ */
/* Tuning                                                              */
/* ------------------------------------------------------------------ */

/* Sampler layouts of an unweighted walk step (Definition 1 (ii): both pick
 * entry floor(u deg / 2^64) of the current row; results are identical). */
#define MCMF_SAMPLER_EDGE 0 /* one 16-byte record per step: the picked entry carries
                               the next row's record (one dependent load) */
#define MCMF_SAMPLER_ROW 1  /* the picked column (4 bytes), then the next row's record
                               (8 bytes): two dependent loads, less data per step */
#define MCMF_SAMPLER_VALUE 2 /* mcmf_action on unweighted graphs only: per-call 16-byte
                               records {next row's record, r of the next row}, so a
                               step makes one load and no separate read of r = sAv.
                               Costs 16 bytes per stored entry during the call; falls
                               back to EDGE with a path digest, on weighted graphs or
                               when 16 nnz exceeds 1/16 of device memory */
#define MCMF_SAMPLER_WIDE 3  /* mcmf_diag on graphs with wide hubs only (below): EDGE
                               records, and for each visit the state's 128-byte mask of
                               up to 1024 hubs (the chunks a start row needs, loaded
                               with the step's record); the walk sums <Q_k, C_h> for
                               all those hubs as it goes and the gather skips them */
#define MCMF_SAMPLER_AUTO 5  /* mcmf_diag: per call, WIDE where the wide hub sums save at
                               least 4 probed column entries per recorded walk state
                               (the squared degrees of the active wide hubs beyond the
                               first 32, over the call's n_active N (K-1) states), else
                               EDGE.  The default on graphs with wide hubs unless the ROW
                               default applies; measured crossover on R-MAT graphs at
                               N = 256, K = 40: 3.5 saved per state 2% slower, 5.1 4%
                               faster */
#define MCMF_SAMPLER_ALIAS 4 /* weighted graphs only, action or diagonal: Walker's alias
                               method (Vose's construction) instead of the running sums
                               of |a|.  Entry i = floor(u deg / 2^64) from Philox words
                               X0:X1 is kept when the 53-bit uniform from X2:X3 is below
                               its probability, else its alias is taken: one 16-byte
                               record per step instead of a binary search.  Same law
                               (Definition 1 (ii)), other paths.  The default for both
                               walks on weighted graphs; the records (16 bytes per stored
                               entry, 12 more during the build) are built with the graph,
                               which keeps the running sums when they do not fit.  EDGE or
                               ROW select the running sums of |a| instead */

/* Per-graph choices of the walk kernels and of the diagonal gather.  On
 * unweighted graphs they change memory traffic and the order of
 * floating-point sums only: walk paths and step counts never change.  On
 * weighted graphs ALIAS and the running sums (EDGE, ROW) draw other paths
 * from the same law.  Defaults: action VALUE with cached loads; diag ROW
 * with cached loads when the column array and row records take at most
 * 16 MiB (4 nnz + 8 n bytes; they then stay in cache), AUTO where the graph
 * has wide hubs, else EDGE with cached loads; ALIAS for both walks on
 * weighted graphs; automatic hub threshold.  The batched walks (mcmf_batch
 * and the server) use EDGE records (value records for unweighted actions,
 * alias records for weighted rows when the graph's layout is ALIAS).
 *
 * Hub rows: a graph created unweighted with MCMF_SYMMETRIC and strictly
 * increasing columns in every row keeps its (at most 32) rows of largest
 * degree as hubs, with one 32-bit mask per node of the hubs it is adjacent
 * to (also kept in the spare word of every edge record).  For a start row
 * k next to a hub h, <Q_k, C_h> of Eq. rand_funm_formula_diag is then the
 * sum of the visit weights of k's walks at states adjacent to h, which the
 * diagonal walk adds up as it records the visits (the mask arrives with the
 * record it loads anyway), instead of one probe of Q_k per entry of row h
 * in the gather.  The graph's hubs, and the masks, assume the symmetry that
 * MCMF_SYMMETRIC states.
 *
 * Wide hubs: such a graph with more than 32 rows with entries also keeps its
 * (up to 1024) rows of largest degree as wide hubs, with a 128-byte mask per
 * node of those adjacent to it (130 bytes per node in all), when that fits
 * 1/32 of device memory, and then defaults diag_sampler to MCMF_SAMPLER_AUTO
 * unless the ROW default above applies.  hub_min_degree picks the active wide
 * hubs as it picks the 32-bit ones.  The batched walks keep the 32-bit hubs. */
typedef struct {
    int32_t action_sampler;  /* MCMF_SAMPLER_* of mcmf_action walks */
    int32_t action_stream;   /* 1: the walk's record loads are non-temporal */
    int32_t diag_sampler;    /* MCMF_SAMPLER_* of mcmf_diag walks (WIDE: graphs with wide
                                hub records only; the stream flag does not apply) */
    int32_t diag_stream;     /* 1: non-temporal record loads */
    double action_ms[4];     /* mcmf_tune only: ms of each EDGE/ROW action variant, index
                                sampler*2+stream */
    double diag_ms[4];       /* mcmf_tune only: ms of each diag-walk variant, same index */
    int64_t sample_rows;     /* mcmf_tune only: start rows in the timed sample */
    int32_t hub_min_degree;  /* diagonal (unweighted graphs): a hub row (below) of at least
                                this many entries has its sums taken by the walk kernel
                                instead of being probed entry by entry by the gather;
                                0 = automatic, a degree of at least n_walks (K - 1) / 4;
                                INT32_MAX turns hub sums off.  Batched requests with
                                n_walks < 32 never use them */
    int32_t hub_count;       /* out of mcmf_graph_get_tuning: hub rows the graph holds;
                                ignored on input */
    double action_value_ms[2]; /* mcmf_tune only: ms of the VALUE action walk, index stream
                                  (0 when the graph cannot use it) */
    int32_t walk_threads;    /* lanes per start row of the mcmf_diag / mcmf_action walks,
                                64, 128 or 256 (each lane runs every walk_threads-th
                                walk of the row); 0 = automatic, the walk count rounded
                                up to 64 lanes, at most 256 */
    int32_t gather_item;     /* neighbours of a start row per diagonal-gather work item
                                (every item rebuilds Q_k, so larger items rebuild less
                                and spread a high-degree row over fewer workgroups),
                                64..4096; 0 = 256 */
    double walk_threads_ms[3]; /* mcmf_tune only: ms of the diag walk at 64/128/256 lanes */
    double gather_item_ms[4];  /* mcmf_tune only: ms of the diagonal gather at items of
                                  128/256/512/1024 neighbours */
    double hub_ms[2];          /* mcmf_tune only: ms of diag walk + gather with hub sums at
                                  the automatic threshold / off (0 without hubs) */
    double wide_ms;            /* mcmf_tune only: ms of the same with wide hub sums
                                  (MCMF_SAMPLER_WIDE; 0 without wide hubs) */
    double alias_ms[2];        /* mcmf_tune only, weighted graphs: ms of the action and the
                                  diagonal walk with MCMF_SAMPLER_ALIAS (0 otherwise) */
    int32_t wide_hub_count;    /* out of mcmf_graph_get_tuning: wide hub rows the graph holds
                                  (0: MCMF_SAMPLER_WIDE is not available); ignored on input */
    int32_t reserved;          /* zero */
} mcmf_tuning;

/* Set / read a graph's tuning.  Not to be called while a request on the
 * graph runs.  Errors: MCMF_E_ARG (null pointers, values out of range). */
mcmf_status mcmf_graph_set_tuning(mcmf_graph *g, const mcmf_tuning *t);
mcmf_status mcmf_graph_get_tuning(const mcmf_graph *g, mcmf_tuning *t);

/*
 * mcmf_tune -- the autotuner.  On a sample of the graph's rows (rows with
 * entries taken at an even stride, about 2^28 walk steps in all, with the
 * function, n_walks and K of the intended requests) it times, in turn:
 * every sampler layout and load policy of the action and diagonal walk
 * kernels; the diagonal walk at 64, 128 and 256 lanes per start row; the
 * diagonal gather (every neighbour of the sampled rows requested) at work
 * items of 128, 256, 512 and 1024 neighbours; and, on graphs with hub rows,
 * diagonal walk plus gather with hub sums at the automatic threshold and
 * off, and with wide hub sums where the graph has wide hubs; on weighted
 * graphs, both walks with the running sums and with alias records.  It keeps
 * the fastest of each, except that the lanes, the work-item size, hub sums
 * on and the graph's current wide-hub choice stay unless another option is
 * more than 3% faster on the sample (its timings carry a few per cent of
 * noise and of sampling bias), and stores the result in the graph
 * (mcmf_graph_set_tuning).  out receives the choice and the measured times.
 * The caller may cache the result by a fingerprint of the graph and reapply
 * it with mcmf_graph_set_tuning.
 * Errors: as mcmf_action (K >= 2, n_walks >= 1 required), MCMF_E_NOMEM,
 * MCMF_E_DEVICE.
 */
mcmf_status mcmf_tune(mcmf_graph *g, const mcmf_fn *f, int64_t n_walks, int32_t K, mcmf_tuning *out);

/* Release the graph's device memory.  NULL is ignored. */
void mcmf_graph_destroy(mcmf_graph *g);

/*
 * mcmf_graph_info -- sizes of a graph: n, nnz, the largest row length d_max
 * (used for the scale 1/d_max) and the number of rows with at least one
 * entry.  Any output pointer may be NULL.
 */
mcmf_status mcmf_graph_info(const mcmf_graph *g, int64_t *n, int64_t *nnz, int64_t *d_max,
                            int64_t *active_rows);

/*
 * mcmf_diag -- RandFunmDiag (Section 3.3): out[p] estimates f(sA)_{ii} for
 * i = rows[p],
 *
 *   d_i = c0 + c1 s a_ii + s^2 sum_k a_ik <Q_k, C_i>      (Eq. rand_funm_formula_diag)
 *
 * with Q_k = (1/n_walks) sum_{walks from k} sum_t c_{t+2} W_t e_{l_t}
 * (Eq. rand_funm_Q).  Walks start from every row k adjacent to a requested
 * row; each Q_k is used for all requested rows adjacent to k.
 *
 *   g        graph created with MCMF_SYMMETRIC
 *   f        function and scale
 *   rows     int32[n_rows] requested rows, any order, duplicates allowed, or
 *            NULL for every row (then n_rows is ignored and out has n entries)
 *   n_walks  walks per start row, >= 1 when K >= 2
 *   K        highest power kept, 0 <= K <= 4096
 *   opts     may be NULL (seed 0, request 0, FP64, no cutoff, own stream)
 *   out      double[n_rows] (or [n])
 *   stats    optional
 *
 * Device memory: the visit records (12 bytes per walk step, 8 with FP32
 * weights) go through one buffer of at most the MCMF_DIAG_CHUNK_BYTES
 * environment value, else 1/16 of device memory within [256 MiB, 16 GiB],
 * halved (down to 256 MiB) while the allocation fails for lack of memory; a
 * larger total is walked and gathered in chunks of start rows.  Each chunk's
 * gather also takes a map of its work items (4 bytes per item: at most one
 * per start row plus one per 256 stored entries, at most 32 MiB).
 *
 * Errors: MCMF_E_ARG (null g/f/out, K out of range, n_walks < 1 with K >= 2,
 * n_rows < 0, a row outside [0, n), non-finite scale or coefficients,
 * n_coeffs < K+1, non-zero reserved words), MCMF_E_NOT_SYMMETRIC,
 * MCMF_E_NOMEM, MCMF_E_DEVICE.  MCMF_E_DEVICE also reports a lost insert
 * into a Q_k table (an internal sizing error that the table plan rules
 * out): a synchronising call reports its own; an asynchronous call records
 * it on the graph, and the next synchronising mcmf_diag on that graph whose
 * stream has passed the failing work returns it (and clears the record).
 */
mcmf_status mcmf_diag(const mcmf_graph *g, const mcmf_fn *f, const int32_t *rows, int64_t n_rows,
                      int64_t n_walks, int32_t K, const mcmf_opts *opts, double *out,
                      mcmf_stats *stats);

/*
 * mcmf_action -- RandFunmAction (Section 3.4, Algorithm 3): out = estimate of
 * f(sA) v,
 *
 *   r = s A v,  q_k = (1/n_walks) sum_{walks from k} sum_t c_{t+2} W_t r_{l_t},
 *   out = c0 v + c1 r + s A q                       (Eq. rand_funm_action_formula)
 *
 * Walks start from every row with at least one entry.  A need not be
 * symmetric; a walk that reaches a row without entries stops.
 *
 *   v        double[n]
 *   out      double[n]; may not alias v
 *   other arguments as for mcmf_diag
 *
 * Errors: MCMF_E_ARG (null g/f/v/out, K out of range, n_walks < 1 with
 * K >= 2, non-finite scale or coefficients, n_coeffs < K+1, non-zero reserved
 * words), MCMF_E_NOMEM, MCMF_E_DEVICE.
 */
mcmf_status mcmf_action(const mcmf_graph *g, const mcmf_fn *f, const double *v, int64_t n_walks,
                        int32_t K, const mcmf_opts *opts, double *out, mcmf_stats *stats);

/*
 * mcmf_action_noalloc -- mcmf_action for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, and hosts that
 * forbid allocation during a request.  It computes what mcmf_action computes
 * (same walks, same estimate up to the order of floating-point additions)
 * and calls no hipMalloc, hipFree or other allocating routine.
 *
 * Its temporaries (r = sAv, q, the coefficients: 16 n bytes + 32 KiB) live in
 * one 64 MiB device array of the library, one copy per device, held until
 * the process ends; its address is looked up once per device on the first
 * call there.  Every call on a device shares that device's array and leaves
 * its contents behind (each call writes what it reads first): calls that
 * overlap on one device, on any streams or threads, race and give wrong
 * results.  Order them on one stream or serialise them.
 *
 *   g, f, n_walks, K   as for mcmf_action; g has n <= MCMF_NOALLOC_MAX_ROWS
 *   v, out             double[n] in device memory of the graph's device
 *   opts               may be NULL; allocation must be MCMF_ALLOC_PER_ROW and
 *                      walks_out NULL; path_digest and q_out, if given, in
 *                      device memory.  stream NULL: the graph's stream, and
 *                      the call returns when out is complete; otherwise the
 *                      call is asynchronous on that stream.
 *
 * Walks use the graph's EDGE or ROW records (a VALUE tuning runs EDGE).
 *
 * Errors: those of mcmf_action; MCMF_E_ARG also when v, out, path_digest or
 * q_out is host memory; MCMF_E_UNSUPPORTED when n exceeds
 * MCMF_NOALLOC_MAX_ROWS, for another allocation mode or a walks_out array.
 */
#define MCMF_NOALLOC_MAX_ROWS 4192256LL /* (64 MiB - 32 KiB) / 16 */
mcmf_status mcmf_action_noalloc(const mcmf_graph *g, const mcmf_fn *f, const double *v,
                                int64_t n_walks, int32_t K, const mcmf_opts *opts, double *out);

/* ------------------------------------------------------------------ */
/* Batched execution                                                   */
/* ------------------------------------------------------------------ */

typedef enum { MCMF_REQ_DIAG = 0, MCMF_REQ_ACTION = 1 } mcmf_request_kind;

/* One request of a batch: the arguments of one mcmf_diag / mcmf_action call.
 * Arrays follow the conventions above (host or device memory). */
typedef struct {
    int32_t kind;               /* mcmf_request_kind */
    int32_t K;                  /* highest power kept, 0 <= K <= 4096 */
    const mcmf_graph *graph;    /* diag: created with MCMF_SYMMETRIC */
    mcmf_fn fn;
    const int32_t *rows;        /* diag: requested rows (NULL: every row) */
    int64_t n_rows;             /* diag: number of requested rows */
    const double *v;            /* action: double[n] */
    int64_t n_walks;            /* walks per start row, >= 1 when K >= 2 */
    uint64_t seed;
    uint32_t request_id;
    int32_t precision;          /* MCMF_PRECISION_* */
    double weight_cutoff;       /* as in mcmf_opts */
    double *out;                /* diag: double[n_rows] (or [n]); action: double[n] */
    uint64_t *path_digest;      /* optional, as in mcmf_opts */
    mcmf_status status;         /* out: this request's status */
    uint64_t walk_steps;        /* out: recorded walk states of this request */
} mcmf_request;

typedef struct {
    void *stream;               /* hipStream_t the batch is ordered on, or NULL for the
                                   stream of the first request's graph */
    int32_t use_graph;          /* 1: record the batch's launches in a hipGraph, then
                                   launch that graph (one submission for the batch).  If
                                   another host thread invalidates the capture (some HIP
                                   calls in threads left in the default capture-interaction
                                   mode do), the batch is launched directly instead */
    int32_t reserved0;          /* must be zero */
    uint64_t visit_chunk_bytes; /* diagonal visit-record buffer of the batch; 0: the
                                   MCMF_DIAG_CHUNK_BYTES environment value, else 1/16 of
                                   device memory within [256 MiB, 16 GiB] */
    uint32_t reserved[4];       /* must be zero */
} mcmf_batch_opts;

/*
 * mcmf_batch -- run several diag / action requests (any mix of graphs,
 * functions, walk counts, K and precisions on one device) as one unit of
 * GPU work.  All walks of all requests run in one persistent walk kernel
 * (work items: 64 walks of one start row of one request, taken by
 * wavefronts in turn), the diagonal gathers in persistent gather kernels
 * (one per visit-buffer chunk and kernel variant: FP64 / FP32 weights,
 * unweighted / weighted graph).  Every request's walks are the ones its own
 * mcmf_diag / mcmf_action call would draw (same keyed counters), so its
 * result equals that call's result up to the order of floating-point
 * additions.  The call returns once the whole batch is complete and its
 * outputs are written.
 *
 *   reqs    array of n_reqs requests; status and walk_steps are written
 *   opts    may be NULL
 *   stats   optional: totals over the batch (start_rows, walks, walk_steps,
 *           gather_probes, ms_total)
 *
 * Calls that overlap on one stream are ordered; on different streams they
 * are independent (each call owns its scratch buffers).
 *
 * Errors: a request with invalid arguments gets its own status and fails the
 * whole batch with that status before any work starts (no output written);
 * MCMF_E_NOMEM, MCMF_E_DEVICE as for the single calls.
 */
mcmf_status mcmf_batch(mcmf_request *reqs, int64_t n_reqs, const mcmf_batch_opts *opts,
                       mcmf_stats *stats);

/* ------------------------------------------------------------------ */
/* Serving                                                             */
/* ------------------------------------------------------------------ */

/*
 * A request server on one device: graphs stay resident (created beforehand
 * with mcmf_graph_create), requests arrive from any host thread, and the
 * server runs them with continuous batching.  A dispatcher admits queued
 * requests in arrival order against a device-memory budget, groups them into
 * a batch (mcmf_batch) whenever one of its n_streams stream slots is free,
 * and hands the batch to that slot's worker; batches on different streams
 * overlap on the device.  A batch completes as a unit, so requests join one
 * only while its estimated walk steps stay within max_batch_steps: a large
 * request runs on its own stream while small ones keep flowing on the
 * others, and at most max_large_in_flight large requests share the device
 * (so that large requests do not slow each other down).  Requests that
 * arrive while batches run join the next batch as slots and memory free up.  Results equal those of the
 * request's own mcmf_diag / mcmf_action call up to the order of
 * floating-point additions (keyed walks).
 */
typedef struct mcmf_server mcmf_server;

typedef struct {
    uint64_t hbm_budget_bytes;  /* admission budget: estimated device bytes of all
                                   batches in flight; 0: no limit.  A request larger
                                   than the budget runs alone once the device is idle. */
    uint64_t visit_chunk_bytes; /* diagonal visit-record buffer per batch; 0: 256 MiB */
    int32_t n_streams;          /* stream slots (batches in flight), 1..16; 0: 2 */
    int32_t max_batch;          /* most requests per batch, >= 1; 0: 64 */
    int32_t device;             /* HIP device of the server and its graphs */
    int32_t use_graph;          /* 1: each batch is recorded into a hipGraph and launched */
    uint64_t max_batch_steps;   /* a batch takes further requests only while its estimated
                                   walk steps stay within this; a request above it runs
                                   alone; 0: 2^28 */
    int32_t max_large_in_flight; /* most requests above max_batch_steps running at once,
                                   1..n_streams; 0: 1.  A large request that would exceed
                                   it waits, and the smaller requests queued behind it
                                   are dispatched past it in arrival order */
    uint32_t reserved[5];       /* must be zero */
} mcmf_server_opts;

typedef struct {
    mcmf_status status;         /* the request's status */
    int32_t batch_size;         /* requests in the batch it ran in */
    double queue_ms;            /* submit -> start of its batch (host clock) */
    double run_ms;              /* start -> end of its batch */
    uint64_t est_bytes;         /* its admission estimate */
    uint64_t est_steps;         /* its estimate of walk steps (batch forming); for actions
                                   and full diagonals an upper bound */
} mcmf_ticket_info;

typedef struct {
    uint64_t submitted, completed, batches;
    uint64_t bytes_in_flight;       /* current admission total */
    uint64_t peak_bytes_in_flight;  /* largest admission total so far */
    uint64_t peak_batches_in_flight;
    uint64_t largest_batch;
    uint64_t peak_large_in_flight;  /* most requests above max_batch_steps run at once */
    uint32_t reserved[6];
} mcmf_server_stats;

/*
 * mcmf_server_create -- start a server (its dispatcher and one worker thread
 * per stream slot; streams at default priority).
 * Errors: MCMF_E_ARG (null out, values out of range, non-zero reserved
 * words), MCMF_E_DEVICE.
 */
mcmf_status mcmf_server_create(const mcmf_server_opts *opts, mcmf_server **out);

/*
 * mcmf_server_submit -- queue one request.  The request is checked here (an
 * invalid one is refused with its status and never queued) and sized from
 * its sizes alone (no device access: submitting never waits for the device).
 * The request struct and every array it names must stay valid until
 * mcmf_server_wait for its ticket returns; the outputs, status and
 * walk_steps are written by then.  Thread-safe.
 */
mcmf_status mcmf_server_submit(mcmf_server *s, mcmf_request *req, uint64_t *ticket);

/*
 * mcmf_server_wait -- block until the ticket's request has run; returns its
 * status (info optional).  Each ticket is waited for exactly once; an
 * unknown or already-waited ticket gives MCMF_E_ARG.  Thread-safe.
 */
mcmf_status mcmf_server_wait(mcmf_server *s, uint64_t ticket, mcmf_ticket_info *info);

/* Counters of the server (thread-safe snapshot). */
mcmf_status mcmf_server_query(mcmf_server *s, mcmf_server_stats *stats);

/* Run every queued request, stop the threads, free the server. */
void mcmf_server_destroy(mcmf_server *s);

/* Static name of a status code. */
const char *mcmf_status_string(mcmf_status s);

/* Message describing the calling thread's last failure ("" if none). */
const char *mcmf_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* MCMF_H */
