// Launchers of the library's kernels, callable from any translation unit.
#pragma once

#include <vector>

#include "common.hpp"

namespace mcmf {

// out[i] = value for i < n (a kernel, so it is also safe inside captured graphs).
Status fill_u8(uint8_t *out, uint8_t value, int64_t n, hipStream_t s);
Status fill_i32(int32_t *out, int32_t value, int64_t n, hipStream_t s);
Status fill_f64(double *out, double value, int64_t n, hipStream_t s);
Status fill_u64(uint64_t *out, uint64_t value, int64_t n, hipStream_t s);

// Mask of the graph's hubs whose sums (by the walk kernel) replace the
// gather's probes for n_walks walks per start row and K: hubs of degree >=
// the tuning's hub_min_degree, by default >= n_walks (K - 1) / 4 (the walk
// adds a few operations per visit; a hub saves one probe per entry of its
// row per adjacent start row); 0 without hubs.
uint32_t active_hubs(const mcmf_graph *g, int64_t n_walks, int K);

// Builds the graph's alias records (weighted graphs; once, synchronously).
Status ensure_alias(mcmf_graph *g);

// Wide hubs (degree descending) whose sums the wide diagonal walk takes for
// n_walks and K: the prefix of degree >= the same threshold; 0 without them.
int32_t active_wide_hubs(const mcmf_graph *g, int64_t n_walks, int K);

// MCMF_SAMPLER_AUTO's choice for n_walks and K: the wide hub sums save at
// least kWideMinSavedPerState probed entries per recorded state.
bool auto_wide(const mcmf_graph *g, int64_t n_walks, int K);


// Ascending indices i < n with flags[i] == match written to out; *count (host)
// receives how many.  Synchronises the stream to read the count back.
Status compact(const uint8_t *flags, int64_t n, uint8_t match, int32_t *out, int64_t *count,
               hipStream_t s);

// Per-call walk parameters shared by the walk kernels.
struct WalkParams {
    const double *coef; // device: c_{t+2} at index t, t = 0..K-2
    int K;
    double scale;
    int64_t n_walks;
    uint32_t key0, key1;
    uint32_t request;
    double cutoff; // 0 = off
    int precision; // MCMF_PRECISION_*
    // Sampler layout, load policy and lanes per start row: -1 = the graph's tuning.
    int sampler = -1;
    int stream = -1;
    int threads = -1;
    // Neighbours per diagonal-gather work item: 0 = the graph's tuning.
    uint32_t gather_item = 0;
    // Walks per start row (device, indexed like the start list passed to the
    // walk launcher) and the first visit record of each of those rows
    // (prefix sums of walks * (K-1)); null: n_walks for every row.
    const int32_t *row_walks = nullptr;
    const int64_t *row_rec = nullptr;
    // Diagonal walks: hubs whose sums <Q_k, C_h> the walk kernel adds into
    // dacc as it records the visits (0: none), and the requested rows (null:
    // all).
    uint32_t hub_act = 0;
    const uint8_t *in_set = nullptr;
    double *dacc = nullptr;
    // Diagonal walks with wide hub sums: the active prefix of the graph's wide
    // hubs whose sums the walk takes (0: none; then hub_act applies).
    int32_t whub_act = 0;
};
// Whether diag_walks runs the wide-record kernel for these parameters.
bool wide_diag(const mcmf_graph *g, const WalkParams &p);

// r = s A v.
Status spmv_r(const mcmf_graph *g, const double *v, double scale, double *r, hipStream_t s);
// y = c0 v + c1 r + s A q (q may be null when K < 2: then only c0 v + c1 r).
Status spmv_assemble(const mcmf_graph *g, const double *v, const double *r, const double *q,
                     double c0, double c1, double scale, double *y, hipStream_t s);

// Action walks: q[k] for every k in starts[0..n_start).  digest/steps optional.
// Whether the action's value records (16 bytes per stored entry, held for
// the length of a call) stay within 1/16 of device memory.
bool value_records_fit(const mcmf_graph *g);

// rec[e] = {first entry of row col[e], its length, r[col[e]]} (unweighted
// graphs; rec holds nnz entries).
Status build_value_records(const mcmf_graph *g, const double *r, uint4 *rec, hipStream_t s);

Status action_walks(const mcmf_graph *g, const double *r, const int32_t *starts, int64_t n_start,
                    const WalkParams &p, double *q, uint64_t *digest, unsigned long long *steps,
                    hipStream_t s);

// Diag walks for starts[0..n_start): visit records, t-major per start row:
// state[(kk*(K-1) + t)*N + w], x = c_{t+2} W_t; finished walks store -1.
// x is double[] (FP64) or float[] (FP32 walk weights).
Status diag_walks(const mcmf_graph *g, const int32_t *starts, int64_t n_start, const WalkParams &p,
                  int32_t *state, void *x, uint64_t *digest, unsigned long long *steps,
                  hipStream_t s);

// Neighbours per diagonal-gather work item of the graph (its tuning).
uint32_t gather_item(const mcmf_graph *g);

// Recomputes the graph's work items of a full diagonal (after its tuning's
// gather_item changed); synchronises the graph's stream.
Status refresh_active_items(mcmf_graph *g);

// Work items of the diag gather: off[kk] = first item of start row kk
// (ceil(row length / gather_item(g)) items per row), off[n_start] = total.
// off has n_start + 1 entries.
Status gather_items(const mcmf_graph *g, const int32_t *starts, int64_t n_start, int64_t *off,
                    hipStream_t s, uint32_t item = 0);

// Diag gather for start rows starts[row_begin..row_end) of a start list with
// item offsets item_off (gather_items), whose visit records begin at
// state / x: for each requested neighbour i of a start row k,
// dacc[i] += s^2 a_ki <Q_k, C_i> / N.  in_set == null means every row is
// requested.  queue is a zeroed work counter used by this launch only.
Status diag_gather(const mcmf_graph *g, const int32_t *starts, const int64_t *item_off,
                   int64_t row_begin, int64_t row_end, const WalkParams &p, const int32_t *state,
                   const void *x, const uint8_t *in_set, double *dacc, unsigned long long *probes,
                   unsigned long long *overflow, unsigned long long *queue, hipStream_t s);

// Diag setup and assembly (api.hip).
Status mark_rows(const int32_t *rows, int64_t count, int64_t n, uint8_t *in_set, int *bad,
                 hipStream_t s);
Status mark_starts(const mcmf_graph *g, const int32_t *rows, int64_t count, uint8_t *start_flags,
                   hipStream_t s);
Status diag_finish(const mcmf_graph *g, const int32_t *rows, int64_t count, int K, double c0,
                   double c1, double scale, const double *dacc, double *out, hipStream_t s);
Status check_common(const mcmf_graph *g, const mcmf_fn *f, int64_t n_walks, int32_t K,
                    const mcmf_opts *o);

// Walks per start row of MCMF_ALLOC_NORM / MCMF_ALLOC_NORM_MIN1 (device
// arrays for the kernels, host copies for chunking and statistics).  Only the
// rows allocated at least one walk stay in the start list.
struct Allocation {
    DevBuf<int32_t> starts;         // start rows with at least one walk, ascending
    int64_t n_start = 0;
    DevBuf<int32_t> walks;          // per row of that list
    DevBuf<int64_t> rec;            // first visit record per row of the list, n_start + 1
    std::vector<int32_t> host_starts, host_walks;
    std::vector<int64_t> host_rec;
    int64_t total = 0, max_walks = 0;
};
// N_k = round(Ns p_k) over starts[0..n_start) (min_one: at least 1 each).
Status allocate_walks(const mcmf_graph *g, const int32_t *starts, int64_t n_start, int64_t Ns, int K,
                      bool min_one, Allocation &A, hipStream_t s);
Status write_walks_out(const mcmf_graph *g, const int32_t *starts, int64_t n_start, int64_t N_uniform,
                       const Allocation *A, int32_t *walks_out, hipStream_t s);
WalkParams walk_params(const mcmf_opts *o, const double *coef, int K, double scale, int64_t N);

// Batched execution (batch.hip): argument check of one request, and a batch.
Status check_request(mcmf_request &q);
Status run_batch(mcmf_request *reqs, int64_t n_reqs, const mcmf_batch_opts *o, mcmf_stats *stats);

} // namespace mcmf
