/*
 * mcmf_oracle.c -- plain, slow, single-threaded CPU reference of the
 * row/column-sampling Monte Carlo estimator of f(sA) = sum_k c_k (sA)^k
 * (Guidotti, Acebron and Monteiro, "A fast Monte Carlo algorithm for
 * evaluating matrix functions with application in complex networks").
 *
 * TEST INFRASTRUCTURE.  This file exists to check the GPU library; it is
 * not part of the product.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark load it.  It shares no code, header or
 * table with the GPU library.  Build with -O2 -ffp-contract=off (no FMA
 * contraction) so that every floating-point step is the one written here.
 *
 * What it computes, in the paper's notation with B = sA:
 *
 *   Corollary 1:      f(B) = H + U,  H = c0 I + c1 B.
 *   Lemma 2:          U = E[Z], Z = sum_k c_{k+2} C_{X0} W^(k) R_{Xk}; the
 *                     Markov chain has transition t_ij = |b_ij| / sum_k |b_ik|
 *                     (Definition 1 (ii)) and W^(k) = W^(k-1) b/t.
 *   Section 3.2:      walks grouped by start column i give the matrix Q
 *                     (Eq. rand_funm_Q) and U_hat = B Q B (Eq. rand_funm_formula).
 *   Section 3.3:      d_i = c0 + c1 b_ii + sum_k b_ik <Q_k, C_i>
 *                     (Eq. rand_funm_formula_diag), one Q_k alive at a time.
 *   Section 3.4, Algorithm 3:
 *                     r = B v, q_i = (1/N_i) sum_walks sum_k c_{k+2} W r_{l_k},
 *                     y = c0 v + c1 r + B q (Eq. rand_funm_action_formula).
 *
 * Readings fixed for this implementation (the paper leaves them open):
 *   - K is the highest power kept.  A walk records the states t = 0..K-2
 *     (K-1 states, K-2 transitions), so that the expectation is exactly
 *     sum_{k<=K} c_k B^k.  W_0 = 1 and the 1/N of Algorithms 2-3 is applied
 *     once, at the end.
 *   - By default every start row k with deg(k) > 0 gets exactly N walks.
 *     With an allocation (oracle_allocation) start row k gets N_k walks,
 *     N_k = N_s P(l0 = k) rounded to the nearest integer as in Algorithms
 *     2-3; a row with N_k = 0 starts no walk and adds nothing to Q or q, so
 *     an output whose neighbourhood got no walks is exactly H (Section 4.1).
 *   - SelectNextState: a uniform 64-bit word u drives it.  An unweighted row
 *     (all stored values 1) takes index j = floor(u * deg / 2^64).  A
 *     weighted row takes the first j with u53 * rowabs < cum_j, where
 *     u53 = (u >> 11) * 2^-53, rowabs = sum_j |a_lj| and cum_j the running
 *     sum of |a_lj|, both summed left to right; j is clamped to deg-1.
 *   - Weighted rows, alias mode (oracle_set_alias): Walker's alias method
 *     with Vose's construction (Vose, IEEE TSE 17(9), 1991).  Per row of deg
 *     d: q_j = (|a_lj| * d) / rowabs; indices with q_j < 1 go on a "small"
 *     stack, the others on a "large" one, pushed in ascending j; while both
 *     are non-empty, pop s from small and g from large, set prob_s = q_s,
 *     alias_s = g, q_g = (q_g + q_s) - 1 and push g on small if q_g < 1,
 *     else on large; what is left on either stack gets prob 1 and itself as
 *     alias.  A row with rowabs = 0 gets prob 1 and itself everywhere.  A
 *     step takes i = floor(u * d / 2^64) and keeps i if u2_53 < prob_i,
 *     else alias_i, with u2 = X3 * 2^32 + X2 of the same Philox block and
 *     u2_53 = (u2 >> 11) * 2^-53.  P(next = j) = |a_lj| / rowabs as with
 *     the running sums; only the map from random words to j differs.
 *   - The weight update is W <- (W * (s * rowabs(l))), negated when the chosen
 *     entry is negative (b/t = s * sign(a) * rowabs).
 *   - A walk reaching a row with no entries stops (its remaining terms are
 *     exactly zero).
 *   - With a weight cutoff Wc > 0, a walk stops before recording step t as
 *     soon as |W_t| <= Wc (Eq. weight_cutoff with W^(0) = 1); K still caps it.
 *   - Random numbers: Philox4x32-10 (Salmon, Moraes, Dror and Shaw, SC'11)
 *     with counter (k, w, t, request) and key (seed low word, seed high
 *     word); the transition out of step t of walk w from start row k uses
 *     u = X1 * 2^32 + X0 of that block.
 *   - Path digest of start row k: the wrapping 64-bit sum over its walks of
 *     FNV-1a taken over the 32-bit words of the recorded states
 *     (h = 0xcbf29ce484222325; per state h = (h ^ state) * 0x100000001b3).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_E_ARG 1
#define ORC_E_NOT_SYMMETRIC 2
#define ORC_E_NOMEM 3

/* ------------------------------------------------------------------ */
/* Philox-4xW-10 (SC'11, Section 5): per round, two W-bit products       */
/* M0*x0 and M1*x2; the new words are (hi(M1 x2) ^ x1 ^ k0, lo(M1 x2),    */
/* hi(M0 x0) ^ x3 ^ k1, lo(M0 x0)); the key advances by the Weyl          */
/* constants (W0, W1) between rounds; 10 rounds.  One macro serves both   */
/* widths, so checking the 64-bit instance against an independent         */
/* Philox4x64-10 checks the round structure used at 32 bits as well.      */
/* ------------------------------------------------------------------ */

#define PHILOX4_10(UINT, WIDE, BITS, M0, M1, W0, W1, ctr, key, out)          \
    do {                                                                     \
        UINT x0 = (ctr)[0], x1 = (ctr)[1], x2 = (ctr)[2], x3 = (ctr)[3];     \
        UINT k0 = (key)[0], k1 = (key)[1];                                   \
        int round;                                                           \
        for (round = 0; round < 10; ++round) {                               \
            WIDE p0, p1;                                                     \
            UINT y0, y1, y2, y3;                                             \
            if (round > 0) {                                                 \
                k0 += (W0);                                                  \
                k1 += (W1);                                                  \
            }                                                                \
            p0 = (WIDE)(M0) * (WIDE)x0;                                      \
            p1 = (WIDE)(M1) * (WIDE)x2;                                      \
            y0 = (UINT)(p1 >> (BITS)) ^ x1 ^ k0;                             \
            y1 = (UINT)p1;                                                   \
            y2 = (UINT)(p0 >> (BITS)) ^ x3 ^ k1;                             \
            y3 = (UINT)p0;                                                   \
            x0 = y0; x1 = y1; x2 = y2; x3 = y3;                              \
        }                                                                    \
        (out)[0] = x0; (out)[1] = x1; (out)[2] = x2; (out)[3] = x3;          \
    } while (0)

void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    PHILOX4_10(uint32_t, uint64_t, 32, 0xD2511F53u, 0xCD9E8D57u, 0x9E3779B9u, 0xBB67AE85u,
               ctr, key, out);
}

/* The 64-bit instance; exported only so the round structure can be checked
 * against an independent library implementation of Philox4x64-10. */
void oracle_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4])
{
    PHILOX4_10(uint64_t, unsigned __int128, 64, 0xD2E7470EE14C6C93ull, 0xCA5A826395121157ull,
               0x9E3779B97F4A7C15ull, 0xBB67AE8584CAA73Bull, ctr, key, out);
}

/* floor(u * deg / 2^64): index in [0, deg) for an unweighted row. */
int64_t oracle_uniform_index(uint64_t u, int64_t deg)
{
    unsigned __int128 p = (unsigned __int128)u * (uint64_t)deg;
    return (int64_t)(p >> 64);
}

/* ------------------------------------------------------------------ */
/* Graph and per-row metadata                                          */
/* ------------------------------------------------------------------ */

typedef struct {
    int64_t n;
    const int64_t *row_ptr;
    const int32_t *col;
    const double *val; /* NULL: every stored entry is 1 */
    double *rowabs;    /* sum_j |a_lj|, left to right */
    double *cum;       /* running sums of |a_lj| per row (weighted only) */
    double *aprob;     /* alias mode, weighted only: prob_j per stored entry */
    int64_t *alias;    /* alias mode, weighted only: alias_j (index in the row) */
} ograph;

/* Alias mode for weighted rows (see the header); 0: running sums. */
static int g_alias_mode = 0;

void oracle_set_alias(int on)
{
    g_alias_mode = on ? 1 : 0;
}

typedef struct {
    const double *c; /* c_0 .. c_K */
    int K;
    double s;
    int64_t N;
    uint64_t seed;
    uint32_t request;
    double cutoff;
} oparams;

static double entry(const ograph *g, int64_t e)
{
    return g->val ? g->val[e] : 1.0;
}

/* Vose's construction for one row (entries [b, b + d)); stack is scratch of
 * d entries: "small" grows up from stack[0], "large" down from stack[d-1]. */
static void alias_row(const ograph *g, int64_t b, int64_t d, double W, int64_t *stack)
{
    int64_t j, ns = 0, nl = 0;
    double *q = g->aprob + b;
    int64_t *al = g->alias + b;
    if (!(W > 0.0)) {
        for (j = 0; j < d; ++j) {
            q[j] = 1.0;
            al[j] = j;
        }
        return;
    }
    for (j = 0; j < d; ++j) {
        q[j] = (fabs(entry(g, b + j)) * (double)d) / W;
        if (q[j] < 1.0)
            stack[ns++] = j;
        else
            stack[d - 1 - nl++] = j;
    }
    while (ns > 0 && nl > 0) {
        int64_t s = stack[--ns];
        int64_t big = stack[d - nl];
        --nl;
        al[s] = big; /* q[s] stays as prob_s */
        q[big] = (q[big] + q[s]) - 1.0;
        if (q[big] < 1.0)
            stack[ns++] = big;
        else
            stack[d - 1 - nl++] = big;
    }
    while (nl > 0) {
        int64_t big = stack[d - nl];
        --nl;
        q[big] = 1.0;
        al[big] = big;
    }
    while (ns > 0) {
        int64_t s = stack[--ns];
        q[s] = 1.0;
        al[s] = s;
    }
}

static int prepare(ograph *g)
{
    int64_t i, e;
    g->cum = NULL;
    g->aprob = NULL;
    g->alias = NULL;
    g->rowabs = (double *)malloc(sizeof(double) * (size_t)(g->n > 0 ? g->n : 1));
    if (!g->rowabs)
        return ORC_E_NOMEM;
    if (g->val) {
        g->cum = (double *)malloc(sizeof(double) * (size_t)(g->row_ptr[g->n] > 0 ? g->row_ptr[g->n] : 1));
        if (!g->cum)
            return ORC_E_NOMEM;
    }
    for (i = 0; i < g->n; ++i) {
        double sum = 0.0;
        for (e = g->row_ptr[i]; e < g->row_ptr[i + 1]; ++e) {
            sum = sum + fabs(entry(g, e));
            if (g->cum)
                g->cum[e] = sum;
        }
        g->rowabs[i] = sum;
    }
    if (g->val && g_alias_mode) {
        int64_t nnz = g->row_ptr[g->n], dmax = 0;
        int64_t *stack;
        g->aprob = (double *)malloc(sizeof(double) * (size_t)(nnz > 0 ? nnz : 1));
        g->alias = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nnz > 0 ? nnz : 1));
        for (i = 0; i < g->n; ++i)
            if (g->row_ptr[i + 1] - g->row_ptr[i] > dmax)
                dmax = g->row_ptr[i + 1] - g->row_ptr[i];
        stack = (int64_t *)malloc(sizeof(int64_t) * (size_t)(dmax > 0 ? dmax : 1));
        if (!g->aprob || !g->alias || !stack) {
            free(stack);
            return ORC_E_NOMEM;
        }
        for (i = 0; i < g->n; ++i)
            alias_row(g, g->row_ptr[i], g->row_ptr[i + 1] - g->row_ptr[i], g->rowabs[i], stack);
        free(stack);
    }
    return ORC_OK;
}

static void release(ograph *g)
{
    free(g->rowabs);
    free(g->cum);
    free(g->aprob);
    free(g->alias);
}

static int check_csr(int64_t n, const int64_t *row_ptr, const int32_t *col)
{
    int64_t i, e;
    if (n < 0 || !row_ptr || (n > 0 && !col && row_ptr[n] > 0))
        return ORC_E_ARG;
    if (row_ptr[0] != 0)
        return ORC_E_ARG;
    for (i = 0; i < n; ++i)
        if (row_ptr[i + 1] < row_ptr[i])
            return ORC_E_ARG;
    for (e = 0; e < row_ptr[n]; ++e)
        if (col[e] < 0 || col[e] >= n)
            return ORC_E_ARG;
    return ORC_OK;
}

/* Index of the next state inside row l (0 <= j < deg(l)), Definition 1 (ii).
 * u2 is the second random word (alias mode only). */
static int64_t select_next(const ograph *g, int64_t l, uint64_t u, uint64_t u2)
{
    int64_t deg = g->row_ptr[l + 1] - g->row_ptr[l];
    if (!g->val)
        return oracle_uniform_index(u, deg);
    if (g->aprob) {
        int64_t i = oracle_uniform_index(u, deg);
        double v53 = (double)(u2 >> 11) * 0x1p-53;
        return v53 < g->aprob[g->row_ptr[l] + i] ? i : g->alias[g->row_ptr[l] + i];
    }
    {
        double u53 = (double)(u >> 11) * 0x1p-53;
        double target = u53 * g->rowabs[l];
        int64_t j;
        for (j = 0; j < deg; ++j)
            if (target < g->cum[g->row_ptr[l] + j])
                return j;
        return deg - 1;
    }
}

int64_t oracle_select_next(int64_t n, const int64_t *row_ptr, const int32_t *col,
                           const double *val, int64_t l, uint64_t u, uint64_t u2)
{
    ograph g;
    int64_t j;
    g.n = n; g.row_ptr = row_ptr; g.col = col; g.val = val;
    if (l < 0 || l >= n || row_ptr[l + 1] == row_ptr[l])
        return -1;
    if (prepare(&g) != ORC_OK) {
        release(&g);
        return -1;
    }
    j = select_next(&g, l, u, u2);
    release(&g);
    return j;
}

/* Alias mode's tables of a weighted CSR (prob and alias per stored entry,
 * alias as an index inside the row).  Returns 0, or an ORC_E_* code. */
int oracle_alias_table(int64_t n, const int64_t *row_ptr, const int32_t *col, const double *val,
                       double *prob, int64_t *alias)
{
    ograph g;
    int64_t e, nnz;
    int rc, prev = g_alias_mode;
    if (!val || check_csr(n, row_ptr, col) != ORC_OK)
        return ORC_E_ARG;
    g.n = n; g.row_ptr = row_ptr; g.col = col; g.val = val;
    g_alias_mode = 1;
    rc = prepare(&g);
    g_alias_mode = prev;
    if (rc == ORC_OK) {
        nnz = row_ptr[n];
        for (e = 0; e < nnz; ++e) {
            prob[e] = g.aprob[e];
            alias[e] = g.alias[e];
        }
    }
    release(&g);
    return rc;
}

/* One walk from start row k (walk index w).  Records the visited states and
 * their weights W_t in st/wt, returns how many were recorded, and folds the
 * path into *digest.  Lemma 2 / Algorithms 2-3 with the readings above. */
static int walk(const ograph *g, const oparams *p, int64_t k, uint32_t w,
                int32_t *st, double *wt, uint64_t *digest)
{
    int64_t l = k;
    double W = 1.0;
    int cnt = 0, t;
    uint64_t h = 0xcbf29ce484222325ull;
    for (t = 0; t <= p->K - 2; ++t) {
        uint32_t ctr[4], key[2], x[4];
        uint64_t u;
        int64_t deg, e;
        double a;
        if (p->cutoff > 0.0 && !(fabs(W) > p->cutoff))
            break;
        st[cnt] = (int32_t)l;
        wt[cnt] = W;
        ++cnt;
        h = (h ^ (uint64_t)(uint32_t)l) * 0x100000001b3ull;
        if (t == p->K - 2)
            break;
        deg = g->row_ptr[l + 1] - g->row_ptr[l];
        if (deg == 0)
            break;
        ctr[0] = (uint32_t)k;
        ctr[1] = w;
        ctr[2] = (uint32_t)t;
        ctr[3] = p->request;
        key[0] = (uint32_t)(p->seed & 0xffffffffu);
        key[1] = (uint32_t)(p->seed >> 32);
        oracle_philox4x32_10(ctr, key, x);
        u = ((uint64_t)x[1] << 32) | (uint64_t)x[0];
        e = g->row_ptr[l] + select_next(g, l, u, ((uint64_t)x[3] << 32) | (uint64_t)x[2]);
        a = entry(g, e);
        W = W * (p->s * g->rowabs[l]);
        if (a < 0.0)
            W = -W;
        l = g->col[e];
    }
    *digest += h;
    return cnt;
}

/* Exact expectation of the recorded walk sums: rho_0 = e_k and
 * rho_{t+1}[j] = sum_l rho_t[l] * t_lj * (b_lj / t_lj) with the same
 * transition and weight factors as the sampler, so
 * sum_t c_{t+2} rho_t = E[sum_t c_{t+2} W_t e_{l_t}] = row k of
 * sum_t c_{t+2} B^t.  Adds that row into acc (dense, length n). */
static void expected_row(const ograph *g, const oparams *p, int64_t k,
                         double *rho, double *nxt, double *acc)
{
    int64_t i, e;
    int t;
    memset(rho, 0, sizeof(double) * (size_t)g->n);
    rho[k] = 1.0;
    for (t = 0; t <= p->K - 2; ++t) {
        for (i = 0; i < g->n; ++i)
            acc[i] += p->c[t + 2] * rho[i];
        if (t == p->K - 2)
            break;
        memset(nxt, 0, sizeof(double) * (size_t)g->n);
        for (i = 0; i < g->n; ++i) {
            if (rho[i] == 0.0 || g->rowabs[i] == 0.0)
                continue;
            for (e = g->row_ptr[i]; e < g->row_ptr[i + 1]; ++e) {
                double a = entry(g, e);
                double prob = fabs(a) / g->rowabs[i];
                double factor = p->s * g->rowabs[i];
                if (a < 0.0)
                    factor = -factor;
                nxt[g->col[e]] += rho[i] * prob * factor;
            }
        }
        memcpy(rho, nxt, sizeof(double) * (size_t)g->n);
    }
}

static int check_params(const oparams *p)
{
    int k;
    if (p->K < 0 || !p->c || !isfinite(p->s))
        return ORC_E_ARG;
    for (k = 0; k <= p->K; ++k)
        if (!isfinite(p->c[k]))
            return ORC_E_ARG;
    if (p->K >= 2 && p->N < 1)
        return ORC_E_ARG;
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* RandFunmAction (Section 3.4, Algorithm 3)                           */
/* ------------------------------------------------------------------ */

/*
 * y = c0 v + c1 r + B q with r = B v.
 * out_rows == NULL: every output row, walks from every row with deg > 0.
 * Otherwise y is produced only for out_rows[0..n_out) (into y[p]) and walks
 * start only from the rows that those outputs need: the union of their
 * neighbourhoods (the single-entry variant of Section 4.3).
 * mode 0: Monte Carlo; mode 1: exact expectation of the same estimator.
 * q_out (optional, length n): q_k per start row, 0 elsewhere.
 * digest (optional, length n): path digest per start row, 0 elsewhere.
 * steps (optional): number of recorded walk states.
 */
int oracle_action(int64_t n, const int64_t *row_ptr, const int32_t *col, const double *val,
                  const double *c, int K, double s, int64_t N, uint64_t seed, uint32_t request,
                  double cutoff, const double *v, const int32_t *out_rows, int64_t n_out,
                  int mode, double *y, double *q_out, uint64_t *digest, uint64_t *steps,
                  const int64_t *walks)
{
    ograph g;
    oparams p;
    double *r = NULL, *q = NULL, *rho = NULL, *nxt = NULL, *acc = NULL, *wt = NULL;
    int32_t *st = NULL;
    unsigned char *start = NULL;
    uint64_t nsteps = 0;
    int64_t i, e, k, pidx;
    int rc = check_csr(n, row_ptr, col);
    if (rc)
        return rc;
    if (!v || !y || (out_rows && n_out < 0))
        return ORC_E_ARG;
    p.c = c; p.K = K; p.s = s; p.N = N; p.seed = seed; p.request = request; p.cutoff = cutoff;
    if ((rc = check_params(&p)))
        return rc;
    if (out_rows)
        for (pidx = 0; pidx < n_out; ++pidx)
            if (out_rows[pidx] < 0 || out_rows[pidx] >= n)
                return ORC_E_ARG;
    g.n = n; g.row_ptr = row_ptr; g.col = col; g.val = val;
    if ((rc = prepare(&g)))
        goto done;
    rc = ORC_E_NOMEM;
    r = (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    q = (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    start = (unsigned char *)calloc((size_t)(n > 0 ? n : 1), 1);
    st = (int32_t *)malloc(sizeof(int32_t) * (size_t)(K > 1 ? K : 1));
    wt = (double *)malloc(sizeof(double) * (size_t)(K > 1 ? K : 1));
    if (!r || !q || !start || !st || !wt)
        goto done;
    if (mode == 1) {
        rho = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
        nxt = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
        acc = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
        if (!rho || !nxt || !acc)
            goto done;
    }
    rc = ORC_OK;

    /* r = B v = s A v, each row summed left to right. */
    for (i = 0; i < n; ++i) {
        double sum = 0.0;
        for (e = row_ptr[i]; e < row_ptr[i + 1]; ++e)
            sum = sum + entry(&g, e) * v[col[e]];
        r[i] = s * sum;
    }

    /* Start set. */
    if (K >= 2) {
        if (!out_rows) {
            for (k = 0; k < n; ++k)
                start[k] = row_ptr[k + 1] > row_ptr[k];
        } else {
            for (pidx = 0; pidx < n_out; ++pidx)
                for (e = row_ptr[out_rows[pidx]]; e < row_ptr[out_rows[pidx] + 1]; ++e)
                    start[col[e]] = 1;
            for (k = 0; k < n; ++k)
                if (row_ptr[k + 1] == row_ptr[k])
                    start[k] = 0;
        }
    }

    /* q_k = (1/N) sum_w sum_t c_{t+2} W_t r_{l_t}. */
    for (k = 0; k < n; ++k) {
        uint64_t dg = 0;
        if (!start[k])
            continue;
        if (mode == 0) {
            /* N walks from every start row, or walks[k] (Eq. initial_prob);
             * a row allocated no walk contributes q_k = 0. */
            const int64_t Nk = walks ? walks[k] : N;
            double sum = 0.0;
            uint32_t w;
            if (Nk < 0) {
                rc = ORC_E_ARG;
                goto done;
            }
            if (Nk == 0)
                continue;
            for (w = 0; w < (uint32_t)Nk; ++w) {
                int cnt = walk(&g, &p, k, w, st, wt, &dg), t;
                double a = 0.0;
                for (t = 0; t < cnt; ++t)
                    a = a + c[t + 2] * wt[t] * r[st[t]];
                sum = sum + a;
                nsteps += (uint64_t)cnt;
            }
            q[k] = sum / (double)Nk;
        } else {
            double sum = 0.0;
            memset(acc, 0, sizeof(double) * (size_t)n);
            expected_row(&g, &p, k, rho, nxt, acc);
            for (i = 0; i < n; ++i)
                sum = sum + acc[i] * r[i];
            q[k] = sum;
        }
        if (digest)
            digest[k] = dg;
    }

    /* y = c0 v + c1 r + B q. */
    {
        int64_t count = out_rows ? n_out : n;
        for (pidx = 0; pidx < count; ++pidx) {
            int64_t row = out_rows ? out_rows[pidx] : pidx;
            double yi = c[0] * v[row];
            if (K >= 1)
                yi = yi + c[1] * r[row];
            if (K >= 2) {
                double sum = 0.0;
                for (e = row_ptr[row]; e < row_ptr[row + 1]; ++e)
                    sum = sum + entry(&g, e) * q[col[e]];
                yi = yi + s * sum;
            }
            y[pidx] = yi;
        }
    }
    if (q_out)
        memcpy(q_out, q, sizeof(double) * (size_t)n);
    if (steps)
        *steps = nsteps;
done:
    release(&g);
    free(r); free(q); free(start); free(st); free(wt); free(rho); free(nxt); free(acc);
    return rc;
}

/* ------------------------------------------------------------------ */
/* RandFunmDiag (Section 3.3)                                          */
/* ------------------------------------------------------------------ */

static int cmp_u64(const void *a, const void *b)
{
    uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    return x < y ? -1 : (x > y ? 1 : 0);
}

/* 1 if A equals its transpose (pattern and values), 0 if not, <0 on OOM. */
int oracle_is_symmetric(int64_t n, const int64_t *row_ptr, const int32_t *col, const double *val)
{
    int64_t nnz = row_ptr[n], i, e;
    uint64_t *fwd, *bwd;
    int ok = 1;
    /* Each entry becomes (key, value-bits) pairs sorted by key, in both orientations. */
    fwd = (uint64_t *)malloc(sizeof(uint64_t) * 2 * (size_t)(nnz > 0 ? nnz : 1));
    bwd = (uint64_t *)malloc(sizeof(uint64_t) * 2 * (size_t)(nnz > 0 ? nnz : 1));
    if (!fwd || !bwd) {
        free(fwd); free(bwd);
        return -1;
    }
    for (i = 0; i < n; ++i)
        for (e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
            double a = val ? val[e] : 1.0;
            uint64_t bits;
            memcpy(&bits, &a, sizeof bits);
            fwd[2 * e] = (uint64_t)i * (uint64_t)n + (uint64_t)col[e];
            fwd[2 * e + 1] = bits;
            bwd[2 * e] = (uint64_t)col[e] * (uint64_t)n + (uint64_t)i;
            bwd[2 * e + 1] = bits;
        }
    qsort(fwd, (size_t)nnz, 2 * sizeof(uint64_t), cmp_u64);
    qsort(bwd, (size_t)nnz, 2 * sizeof(uint64_t), cmp_u64);
    for (e = 0; e < nnz && ok; ++e)
        if (fwd[2 * e] != bwd[2 * e] || fwd[2 * e + 1] != bwd[2 * e + 1])
            ok = 0;
    free(fwd); free(bwd);
    return ok;
}

/*
 * d_p = f(B)_{ii} estimate for i = rows[p] (rows == NULL: every row, n_rows
 * ignored and d has length n).  Start rows: every k with some b_ik != 0,
 * i in the requested set; Q_k is built from N walks, then used for every
 * requested i adjacent to k (Section 3.3) and dropped.
 * assume_symmetric = 0 checks that A = A^T first (C_i = R_i is needed).
 */
int oracle_diag(int64_t n, const int64_t *row_ptr, const int32_t *col, const double *val,
                const double *c, int K, double s, int64_t N, uint64_t seed, uint32_t request,
                double cutoff, const int32_t *rows, int64_t n_rows, int assume_symmetric,
                int mode, double *d, uint64_t *digest, uint64_t *steps, const int64_t *walks)
{
    ograph g;
    oparams p;
    double *Q = NULL, *dsum = NULL, *rho = NULL, *nxt = NULL, *wt = NULL;
    int32_t *st = NULL;
    int64_t *touched = NULL;
    unsigned char *inS = NULL, *start = NULL;
    uint64_t nsteps = 0;
    int64_t i, e, k, pidx, count, Nk = N;
    int rc = check_csr(n, row_ptr, col);
    if (rc)
        return rc;
    if (!d || (rows && n_rows < 0))
        return ORC_E_ARG;
    p.c = c; p.K = K; p.s = s; p.N = N; p.seed = seed; p.request = request; p.cutoff = cutoff;
    if ((rc = check_params(&p)))
        return rc;
    count = rows ? n_rows : n;
    if (rows)
        for (pidx = 0; pidx < n_rows; ++pidx)
            if (rows[pidx] < 0 || rows[pidx] >= n)
                return ORC_E_ARG;
    if (!assume_symmetric) {
        int sym = oracle_is_symmetric(n, row_ptr, col, val);
        if (sym < 0)
            return ORC_E_NOMEM;
        if (!sym)
            return ORC_E_NOT_SYMMETRIC;
    }
    g.n = n; g.row_ptr = row_ptr; g.col = col; g.val = val;
    if ((rc = prepare(&g)))
        goto done;
    rc = ORC_E_NOMEM;
    Q = (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    dsum = (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    inS = (unsigned char *)calloc((size_t)(n > 0 ? n : 1), 1);
    start = (unsigned char *)calloc((size_t)(n > 0 ? n : 1), 1);
    st = (int32_t *)malloc(sizeof(int32_t) * (size_t)(K > 1 ? K : 1));
    wt = (double *)malloc(sizeof(double) * (size_t)(K > 1 ? K : 1));
    if (!Q || !dsum || !inS || !start || !st || !wt)
        goto done;
    if (mode == 0 && K >= 2) {
        /* every state a start row's walks can visit, to clear Q_k afterwards */
        int64_t most = N;
        if (walks)
            for (k = 0; k < n; ++k)
                if (walks[k] > most)
                    most = walks[k];
        touched = (int64_t *)malloc(sizeof(int64_t) * (size_t)most * (size_t)(K - 1));
        if (!touched)
            goto done;
    }
    if (mode == 1) {
        rho = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
        nxt = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
        if (!rho || !nxt)
            goto done;
    }
    rc = ORC_OK;

    for (pidx = 0; pidx < count; ++pidx)
        inS[rows ? rows[pidx] : pidx] = 1;
    if (K >= 2)
        for (i = 0; i < n; ++i)
            if (inS[i])
                for (e = row_ptr[i]; e < row_ptr[i + 1]; ++e)
                    start[col[e]] = 1;

    for (k = 0; k < n; ++k) {
        uint64_t dg = 0;
        int64_t ntouched = 0;
        if (!start[k])
            continue;
        if (mode == 0) {
            uint32_t w;
            Nk = walks ? walks[k] : N;
            if (Nk < 0) {
                rc = ORC_E_ARG;
                goto done;
            }
            if (Nk == 0)
                continue; /* no walks: Q_k = 0 adds nothing */
            for (w = 0; w < (uint32_t)Nk; ++w) {
                int cnt = walk(&g, &p, k, w, st, wt, &dg), t;
                for (t = 0; t < cnt; ++t) {
                    Q[st[t]] = Q[st[t]] + c[t + 2] * wt[t];
                    touched[ntouched++] = st[t];
                }
                nsteps += (uint64_t)cnt;
            }
        } else {
            expected_row(&g, &p, k, rho, nxt, Q);
        }
        if (digest)
            digest[k] = dg;
        /* d_i += b_ik <Q_k, C_i> for every requested i adjacent to k; with
         * A symmetric, b_ik = b_ki and C_i is row i. */
        for (e = row_ptr[k]; e < row_ptr[k + 1]; ++e) {
            int64_t ii = col[e], e2;
            double inner = 0.0;
            if (!inS[ii])
                continue;
            for (e2 = row_ptr[ii]; e2 < row_ptr[ii + 1]; ++e2)
                inner = inner + entry(&g, e2) * Q[col[e2]];
            inner = s * inner;
            if (mode == 0)
                inner = inner / (double)Nk;
            dsum[ii] = dsum[ii] + (s * entry(&g, e)) * inner;
        }
        /* Drop Q_k. */
        if (mode == 0) {
            for (i = 0; i < ntouched; ++i)
                Q[touched[i]] = 0.0;
        } else {
            memset(Q, 0, sizeof(double) * (size_t)n);
        }
    }

    for (pidx = 0; pidx < count; ++pidx) {
        int64_t row = rows ? rows[pidx] : pidx;
        double di = c[0];
        if (K >= 1) {
            double aii = 0.0;
            for (e = row_ptr[row]; e < row_ptr[row + 1]; ++e)
                if (col[e] == row)
                    aii = entry(&g, e);
            di = di + c[1] * (s * aii);
        }
        if (K >= 2)
            di = di + dsum[row];
        d[pidx] = di;
    }
    if (steps)
        *steps = nsteps;
done:
    release(&g);
    free(Q); free(dsum); free(inS); free(start); free(touched); free(st); free(wt);
    free(rho); free(nxt);
    return rc;
}

/*
 * Walk allocation of Definition 1 (i) (Eq. initial_prob) with N_i = N_s p_i
 * as in Algorithms 2-3: p_k = ||C_k||_2 / sum over the start rows of ||C||_2
 * and N_k = round(N_s p_k), half away from zero.  N_k may be 0: Algorithms
 * 2-3 then run no walk from k (the regime of small N_s in Section 4.1).
 * min_one != 0 instead gives every start row at least one walk (a variant of
 * this library, not the paper's).  The column norms are summed in column
 * order: for symmetric A, C_k = R_k is summed along row k; otherwise
 * (unweighted only) ||C_k||^2 is the number of entries in column k.  The
 * total runs over starts[] in the order given.  walks_out[k] (length n) is
 * set for the start rows and 0 elsewhere.
 */
int oracle_allocation(int64_t n, const int64_t *row_ptr, const int32_t *col, const double *val,
                      int symmetric, const int32_t *starts, int64_t n_start, int64_t Ns,
                      int min_one, int64_t *walks_out)
{
    double *norm = NULL, total = 0.0;
    int64_t i, e;
    int rc = check_csr(n, row_ptr, col);
    if (rc)
        return rc;
    if (!walks_out || (n_start > 0 && !starts) || Ns < 1 || (!symmetric && val))
        return ORC_E_ARG;
    norm = (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    if (!norm)
        return ORC_E_NOMEM;
    if (symmetric) {
        for (i = 0; i < n; ++i) {
            double sq = 0.0;
            for (e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
                double a = val ? val[e] : 1.0;
                sq = sq + a * a;
            }
            norm[i] = sqrt(sq);
        }
    } else {
        for (e = 0; e < row_ptr[n]; ++e)
            norm[col[e]] = norm[col[e]] + 1.0;
        for (i = 0; i < n; ++i)
            norm[i] = sqrt(norm[i]);
    }
    memset(walks_out, 0, sizeof(int64_t) * (size_t)n);
    for (i = 0; i < n_start; ++i) {
        if (starts[i] < 0 || starts[i] >= n) {
            free(norm);
            return ORC_E_ARG;
        }
        total = total + norm[starts[i]];
    }
    for (i = 0; i < n_start; ++i) {
        const int64_t k = starts[i];
        int64_t w = total > 0.0 ? llround((double)Ns * (norm[k] / total)) : 0;
        if (min_one && w < 1)
            w = 1;
        walks_out[k] = w;
    }
    free(norm);
    return ORC_OK;
}

/* c_0..c_K: kind 0 exp (c_k = c_{k-1}/k), kind 1 resolvent (c_k = 1). */
int oracle_coeffs(int kind, int K, double *c)
{
    int k;
    if (K < 0 || !c)
        return ORC_E_ARG;
    if (kind == 0) {
        c[0] = 1.0;
        for (k = 1; k <= K; ++k)
            c[k] = c[k - 1] / (double)k;
    } else if (kind == 1) {
        for (k = 0; k <= K; ++k)
            c[k] = 1.0;
    } else {
        return ORC_E_ARG;
    }
    return ORC_OK;
}
