/* R-MAT graphs (Chakrabarti, Zhan and Faloutsos, SDM 2004) straight to CSR,
 * for graphs too large for the numpy generator (2^26 nodes, 2^30 edge draws).
 *
 * Edge e of m = edge_factor * 2^scale descends `scale` levels; at each level
 * a 32-bit uniform u picks quadrant (0,0) if u < a, (0,1) if u < a+b, (1,0)
 * if u < a+b+c, else (1,1) (thresholds scaled to 2^32); level l sets bit l
 * of the source and destination.  Vertices are relabelled by a random
 * permutation (Fisher-Yates), loops are dropped, every edge is stored in
 * both directions and duplicates are removed; isolated vertices are kept.
 *
 * Random numbers: splitmix64 (Steele, Lea and Flood, OOPSLA 2014).  Edge e
 * draws from its own stream, started at the splitmix64 finaliser of
 * (seed ^ finaliser(e + 1)), so the graph does not depend on the thread count.
 * The permutation draws from the stream seeded with ~seed; an index below k
 * is the high word of the 128-bit product of a draw and k.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

static uint64_t sm64(uint64_t *s)
{
    return mix64(*s += 0x9e3779b97f4a7c15ULL);
}

static int cmp_i32(const void *x, const void *y)
{
    const int32_t a = *(const int32_t *)x, b = *(const int32_t *)y;
    return (a > b) - (a < b);
}

/* Edge e's endpoints before relabelling. */
static void draw_edge(uint64_t seed, int64_t e, int scale, uint32_t ta, uint32_t tab, uint32_t tabc,
                      uint32_t *src, uint32_t *dst)
{
    uint64_t s = mix64(seed ^ mix64((uint64_t)e + 1));
    uint32_t u = 0, v = 0;
    uint64_t r = 0;
    for (int level = 0; level < scale; ++level) {
        if ((level & 1) == 0)
            r = sm64(&s);
        const uint32_t x = (level & 1) ? (uint32_t)(r >> 32) : (uint32_t)r;
        const uint32_t sb = x >= tab;                              /* rows of quadrants (1,*) */
        const uint32_t db = (x >= ta && x < tab) || x >= tabc;     /* columns of (*,1) */
        u |= sb << level;
        v |= db << level;
    }
    *src = u;
    *dst = v;
}

/* Builds the CSR.  row_ptr: int64[2^scale + 1] (caller's); col: int32 of
 * capacity 2 * edge_factor * 2^scale (caller's), of which the first nnz hold
 * the columns, ascending within each row.  Returns nnz, or -1 on bad
 * arguments or allocation failure. */
int64_t graphgen_rmat_csr(int32_t scale, int32_t edge_factor, double a, double b, double c,
                          uint64_t seed, int32_t permute, int64_t *row_ptr, int32_t *col)
{
    if (scale < 1 || scale > 30 || edge_factor < 1 || a < 0 || b < 0 || c < 0 || a + b + c > 1.0)
        return -1;
    const int64_t n = (int64_t)1 << scale;
    const int64_t m = (int64_t)edge_factor * n;
    const double two32 = 4294967296.0;
    const double fa = a * two32, fab = (a + b) * two32, fabc = (a + b + c) * two32;
    const uint32_t ta = fa >= two32 ? 0xffffffffu : (uint32_t)fa;
    const uint32_t tab = fab >= two32 ? 0xffffffffu : (uint32_t)fab;
    const uint32_t tabc = fabc >= two32 ? 0xffffffffu : (uint32_t)fabc;

    uint32_t *perm = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)n);
    int64_t *cursor = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    if (!perm || !cursor) {
        free(perm);
        free(cursor);
        return -1;
    }
    for (int64_t i = 0; i < n; ++i)
        perm[i] = (uint32_t)i;
    if (permute) {
        uint64_t ps = ~seed;
        for (int64_t i = n - 1; i > 0; --i) {
            const uint64_t j = (uint64_t)(((unsigned __int128)sm64(&ps) * (uint64_t)(i + 1)) >> 64);
            const uint32_t t = perm[i];
            perm[i] = perm[j];
            perm[j] = t;
        }
    }
    /* Pass 1: entries per row (both directions, loops dropped). */
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < m; ++e) {
        uint32_t u, v;
        draw_edge(seed, e, scale, ta, tab, tabc, &u, &v);
        if (u == v)
            continue;
        __atomic_fetch_add(&cursor[perm[u] + 1], 1, __ATOMIC_RELAXED);
        __atomic_fetch_add(&cursor[perm[v] + 1], 1, __ATOMIC_RELAXED);
    }
    for (int64_t i = 0; i < n; ++i)
        cursor[i + 1] += cursor[i];
    memcpy(row_ptr, cursor, sizeof(int64_t) * (size_t)(n + 1));
    /* Pass 2: scatter (the same draws again), order within a row arbitrary. */
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < m; ++e) {
        uint32_t u, v;
        draw_edge(seed, e, scale, ta, tab, tabc, &u, &v);
        if (u == v)
            continue;
        const uint32_t pu = perm[u], pv = perm[v];
        col[__atomic_fetch_add(&cursor[pu], 1, __ATOMIC_RELAXED)] = (int32_t)pv;
        col[__atomic_fetch_add(&cursor[pv], 1, __ATOMIC_RELAXED)] = (int32_t)pu;
    }
    /* Sort and deduplicate each row; cursor[i] becomes its distinct count. */
#pragma omp parallel for schedule(dynamic, 4096)
    for (int64_t i = 0; i < n; ++i) {
        int32_t *r = col + row_ptr[i];
        const int64_t len = row_ptr[i + 1] - row_ptr[i];
        if (len > 1)
            qsort(r, (size_t)len, sizeof(int32_t), cmp_i32);
        int64_t k = 0;
        for (int64_t j = 0; j < len; ++j)
            if (k == 0 || r[j] != r[k - 1])
                r[k++] = r[j];
        cursor[i] = k;
    }
    /* Compact the rows in order (a row never moves right). */
    int64_t nnz = 0;
    for (int64_t i = 0; i < n; ++i) {
        const int64_t start = row_ptr[i], k = cursor[i];
        if (start != nnz)
            memmove(col + nnz, col + start, sizeof(int32_t) * (size_t)k);
        row_ptr[i] = nnz;
        nnz += k;
    }
    row_ptr[n] = nnz;
    free(perm);
    free(cursor);
    return nnz;
}
