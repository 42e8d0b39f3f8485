/* Barabasi-Albert preferential attachment, edge list only.
 *
 * Seed graph: the complete graph on m+1 nodes.  Each later node v joins m
 * distinct earlier nodes; each target is drawn uniformly from the list of
 * edge endpoints created so far (so a node is picked with probability
 * proportional to its degree), and a target already chosen for v is drawn
 * again.  Random numbers come from splitmix64 (Steele, Lea and Flood,
 * OOPSLA 2014) seeded with `seed`; an index below `len` is the high word of
 * the 128-bit product of a 64-bit draw and `len`.
 */
#include <stdint.h>
#include <stdlib.h>

static uint64_t sm64(uint64_t *s)
{
    uint64_t z = (*s += 0x9e3779b97f4a7c15ULL);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

/* Writes the undirected edges (src[e], dst[e]) and returns their count, or
 * -1 on bad arguments / allocation failure.  Capacity needed:
 * m(m+1)/2 + (n-m-1)m edges. */
int64_t graphgen_ba_edges(int64_t n, int32_t m, uint64_t seed, int32_t *src, int32_t *dst)
{
    if (m < 1 || n < m + 1)
        return -1;
    int64_t cap = (int64_t)m * (m + 1) / 2 + (n - m - 1) * (int64_t)m;
    int32_t *ends = (int32_t *)malloc(sizeof(int32_t) * 2 * (size_t)cap);
    if (!ends)
        return -1;
    int64_t ne = 0, nend = 0;
    for (int32_t i = 0; i <= m; ++i)
        for (int32_t j = i + 1; j <= m; ++j) {
            src[ne] = i; dst[ne] = j; ++ne;
            ends[nend++] = i; ends[nend++] = j;
        }
    uint64_t state = seed;
    int32_t *pick = (int32_t *)malloc(sizeof(int32_t) * (size_t)m);
    if (!pick) { free(ends); return -1; }
    for (int64_t v = m + 1; v < n; ++v) {
        int32_t got = 0;
        while (got < m) {
            uint64_t u = sm64(&state);
            uint64_t idx = (uint64_t)(((unsigned __int128)u * (uint64_t)nend) >> 64);
            int32_t t = ends[idx];
            int dup = 0;
            for (int32_t q = 0; q < got; ++q)
                if (pick[q] == t) { dup = 1; break; }
            if (!dup)
                pick[got++] = t;
        }
        for (int32_t q = 0; q < m; ++q) {
            src[ne] = (int32_t)v; dst[ne] = pick[q]; ++ne;
            ends[nend++] = (int32_t)v; ends[nend++] = pick[q];
        }
    }
    free(pick);
    free(ends);
    return ne;
}
