/*
 * graphgen.c -- seeded synthetic inputs: graphs in CSR form and synthetic
 * hyperedge sets.
 *
 * These are workload generators only: they stand in for the SNAP / KONECT
 * graphs of the paper's experiments (Sec. 5, graph table in the appendix),
 * which are not available here.  They use their own generator (SplitMix64,
 * Steele, Lea and Flood, OOPSLA 2014), hold none of the method's arithmetic,
 * and serve the HIP path and the oracle alike.
 *
 * Every graph is returned as CSR with rows sorted ascending, without
 * duplicate arcs or self loops.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;

static uint64_t splitmix64(uint64_t *x)
{
    uint64_t z = (*x += 0x9E3779B97F4A7C15ULL);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

static uint64_t below(uint64_t *x, uint64_t bound)
{
    return (uint64_t)(((u128)splitmix64(x) * bound) >> 64);
}

static double unit(uint64_t *x)
{
    return (double)(splitmix64(x) >> 11) * 0x1.0p-53;
}

static int cmp_u32(const void *a, const void *b)
{
    uint32_t x = *(const uint32_t *)a, y = *(const uint32_t *)b;
    return x < y ? -1 : (x > y);
}

/* Builds a CSR from an arc list (src[i] -> dst[i]); drops self loops and
 * duplicate arcs.  row_ptr has n+1 entries, col_idx capacity n_in.  Returns
 * the number of arcs kept. */
static uint64_t build_csr(uint32_t n, uint64_t n_in, const uint32_t *src, const uint32_t *dst,
                          uint32_t *row_ptr, uint32_t *col_idx)
{
    uint64_t *cnt = calloc((size_t)n + 1, sizeof(uint64_t));
    for (uint64_t i = 0; i < n_in; i++)
        if (src[i] != dst[i]) cnt[src[i] + 1]++;
    for (uint32_t u = 0; u < n; u++) cnt[u + 1] += cnt[u];
    uint64_t *pos = malloc(sizeof(uint64_t) * ((size_t)n + 1));
    memcpy(pos, cnt, sizeof(uint64_t) * ((size_t)n + 1));
    for (uint64_t i = 0; i < n_in; i++)
        if (src[i] != dst[i]) col_idx[pos[src[i]]++] = dst[i];
    uint64_t out = 0;
    row_ptr[0] = 0;
    for (uint32_t u = 0; u < n; u++) {
        uint64_t b = cnt[u], e = cnt[u + 1];
        qsort(col_idx + b, e - b, sizeof(uint32_t), cmp_u32);
        for (uint64_t i = b; i < e; i++)
            if (i == b || col_idx[i] != col_idx[i - 1]) col_idx[out++] = col_idx[i];
        row_ptr[u + 1] = (uint32_t)out;
    }
    free(cnt);
    free(pos);
    return out;
}

/* Number of arcs of gg_ba(n, m0, .): an (m0+1)-clique plus m0 edges per
 * later node, each edge stored as two arcs. */
uint64_t gg_ba_arcs(uint32_t n, uint32_t m0)
{
    return 2ull * ((uint64_t)m0 * (m0 + 1) / 2 + (uint64_t)(n - m0 - 1) * m0);
}

/* Barabasi-Albert preferential attachment: a clique on nodes 0..m0, then
 * each node v > m0 joins m0 distinct earlier nodes chosen with probability
 * proportional to degree (uniform draws from the list of arc endpoints,
 * repeats redrawn).  Undirected.  Returns the number of arcs. */
uint64_t gg_ba(uint32_t n, uint32_t m0, uint64_t seed, uint32_t *row_ptr, uint32_t *col_idx)
{
    if (m0 < 1 || n <= m0 + 1) return 0;
    uint64_t rng = seed;
    uint64_t n_edges = gg_ba_arcs(n, m0) / 2;
    uint32_t *ends = malloc(sizeof(uint32_t) * 2 * n_edges);
    uint64_t ne = 0;
    for (uint32_t a = 0; a <= m0; a++)
        for (uint32_t b = a + 1; b <= m0; b++) {
            ends[2 * ne] = a;
            ends[2 * ne + 1] = b;
            ne++;
        }
    uint32_t *pick = malloc(sizeof(uint32_t) * m0);
    for (uint32_t v = m0 + 1; v < n; v++) {
        uint32_t got = 0;
        uint64_t pool = 2 * ne;
        while (got < m0) {
            uint32_t x = ends[below(&rng, pool)];
            int dup = 0;
            for (uint32_t q = 0; q < got; q++) dup |= pick[q] == x;
            if (!dup) pick[got++] = x;
        }
        for (uint32_t q = 0; q < m0; q++) {
            ends[2 * ne] = v;
            ends[2 * ne + 1] = pick[q];
            ne++;
        }
    }
    free(pick);
    uint32_t *src = malloc(sizeof(uint32_t) * 4 * ne), *dst = malloc(sizeof(uint32_t) * 4 * ne);
    for (uint64_t i = 0; i < ne; i++) {
        src[2 * i] = ends[2 * i];     dst[2 * i] = ends[2 * i + 1];
        src[2 * i + 1] = ends[2 * i + 1]; dst[2 * i + 1] = ends[2 * i];
    }
    free(ends);
    uint64_t arcs = build_csr(n, 2 * ne, src, dst, row_ptr, col_idx);
    free(src);
    free(dst);
    return arcs;
}

/* L x L 4-neighbour grid, node id r*L + c, undirected: 4L(L-1) arcs. */
uint64_t gg_grid(uint32_t L, uint32_t *row_ptr, uint32_t *col_idx)
{
    uint64_t out = 0;
    row_ptr[0] = 0;
    for (uint32_t r = 0; r < L; r++)
        for (uint32_t c = 0; c < L; c++) {
            uint32_t id = r * L + c;
            /* ascending neighbour ids: up, left, right, down */
            if (r > 0) col_idx[out++] = id - L;
            if (c > 0) col_idx[out++] = id - 1;
            if (c + 1 < L) col_idx[out++] = id + 1;
            if (r + 1 < L) col_idx[out++] = id + L;
            row_ptr[id + 1] = (uint32_t)out;
        }
    return out;
}

/* R-MAT (Chakrabarti, Zhan, Faloutsos, SDM 2004): edge_factor * 2^scale arc
 * draws, each descending `scale` quadrant levels with probabilities
 * (a, b, c, 1-a-b-c); node labels are shuffled with a seeded permutation;
 * self loops and duplicates are dropped.  Directed.  row_ptr/col_idx get the
 * out-arcs; capacity edge_factor * 2^scale.  Returns the number of arcs. */
uint64_t gg_rmat(uint32_t scale, uint32_t edge_factor, double a, double b, double c,
                 uint64_t seed, uint32_t *row_ptr, uint32_t *col_idx)
{
    uint32_t n = 1u << scale;
    uint64_t draws = (uint64_t)edge_factor << scale;
    uint64_t rng = seed;
    uint32_t *perm = malloc(sizeof(uint32_t) * n);
    for (uint32_t i = 0; i < n; i++) perm[i] = i;
    for (uint32_t i = n - 1; i > 0; i--) {
        uint32_t j = (uint32_t)below(&rng, (uint64_t)i + 1);
        uint32_t tmp = perm[i]; perm[i] = perm[j]; perm[j] = tmp;
    }
    uint32_t *src = malloc(sizeof(uint32_t) * draws), *dst = malloc(sizeof(uint32_t) * draws);
    const double ab = a + b, abc = a + b + c;
    for (uint64_t i = 0; i < draws; i++) {
        uint32_t u = 0, v = 0;
        for (uint32_t lev = 0; lev < scale; lev++) {
            double x = unit(&rng);
            u <<= 1; v <<= 1;
            if (x < a) {
            } else if (x < ab) {
                v |= 1;
            } else if (x < abc) {
                u |= 1;
            } else {
                u |= 1; v |= 1;
            }
        }
        src[i] = perm[u];
        dst[i] = perm[v];
    }
    free(perm);
    uint64_t arcs = build_csr(n, draws, src, dst, row_ptr, col_idx);
    free(src);
    free(dst);
    return arcs;
}

/* Reverse CSR: rrow_ptr/rcol_idx list the in-neighbours of each node,
 * ascending. */
void gg_reverse(uint32_t n, const uint32_t *row_ptr, const uint32_t *col_idx,
                uint32_t *rrow_ptr, uint32_t *rcol_idx)
{
    uint64_t arcs = row_ptr[n];
    memset(rrow_ptr, 0, sizeof(uint32_t) * ((size_t)n + 1));
    for (uint64_t e = 0; e < arcs; e++) rrow_ptr[col_idx[e] + 1]++;
    for (uint32_t v = 0; v < n; v++) rrow_ptr[v + 1] += rrow_ptr[v];
    uint32_t *pos = malloc(sizeof(uint32_t) * ((size_t)n + 1));
    memcpy(pos, rrow_ptr, sizeof(uint32_t) * ((size_t)n + 1));
    /* sources visited in ascending order, so every in-row comes out sorted */
    for (uint32_t u = 0; u < n; u++)
        for (uint32_t e = row_ptr[u]; e < row_ptr[u + 1]; e++)
            rcol_idx[pos[col_idx[e]]++] = u;
    free(pos);
}

/* Synthetic hyperedge set shaped like shortest-path samples on a scale-free
 * graph: m hyperedges, lengths uniform in [0, max_len], nodes distinct
 * within a hyperedge, node popularity skewed towards low ids (id =
 * floor(n * U^skew), skew a positive integer).  he_off has m+1 entries; he_nodes capacity
 * m * max_len.  Returns the total number of nodes. */
uint64_t gg_hyperedges(uint32_t n, uint64_t m, uint32_t max_len, uint32_t skew, uint64_t seed,
                       uint64_t *he_off, uint32_t *he_nodes)
{
    uint64_t rng = seed;
    uint64_t total = 0;
    he_off[0] = 0;
    for (uint64_t s = 0; s < m; s++) {
        uint32_t len = (uint32_t)below(&rng, (uint64_t)max_len + 1);
        if (len > n) len = n;
        uint32_t got = 0;
        while (got < len) {
            double x = unit(&rng);
            double p = x;
            for (uint32_t q = 1; q < skew; q++) p *= x;
            uint32_t u = (uint32_t)(p * n);
            if (u >= n) u = n - 1;
            int dup = 0;
            for (uint32_t q = 0; q < got; q++) dup |= he_nodes[total + q] == u;
            if (!dup) he_nodes[total + got++] = u;
        }
        total += len;
        he_off[s + 1] = total;
    }
    return total;
}
