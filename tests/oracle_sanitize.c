/* Test driver, not oracle code: runs every oracle function on small graphs
 * so that a build with AddressSanitizer and UndefinedBehaviorSanitizer
 * (tests/test_oracle_sanitized.py) sees each of its code paths: a grid
 * (with a small count bit budget, so that levels are shifted), a random
 * directed graph with its reverse rows, and a complete graph. */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "centra_oracle.h"

typedef struct {
    uint32_t n;
    uint64_t m;
    uint32_t *row, *col, *rrow, *rcol;
} csr;

static int cmp_u64(const void *a, const void *b)
{
    const uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    return x < y ? -1 : x > y;
}

/* rows from (src << 32 | dst) keys, sorted and deduplicated */
static void build_rows(uint32_t n, uint64_t *keys, uint64_t m, uint32_t **row, uint32_t **col, uint64_t *out_m)
{
    qsort(keys, m, sizeof(uint64_t), cmp_u64);
    uint64_t u = 0;
    for (uint64_t i = 0; i < m; i++)
        if (i == 0 || keys[i] != keys[i - 1]) keys[u++] = keys[i];
    *row = calloc(n + 1, sizeof(uint32_t));
    *col = malloc(sizeof(uint32_t) * (u ? u : 1));
    for (uint64_t i = 0; i < u; i++) {
        (*row)[(keys[i] >> 32) + 1]++;
        (*col)[i] = (uint32_t)keys[i];
    }
    for (uint32_t v = 0; v < n; v++) (*row)[v + 1] += (*row)[v];
    *out_m = u;
}

static csr make(uint32_t n, const uint32_t *src, const uint32_t *dst, uint64_t m, int directed)
{
    csr g;
    memset(&g, 0, sizeof(g));
    g.n = n;
    uint64_t *k = malloc(sizeof(uint64_t) * 2 * (m ? m : 1)), c = 0;
    for (uint64_t i = 0; i < m; i++) {
        if (src[i] == dst[i]) continue;
        k[c++] = (uint64_t)src[i] << 32 | dst[i];
        if (!directed) k[c++] = (uint64_t)dst[i] << 32 | src[i];
    }
    build_rows(n, k, c, &g.row, &g.col, &g.m);
    if (directed) {
        c = 0;
        for (uint32_t v = 0; v < n; v++)
            for (uint32_t e = g.row[v]; e < g.row[v + 1]; e++) k[c++] = (uint64_t)g.col[e] << 32 | v;
        uint64_t mr;
        build_rows(n, k, c, &g.rrow, &g.rcol, &mr);
    }
    free(k);
    return g;
}

static orc_graph view(const csr *g, int directed)
{
    orc_graph o = {g->n, (uint32_t)directed, g->m, g->row, g->col, g->rrow, g->rcol};
    return o;
}

static int failures = 0;
#define CHECK(c)                                                        \
    do {                                                                \
        if (!(c)) {                                                     \
            fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
            failures++;                                                 \
        }                                                               \
    } while (0)

static void exercise(const orc_graph *g, uint32_t c_bits, int triangles)
{
    CHECK(orc_graph_check(g) == 0);
    const uint64_t count = 400;
    uint64_t *off = malloc(sizeof(uint64_t) * (count + 1));
    uint64_t cap = count * g->n;
    uint32_t *nodes = malloc(sizeof(uint32_t) * cap);
    orc_sample_info *info = malloc(sizeof(orc_sample_info) * count);
    CHECK(orc_sample_paths(g, c_bits, 3, 1, 100, count, off, nodes, cap, info) != UINT64_MAX);
    uint32_t *level = malloc(sizeof(uint32_t) * g->n);
    uint64_t *sigma = malloc(sizeof(uint64_t) * g->n);
    orc_bfs_counts(g, c_bits, 0, level, sigma);
    uint32_t picks[12];
    uint64_t cov[12];
    CHECK(orc_greedy_cover(g->n, count, off, nodes, 12, picks, cov) <= 12);
    int64_t *R = malloc(sizeof(int64_t) * g->n * 70);
    orc_rade_sums(g->n, count, off, nodes, 5, 0, 70, R);
    int64_t topk[70];
    uint64_t dk;
    uint32_t bm;
    orc_mcera(g->n, count, off, nodes, 5, 0, 70, 7, topk, &dk, &bm);
    orc_bound_out b;
    orc_bound(count, cov[0], topk[0], 70, dk, bm, 0.1, 0.05, &b);
    uint64_t *koff = malloc(sizeof(uint64_t) * (count + 1));
    uint32_t *knodes = malloc(sizeof(uint32_t) * count * 6);
    CHECK(orc_sample_kpaths(g, 6, 2, 0, 7, count, koff, knodes) == 0);
    for (uint32_t space = 0; space <= 3; space++) {
        if (space == 1 && !triangles) continue;
        for (uint32_t sched = 0; sched <= 2; sched++) {
            for (uint32_t method = 0; method <= 1; method++) {
                uint32_t p[5];
                orc_result res;
                uint64_t mlog[64];
                const int rc = orc_progressive(g, c_bits, 5, 9, 0.2, 0.1, 4, 0, 200, 3000, 2, 1, sched, space, 4,
                                               method, p, &res, mlog, 64);
                CHECK(rc == 0 || rc == 1);
            }
        }
    }
    {
        uint64_t boff[41];
        uint32_t bnodes[40 * 64];
        CHECK(orc_sample_paths_bidir(g, c_bits, orc_count_bits_out(g), 3, 1, 0, 40, boff, bnodes, 40 * 64, NULL) !=
              UINT64_MAX || g->n > 64);
    }
    if (triangles) {
        const uint64_t T = orc_triangles(g, NULL, 0);
        uint32_t *tri = malloc(sizeof(uint32_t) * 3 * (T ? T : 1));
        CHECK(orc_triangles(g, tri, T) == T);
        uint64_t rows = 0;
        for (uint32_t a = 0; a < g->n; a++) rows += orc_row_triangles(g, a, NULL, 0);
        CHECK(rows == T);
        uint64_t toff[51];
        uint32_t tn[150];
        if (T) CHECK(orc_sample_triangles(g, 1, 0, 0, 50, toff, tn) == 0);
        free(tri);
    }
    free(off); free(nodes); free(info); free(level); free(sigma); free(R); free(koff); free(knodes);
}

int main(void)
{
    /* grid 12 x 12 */
    const uint32_t L = 12;
    uint32_t src[2 * 12 * 12], dst[2 * 12 * 12];
    uint64_t m = 0;
    for (uint32_t r = 0; r < L; r++)
        for (uint32_t c = 0; c < L; c++) {
            if (c + 1 < L) { src[m] = r * L + c; dst[m++] = r * L + c + 1; }
            if (r + 1 < L) { src[m] = r * L + c; dst[m++] = (r + 1) * L + c; }
        }
    csr grid = make(L * L, src, dst, m, 0);
    orc_graph gg = view(&grid, 0);
    exercise(&gg, 8, 0);
    exercise(&gg, orc_count_bits(&gg), 0);
    CHECK(orc_triangles(&gg, NULL, 0) == 0);   /* bipartite */
    /* random directed graph, 200 nodes */
    uint32_t ds[1200], dd[1200];
    uint64_t x = 12345;
    for (int i = 0; i < 1200; i++) {
        x = x * 6364136223846793005ULL + 1442695040888963407ULL;
        ds[i] = (uint32_t)(x >> 33) % 200;
        x = x * 6364136223846793005ULL + 1442695040888963407ULL;
        dd[i] = (uint32_t)(x >> 33) % 200;
    }
    csr dir = make(200, ds, dd, 1200, 1);
    orc_graph dg = view(&dir, 1);
    exercise(&dg, orc_count_bits(&dg), 0);
    CHECK(orc_triangles(&dg, NULL, 0) == UINT64_MAX);
    /* complete graph on 8 nodes */
    uint32_t ks[28], kd[28];
    uint64_t km = 0;
    for (uint32_t a = 0; a < 8; a++)
        for (uint32_t b = a + 1; b < 8; b++) { ks[km] = a; kd[km++] = b; }
    csr kg = make(8, ks, kd, km, 0);
    orc_graph kv = view(&kg, 0);
    exercise(&kv, orc_count_bits(&kv), 1);
    uint32_t d1;
    uint64_t dl, du;
    CHECK(orc_vc_dims(3, 50, 1000000, &d1, &dl, &du) == 0 && d1 == 2);
    CHECK(orc_vc_dims(0, 1, 1, &d1, &dl, &du) == -1);
    CHECK(orc_next_sample_size(1000, 0.3, 0.05, 0.01, 6, 5, 100000, 1) >= 1200);
    free(grid.row); free(grid.col); free(dir.row); free(dir.col); free(dir.rrow); free(dir.rcol);
    free(kg.row); free(kg.col);
    printf("sanitized oracle run: %d failed checks\n", failures);
    return failures ? 1 : 0;
}
