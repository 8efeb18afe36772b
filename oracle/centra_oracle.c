/*
 * centra_oracle.c -- plain, slow CPU oracle for the CentRA hot path.
 *
 * TEST INFRASTRUCTURE ONLY: used by tests/, the smoke check and the
 * benchmark's CPU-baseline leg.  Shares no code with the HIP path.
 *
 * Paper: L. Pellegrina, "Efficient Centrality Maximization with Rademacher
 * Averages", KDD 2023 (arXiv 2306.03651).  Section / theorem / algorithm
 * references below are to that paper.  Readings of points it leaves open:
 *
 *  R1  Randomness.  The paper fixes no generator.  All draws come from
 *      Philox4x64-10 (Salmon et al., SC'11) with key (seed, 0) and counter
 *      (block, sample index, instance, tag); tag 0 = path sampling, tag 1 =
 *      Rademacher signs.  The sample index is global, so the sample of
 *      iteration i extends the sample of iteration i-1 exactly (Algorithm 1,
 *      H_i = H_{i-1} plus new hyperedges).
 *  R2  Bounded draws use Lemire's multiply-and-reject method (TOMACS 2019).
 *  R3  The pair is an ordered uniform pair s != t (Sec. 3.1 defines the
 *      hyperedge space over all pairs u != v; Sec. 5 draws the endpoints
 *      uniformly).
 *  R4  Shortest-path counts are kept as normalised integers: level by level,
 *      the raw count of a node is the sum of its predecessors' normalised
 *      counts; if the largest raw count of the level needs more than C bits
 *      (C = 63 - bitlen(max in-degree)), every count of that level is shifted
 *      right by the excess, and clamped to at least 1.  While no level
 *      exceeds 2^C the counts are exact.  (The paper samples a uniform
 *      shortest path but does not say how counts are represented.)
 *  R5  A single BFS from s followed by a backtrack from t replaces the
 *      balanced bidirectional BFS of Sec. 5: the same distribution over
 *      shortest paths, different random bits.
 *  R6  Backtracking visits predecessors in ascending node id and always
 *      draws, even when there is one predecessor.  An unreachable t, or t
 *      adjacent to s, gives the empty hyperedge with no draws (Sec. 5: an
 *      unreachable target gives the empty set; Sec. 3.1: only internal nodes
 *      belong to the hyperedge).
 *  R7  greedyCover breaks ties by lowest node id and stops early when the
 *      best marginal gain is 0 (|S| <= k is allowed by the problem statement).
 *  R8  sigma is extended column by column instead of redrawn each iteration
 *      (Sec. 4.2 remark on incremental computation); sigma_js = +1 iff bit
 *      (j mod 64) of word ((j mod 256) div 64) of Philox block
 *      (j div 256, s, instance, 1) is set.
 *  R9  The sup over |S'| <= k of sum_{u in S'} r_j^u is the sum of the
 *      min(k, #positive) largest positive values (S' = empty is allowed).
 *  R10 Iterations count from i = 1 with delta_i = delta / 2^i (Algorithm 1),
 *      ln is the natural log, and the schedule is geometric with a cap m_max.
 */
#include "centra_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;

#define UNSEEN 0xFFFFFFFFu

/* ------------------------------------------------------------------ */
/* Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11, Sec. 3.4): ten rounds
 * of two 64x64->128 multiplications with the published multipliers and a
 * Weyl sequence on the key. */
void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4])
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
    uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; round++) {
        u128 p0 = (u128)M0 * x0;
        u128 p1 = (u128)M1 * x2;
        uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        x0 = hi1 ^ x1 ^ k0;
        x1 = lo1;
        x2 = hi0 ^ x3 ^ k1;
        x3 = lo0;
        k0 += W0;
        k1 += W1;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

void orc_stream_init(orc_stream *st, uint64_t seed, uint64_t c1, uint64_t c2, uint64_t c3)
{
    st->key[0] = seed;
    st->key[1] = 0;
    st->ctr[0] = 0;
    st->ctr[1] = c1;
    st->ctr[2] = c2;
    st->ctr[3] = c3;
    st->pos = 4;
}

uint64_t orc_stream_next(orc_stream *st)
{
    if (st->pos == 4) {
        orc_philox4x64_10(st->ctr, st->key, st->buf);
        st->ctr[0] += 1;
        st->pos = 0;
    }
    return st->buf[st->pos++];
}

/* Lemire, "Fast random integer generation in an interval", TOMACS 2019,
 * Algorithm 5: multiply a 64-bit word by W, keep the high half, and reject
 * the low half if it falls below (2^64 - W) mod W. */
uint64_t orc_bounded(orc_stream *st, uint64_t W)
{
    uint64_t x = orc_stream_next(st);
    u128 p = (u128)x * W;
    uint64_t low = (uint64_t)p;
    if (low < W) {
        uint64_t threshold = (0 - W) % W;
        while (low < threshold) {
            x = orc_stream_next(st);
            p = (u128)x * W;
            low = (uint64_t)p;
        }
    }
    return (uint64_t)(p >> 64);
}

void orc_bounded_many(uint64_t seed, uint64_t c1, uint64_t c2, uint64_t c3,
                      uint64_t W, uint64_t count, uint64_t *out)
{
    orc_stream st;
    orc_stream_init(&st, seed, c1, c2, c3);
    for (uint64_t i = 0; i < count; i++)
        out[i] = orc_bounded(&st, W);
}

/* ------------------------------------------------------------------ */
/* Graph helpers. */

static const uint32_t *in_ptr(const orc_graph *g) { return g->directed ? g->rrow_ptr : g->row_ptr; }
static const uint32_t *in_idx(const orc_graph *g) { return g->directed ? g->rcol_idx : g->col_idx; }

static int check_rows(uint32_t n, uint64_t n_arcs, const uint32_t *ptr, const uint32_t *idx)
{
    if (!ptr || !idx) return -2;
    if (ptr[0] != 0 || ptr[n] != n_arcs) return -3;
    for (uint32_t u = 0; u < n; u++) {
        if (ptr[u + 1] < ptr[u]) return -4;
        for (uint32_t e = ptr[u]; e < ptr[u + 1]; e++) {
            if (idx[e] >= n) return -5;
            if (idx[e] == u) return -6;
            if (e > ptr[u] && idx[e] <= idx[e - 1]) return -7;
        }
    }
    return 0;
}

int orc_graph_check(const orc_graph *g)
{
    if (g->n < 2) return -1;
    int rc = check_rows(g->n, g->n_arcs, g->row_ptr, g->col_idx);
    if (rc) return rc;
    if (g->directed) {
        rc = check_rows(g->n, g->n_arcs, g->rrow_ptr, g->rcol_idx);
        if (rc) return rc - 10;
        /* the reverse rows hold exactly the reversed arcs */
        uint64_t *cnt = calloc(g->n, sizeof(uint64_t));
        for (uint32_t u = 0; u < g->n; u++)
            for (uint32_t e = g->row_ptr[u]; e < g->row_ptr[u + 1]; e++)
                cnt[g->col_idx[e]]++;
        for (uint32_t v = 0; v < g->n; v++)
            if (cnt[v] != (uint64_t)(g->rrow_ptr[v + 1] - g->rrow_ptr[v])) { free(cnt); return -20; }
        free(cnt);
        /* with equal row sizes and no duplicates, every arc u -> v having u
         * in v's reverse row makes the reverse rows the reversed arcs */
        for (uint32_t u = 0; u < g->n; u++)
            for (uint32_t e = g->row_ptr[u]; e < g->row_ptr[u + 1]; e++) {
                const uint32_t v = g->col_idx[e];
                int found = 0;
                for (uint32_t f = g->rrow_ptr[v]; f < g->rrow_ptr[v + 1]; f++)
                    if (g->rcol_idx[f] == u) { found = 1; break; }
                if (!found) return -21;
            }
    }
    return 0;
}

static uint32_t bitlen64(uint64_t x)
{
    uint32_t b = 0;
    while (x) { b++; x >>= 1; }
    return b;
}

uint32_t orc_count_bits(const orc_graph *g)
{
    const uint32_t *ip = in_ptr(g);
    uint64_t dmax = 0;
    for (uint32_t v = 0; v < g->n; v++) {
        uint64_t d = ip[v + 1] - ip[v];
        if (d > dmax) dmax = d;
    }
    return 63 - bitlen64(dmax);
}

/* ------------------------------------------------------------------ */
/* BFS with normalised counts (reading R4).  Expands whole levels from s
 * until `stop` has a level, or the graph is exhausted if stop == UNSEEN.
 * On return level[] and sigma[] hold the levels and normalised counts of
 * every node reached, and *visited holds the reached nodes. */
typedef struct {
    uint32_t *level;
    uint64_t *sigma;
    uint32_t *visited;   /* reached nodes, in level order */
    uint32_t n_visited;
    uint64_t arcs_scanned;
} bfs_state;

static void bfs_from(const orc_graph *g, uint32_t c_bits, uint32_t s, uint32_t stop,
                     bfs_state *b)
{
    b->n_visited = 0;
    b->arcs_scanned = 0;
    b->level[s] = 0;
    b->sigma[s] = 1;
    b->visited[b->n_visited++] = s;
    uint32_t lo = 0, hi = 1;        /* visited[lo, hi) is the current level */
    uint32_t L = 0;
    while (lo < hi && (stop == UNSEEN || b->level[stop] == UNSEEN)) {
        /* expand level L: discover level L+1 and accumulate raw counts */
        for (uint32_t q = lo; q < hi; q++) {
            uint32_t w = b->visited[q];
            for (uint32_t e = g->row_ptr[w]; e < g->row_ptr[w + 1]; e++) {
                uint32_t v = g->col_idx[e];
                b->arcs_scanned++;
                if (b->level[v] == UNSEEN) {
                    b->level[v] = L + 1;
                    b->sigma[v] = 0;
                    b->visited[b->n_visited++] = v;
                }
                if (b->level[v] == L + 1)
                    b->sigma[v] += b->sigma[w];
            }
        }
        lo = hi;
        hi = b->n_visited;
        /* normalise level L+1: shift by the excess of its largest raw count */
        uint64_t mx = 0;
        for (uint32_t q = lo; q < hi; q++)
            if (b->sigma[b->visited[q]] > mx) mx = b->sigma[b->visited[q]];
        uint32_t bl = bitlen64(mx);
        uint32_t shift = bl > c_bits ? bl - c_bits : 0;
        for (uint32_t q = lo; q < hi; q++) {
            uint64_t x = b->sigma[b->visited[q]] >> shift;
            b->sigma[b->visited[q]] = x ? x : 1;
        }
        L++;
    }
}

static void bfs_reset(bfs_state *b)
{
    for (uint32_t q = 0; q < b->n_visited; q++) {
        b->level[b->visited[q]] = UNSEEN;
        b->sigma[b->visited[q]] = 0;
    }
    b->n_visited = 0;
}

static int bfs_alloc(bfs_state *b, uint32_t n)
{
    b->level = malloc(sizeof(uint32_t) * n);
    b->sigma = calloc(n, sizeof(uint64_t));
    b->visited = malloc(sizeof(uint32_t) * n);
    if (!b->level || !b->sigma || !b->visited) return -1;
    for (uint32_t v = 0; v < n; v++) b->level[v] = UNSEEN;
    b->n_visited = 0;
    return 0;
}

static void bfs_free(bfs_state *b)
{
    free(b->level); free(b->sigma); free(b->visited);
}

void orc_bfs_counts(const orc_graph *g, uint32_t c_bits, uint32_t s,
                    uint32_t *level, uint64_t *sigma)
{
    bfs_state b;
    bfs_alloc(&b, g->n);
    bfs_from(g, c_bits, s, UNSEEN, &b);
    for (uint32_t v = 0; v < g->n; v++) {
        level[v] = b.level[v];
        sigma[v] = b.level[v] == UNSEEN ? 0 : b.sigma[v];
    }
    bfs_free(&b);
}

/* One hyperedge of the set-betweenness space (Sec. 3.1; sampling procedure
 * of Sec. 5 under readings R1-R6). */
static uint32_t sample_one(const orc_graph *g, uint32_t c_bits, uint64_t seed,
                           uint32_t instance, uint64_t sample, uint32_t *h,
                           orc_sample_info *info, bfs_state *b)
{
    orc_stream st;
    orc_stream_init(&st, seed, sample, instance, 0);
    uint32_t n = g->n;
    uint32_t s = (uint32_t)orc_bounded(&st, n);
    uint32_t tp = (uint32_t)orc_bounded(&st, n - 1);
    uint32_t t = tp + (tp >= s ? 1u : 0u);

    bfs_from(g, c_bits, s, t, b);
    uint32_t d = b->level[t];
    uint32_t len = 0;
    if (d != UNSEEN && d >= 2) {
        const uint32_t *ip = in_ptr(g), *ii = in_idx(g);
        uint32_t v = t;
        while (b->level[v] >= 2) {
            uint32_t want = b->level[v] - 1;
            uint64_t W = 0;
            for (uint32_t e = ip[v]; e < ip[v + 1]; e++)
                if (b->level[ii[e]] == want) W += b->sigma[ii[e]];
            uint64_t r = orc_bounded(&st, W);
            uint64_t acc = 0;
            uint32_t pick = UNSEEN;
            for (uint32_t e = ip[v]; e < ip[v + 1]; e++) {
                uint32_t w = ii[e];
                if (b->level[w] != want) continue;
                acc += b->sigma[w];
                if (acc > r) { pick = w; break; }
            }
            h[len++] = pick;
            v = pick;
        }
    }
    if (info) {
        info->s = s;
        info->t = t;
        info->dist = d;
        info->len = len;
        info->arcs_scanned = b->arcs_scanned;
        info->nodes_visited = b->n_visited;
    }
    bfs_reset(b);
    return len;
}

uint32_t orc_sample_path(const orc_graph *g, uint32_t c_bits, uint64_t seed,
                         uint32_t instance, uint64_t sample, uint32_t *h,
                         orc_sample_info *info)
{
    bfs_state b;
    if (bfs_alloc(&b, g->n)) return 0;
    uint32_t len = sample_one(g, c_bits, seed, instance, sample, h, info, &b);
    bfs_free(&b);
    return len;
}

uint64_t orc_sample_paths(const orc_graph *g, uint32_t c_bits, uint64_t seed,
                          uint32_t instance, uint64_t first, uint64_t count,
                          uint64_t *he_off, uint32_t *he_nodes, uint64_t he_cap,
                          orc_sample_info *infos)
{
    bfs_state b;
    if (bfs_alloc(&b, g->n)) return UINT64_MAX;
    uint32_t *h = malloc(sizeof(uint32_t) * g->n);
    uint64_t total = 0;
    he_off[0] = 0;
    for (uint64_t i = 0; i < count; i++) {
        uint32_t len = sample_one(g, c_bits, seed, instance, first + i, h,
                                  infos ? &infos[i] : NULL, &b);
        if (total + len > he_cap) { total = UINT64_MAX; break; }
        memcpy(he_nodes + total, h, sizeof(uint32_t) * len);
        total += len;
        he_off[i + 1] = total;
    }
    free(h);
    bfs_free(&b);
    return total;
}

/* ------------------------------------------------------------------ */
/* Balanced bidirectional sampler (the sampling procedure of Sec. 5, under
 * reading R16): a search from s over out-arcs and one from t over in-arcs,
 * each level with normalised counts (R4; the forward budget from the
 * largest in-degree, the backward one from the largest out-degree); each
 * step expands the side whose frontier has fewer arcs to scan (the forward
 * side on ties).  When a new level meets the other side's last level, the
 * meeting nodes M split every shortest path: one node of M is drawn with
 * weight sigma_f * sigma_b (scaled so that the sum fits 63 bits), then the
 * path is walked from it to t over the backward counts and to s over the
 * forward counts. */
uint32_t orc_count_bits_out(const orc_graph *g)
{
    uint64_t dmax = 0;
    for (uint32_t v = 0; v < g->n; v++) {
        uint64_t d = g->row_ptr[v + 1] - g->row_ptr[v];
        if (d > dmax) dmax = d;
    }
    return 63 - bitlen64(dmax);
}

typedef struct {
    uint32_t *level;
    uint64_t *sigma;
    uint32_t *visited;
    uint32_t n_visited;
    uint32_t lo, hi;      /* visited[lo, hi) is the last level */
} side_state;

static int side_alloc(side_state *z, uint32_t n)
{
    z->level = malloc(sizeof(uint32_t) * n);
    z->sigma = calloc(n, sizeof(uint64_t));
    z->visited = malloc(sizeof(uint32_t) * n);
    if (!z->level || !z->sigma || !z->visited) return -1;
    for (uint32_t v = 0; v < n; v++) z->level[v] = UNSEEN;
    z->n_visited = 0;
    return 0;
}

static void side_free(side_state *z) { free(z->level); free(z->sigma); free(z->visited); }

static void side_reset(side_state *z)
{
    for (uint32_t q = 0; q < z->n_visited; q++) {
        z->level[z->visited[q]] = UNSEEN;
        z->sigma[z->visited[q]] = 0;
    }
    z->n_visited = 0;
}

static void side_start(side_state *z, uint32_t root)
{
    z->level[root] = 0;
    z->sigma[root] = 1;
    z->visited[0] = root;
    z->n_visited = 1;
    z->lo = 0;
    z->hi = 1;
}

/* Arcs that expanding the side's last level would scan (rows of ptr). */
static uint64_t side_cost(const side_state *z, const uint32_t *ptr)
{
    uint64_t c = 0;
    for (uint32_t q = z->lo; q < z->hi; q++) c += ptr[z->visited[q] + 1] - ptr[z->visited[q]];
    return c;
}

/* Expands the side's last level L over the rows (ptr, idx): level L + 1 and
 * its raw counts, then the level's normalisation with budget c_bits. */
static void side_expand(side_state *z, const uint32_t *ptr, const uint32_t *idx, uint32_t c_bits,
                        uint64_t *arcs)
{
    const uint32_t L = z->level[z->visited[z->lo]];
    const uint32_t lo = z->lo, hi = z->hi;
    for (uint32_t q = lo; q < hi; q++) {
        uint32_t w = z->visited[q];
        for (uint32_t e = ptr[w]; e < ptr[w + 1]; e++) {
            uint32_t v = idx[e];
            (*arcs)++;
            if (z->level[v] == UNSEEN) {
                z->level[v] = L + 1;
                z->sigma[v] = 0;
                z->visited[z->n_visited++] = v;
            }
            if (z->level[v] == L + 1) z->sigma[v] += z->sigma[w];
        }
    }
    z->lo = hi;
    z->hi = z->n_visited;
    uint64_t mx = 0;
    for (uint32_t q = z->lo; q < z->hi; q++)
        if (z->sigma[z->visited[q]] > mx) mx = z->sigma[z->visited[q]];
    uint32_t bl = bitlen64(mx);
    uint32_t shift = bl > c_bits ? bl - c_bits : 0;
    for (uint32_t q = z->lo; q < z->hi; q++) {
        uint64_t x = z->sigma[z->visited[q]] >> shift;
        z->sigma[z->visited[q]] = x ? x : 1;
    }
}

static int cmp_u32(const void *x, const void *y)
{
    uint32_t a = *(const uint32_t *)x, b = *(const uint32_t *)y;
    return a < b ? -1 : a > b;
}

/* One step of a walk: among the row entries of cur (rows ptr, idx) whose
 * level on side z is `want`, in row order, the one drawn with weight sigma. */
static uint32_t walk_step(const side_state *z, const uint32_t *ptr, const uint32_t *idx, uint32_t cur,
                          uint32_t want, orc_stream *st)
{
    uint64_t W = 0;
    for (uint32_t e = ptr[cur]; e < ptr[cur + 1]; e++)
        if (z->level[idx[e]] == want) W += z->sigma[idx[e]];
    uint64_t r = orc_bounded(st, W);
    uint64_t acc = 0;
    for (uint32_t e = ptr[cur]; e < ptr[cur + 1]; e++) {
        uint32_t u = idx[e];
        if (z->level[u] != want) continue;
        acc += z->sigma[u];
        if (acc > r) return u;
    }
    return UNSEEN;
}

/* Meeting weight of v before scaling: the number of shortest s-v paths
 * times the number of shortest v-t paths (normalised counts). */
static unsigned __int128 meet_weight(const side_state *F, const side_state *B, uint32_t v)
{
    return (unsigned __int128)F->sigma[v] * B->sigma[v];
}

static uint32_t bidir_one(const orc_graph *g, uint32_t c_f, uint32_t c_b, uint64_t seed, uint32_t instance,
                          uint64_t sample, uint32_t *h, orc_sample_info *info, side_state *F, side_state *B,
                          uint32_t *scratch)
{
    orc_stream st;
    orc_stream_init(&st, seed, sample, instance, 7);
    uint32_t n = g->n;
    uint32_t s = (uint32_t)orc_bounded(&st, n);
    uint32_t tp = (uint32_t)orc_bounded(&st, n - 1);
    uint32_t t = tp >= s ? tp + 1u : tp;   /* the pair rule of R3 */
    const uint32_t *ip = in_ptr(g), *ii = in_idx(g);
    uint64_t arcs = 0;
    side_start(F, s);
    side_start(B, t);
    uint32_t a = 0, b = 0, d = UNSEEN;
    uint32_t *M = scratch, nm = 0;
    while (F->lo < F->hi && B->lo < B->hi) {
        if (side_cost(F, g->row_ptr) <= side_cost(B, ip)) {
            side_expand(F, g->row_ptr, g->col_idx, c_f, &arcs);
            a++;
            for (uint32_t q = F->lo; q < F->hi; q++)
                if (B->level[F->visited[q]] == b) M[nm++] = F->visited[q];
        } else {
            side_expand(B, ip, ii, c_b, &arcs);
            b++;
            for (uint32_t q = B->lo; q < B->hi; q++)
                if (F->level[B->visited[q]] == a) M[nm++] = B->visited[q];
        }
        if (nm) {
            d = a + b;
            break;
        }
    }
    uint32_t len = 0;
    if (d != UNSEEN && d >= 2) {
        qsort(M, nm, sizeof(uint32_t), cmp_u32);
        /* weights sigma_f sigma_b, scaled so that their sum stays below 2^63 */
        unsigned __int128 pmax = 0;
        for (uint32_t i = 0; i < nm; i++) {
            unsigned __int128 p = meet_weight(F, B, M[i]);
            if (p > pmax) pmax = p;
        }
        uint32_t pbits = 0;
        for (unsigned __int128 x = pmax; x; x >>= 1) pbits++;
        const uint32_t room = 63 - bitlen64(nm);
        const uint32_t shift = pbits > room ? pbits - room : 0;
        uint64_t W = 0;
        for (uint32_t i = 0; i < nm; i++) {
            uint64_t w = (uint64_t)(meet_weight(F, B, M[i]) >> shift);
            W += w ? w : 1;
        }
        uint64_t r = orc_bounded(&st, W), acc = 0;
        uint32_t v = UNSEEN;
        for (uint32_t i = 0; i < nm; i++) {
            uint64_t w = (uint64_t)(meet_weight(F, B, M[i]) >> shift);
            acc += w ? w : 1;
            if (acc > r) { v = M[i]; break; }
        }
        /* toward t over the backward counts (successors on out-rows) */
        uint32_t nt = 0, cur = v;
        uint32_t *tside = scratch;   /* M is no longer needed */
        while (B->level[cur] >= 2) {
            cur = walk_step(B, g->row_ptr, g->col_idx, cur, B->level[cur] - 1, &st);
            tside[nt++] = cur;
        }
        for (uint32_t i = nt; i > 0; i--) h[len++] = tside[i - 1];
        if (a >= 1 && b >= 1) h[len++] = v;
        /* toward s over the forward counts (predecessors on in-rows) */
        cur = v;
        while (F->level[cur] >= 2) {
            cur = walk_step(F, ip, ii, cur, F->level[cur] - 1, &st);
            h[len++] = cur;
        }
    }
    if (info) {
        info->s = s;
        info->t = t;
        info->dist = d;
        info->len = len;
        info->arcs_scanned = arcs;
        info->nodes_visited = F->n_visited + B->n_visited;
    }
    side_reset(F);
    side_reset(B);
    return len;
}

uint64_t orc_sample_paths_bidir(const orc_graph *g, uint32_t c_f, uint32_t c_b, uint64_t seed,
                                uint32_t instance, uint64_t first, uint64_t count, uint64_t *he_off,
                                uint32_t *he_nodes, uint64_t he_cap, orc_sample_info *infos)
{
    side_state F, B;
    uint32_t *h = malloc(sizeof(uint32_t) * g->n);
    uint32_t *scratch = malloc(sizeof(uint32_t) * g->n);
    if (!h || !scratch || side_alloc(&F, g->n) || side_alloc(&B, g->n)) return UINT64_MAX;
    uint64_t total = 0;
    he_off[0] = 0;
    for (uint64_t i = 0; i < count; i++) {
        uint32_t len = bidir_one(g, c_f, c_b, seed, instance, first + i, h, infos ? &infos[i] : NULL, &F, &B,
                                 scratch);
        if (total + len > he_cap) { total = UINT64_MAX; break; }
        memcpy(he_nodes + total, h, sizeof(uint32_t) * len);
        total += len;
        he_off[i + 1] = total;
    }
    free(h);
    free(scratch);
    side_free(&F);
    side_free(&B);
    return total;
}

/* ------------------------------------------------------------------ */
/* greedyCover(k, H) (Sec. 3.1; Algorithm 1 greedy step).  Each round
 * recomputes, for every node, the number of not-yet-covered hyperedges it
 * belongs to -- its marginal gain m*(C_H(S u {u}) - C_H(S)) -- and adds the
 * node with the largest gain (reading R7). */
uint32_t orc_greedy_cover(uint32_t n, uint64_t m, const uint64_t *he_off,
                          const uint32_t *he_nodes, uint32_t k,
                          uint32_t *picks, uint64_t *cov_cum)
{
    uint8_t *covered = calloc(m ? m : 1, 1);
    uint64_t *gain = malloc(sizeof(uint64_t) * n);
    uint64_t cov = 0;
    uint32_t r;
    for (r = 0; r < k; r++) {
        memset(gain, 0, sizeof(uint64_t) * n);
        for (uint64_t s = 0; s < m; s++) {
            if (covered[s]) continue;
            for (uint64_t e = he_off[s]; e < he_off[s + 1]; e++)
                gain[he_nodes[e]]++;
        }
        uint32_t best = 0;
        for (uint32_t u = 1; u < n; u++)
            if (gain[u] > gain[best]) best = u;
        if (gain[best] == 0) break;
        for (uint64_t s = 0; s < m; s++) {
            if (covered[s]) continue;
            for (uint64_t e = he_off[s]; e < he_off[s + 1]; e++)
                if (he_nodes[e] == best) { covered[s] = 1; cov++; break; }
        }
        picks[r] = best;
        cov_cum[r] = cov;
    }
    free(covered);
    free(gain);
    return r;
}

/* ------------------------------------------------------------------ */
/* Rademacher matrix (Sec. 2.2 definition of sigma; reading R8). */
int orc_rademacher(uint64_t seed, uint32_t instance, uint64_t s, uint32_t j)
{
    uint64_t ctr[4] = { j / 256u, s, instance, 1 };
    uint64_t key[2] = { seed, 0 };
    uint64_t out[4];
    orc_philox4x64_10(ctr, key, out);
    uint64_t word = out[(j % 256u) / 64u];
    return ((word >> (j % 64u)) & 1u) ? 1 : -1;
}

/* m * r_j^u of Algorithm 1 (AMCERA step): R[u][j] = sum_s sigma_js f_u(h_s). */
void orc_rade_sums(uint32_t n, uint64_t m, const uint64_t *he_off,
                   const uint32_t *he_nodes, uint64_t seed, uint32_t instance,
                   uint32_t t, int64_t *R)
{
    memset(R, 0, sizeof(int64_t) * (size_t)n * t);
    int *sig = malloc(sizeof(int) * t);
    for (uint64_t s = 0; s < m; s++) {
        if (he_off[s + 1] == he_off[s]) continue;
        for (uint32_t j = 0; j < t; j++)
            sig[j] = orc_rademacher(seed, instance, s, j);
        for (uint64_t e = he_off[s]; e < he_off[s + 1]; e++) {
            uint32_t u = he_nodes[e];
            for (uint32_t j = 0; j < t; j++)
                R[(size_t)u * t + j] += sig[j];
        }
    }
    free(sig);
}

static int cmp_desc_i64(const void *a, const void *b)
{
    int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    return x < y ? 1 : (x > y ? -1 : 0);
}

static int cmp_desc_u64(const void *a, const void *b)
{
    uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    return x < y ? 1 : (x > y ? -1 : 0);
}

/* AMCERA (Sec. 4.1 definition; Algorithm 1 AMCERA steps) and the inputs of
 * the approximate wimpy variance (Sec. 4.1 definition): the per-trial
 * supremum is the sum of the largest positive sums (reading R9). */
double orc_mcera(uint32_t n, uint64_t m, const uint64_t *he_off,
                 const uint32_t *he_nodes, uint64_t seed, uint32_t instance,
                 uint32_t t, uint32_t k, int64_t *topk_sum,
                 uint64_t *deg_topk, uint32_t *b_max)
{
    int64_t *R = malloc(sizeof(int64_t) * (size_t)n * t);
    orc_rade_sums(n, m, he_off, he_nodes, seed, instance, t, R);
    int64_t *col = malloc(sizeof(int64_t) * n);
    int64_t total = 0;
    for (uint32_t j = 0; j < t; j++) {
        uint32_t npos = 0;
        for (uint32_t u = 0; u < n; u++) {
            int64_t x = R[(size_t)u * t + j];
            if (x > 0) col[npos++] = x;
        }
        qsort(col, npos, sizeof(int64_t), cmp_desc_i64);
        int64_t sum = 0;
        for (uint32_t q = 0; q < npos && q < k; q++) sum += col[q];
        topk_sum[j] = sum;
        total += sum;
    }
    free(col);
    free(R);

    uint64_t *deg = calloc(n, sizeof(uint64_t));
    uint32_t bm = 0;
    for (uint64_t s = 0; s < m; s++) {
        uint64_t len = he_off[s + 1] - he_off[s];
        if (len > bm) bm = (uint32_t)len;
        for (uint64_t e = he_off[s]; e < he_off[s + 1]; e++) deg[he_nodes[e]]++;
    }
    qsort(deg, n, sizeof(uint64_t), cmp_desc_u64);
    uint64_t dk = 0;
    for (uint32_t q = 0; q < n && q < k; q++) dk += deg[q];
    free(deg);
    *deg_topk = dk;
    *b_max = bm;
    return (double)total / ((double)t * (double)m);
}

/* ------------------------------------------------------------------ */
/* Theorem bound_dev (eq. epsrade) with the Algorithm 1 definition of xi and
 * its stopping condition; a = 1 - 1/e and L = ln(5/delta_i). */
void orc_bound(uint64_t m, uint64_t cov, int64_t sum_topk, uint32_t t,
               uint64_t deg_topk, uint32_t b_max, double eps, double delta_i,
               orc_bound_out *o)
{
    const double a = 1.0 - exp(-1.0);
    const double md = (double)m;
    const double L = log(5.0 / delta_i);
    const double C = (double)cov / md;
    const double amcera = (double)sum_topk / ((double)t * md);
    const double wimpy = (double)b_max * (double)deg_topk / md;
    const double xi = sqrt((L / md) * (L / md) + 2.0 * C * L / (a * md)) + L / md;
    const double nu = C / a + xi;
    const double rtilde = amcera + sqrt(4.0 * wimpy * L / ((double)t * md));
    const double r = rtilde + sqrt((L / md) * (L / md) + 2.0 * L * rtilde / md) + L / md;
    const double eta = 2.0 * r + sqrt(2.0 * L * (nu + 4.0 * r) / md) + L / (3.0 * md);
    o->c_hat = C;
    o->amcera = amcera;
    o->wimpy = wimpy;
    o->xi = xi;
    o->nu = nu;
    o->rtilde = rtilde;
    o->r = r;
    o->eta = eta;
    o->certified = a * ((a - eps) * xi + eta) <= eps * C;
}

/* HEDGE-P's bound (Sec. 5 describes HEDGE-P: Algorithm 1's iterations with
 * a union-bound eta^UB in place of the AMCERA and HEDGE's stopping rule
 * SD <= eps C(S*) / 2; the paper does not print eta^UB, so this form is the
 * builder's own, reading R17).  There are N_k = sum_{j <= k} C(n, j) node
 * sets of at most k nodes; for each, C_H(S) is the mean of m independent
 * indicators with mean C(S), and Hoeffding's two-sided inequality with a
 * union bound over all of them at confidence delta_i gives
 *   eta^UB = sqrt((ln(2 N_k) + ln(1 / delta_i)) / (2 m)).
 * On that event C(S*) >= C(S) >= C_H(S) - eta^UB for the greedy set S, so
 * the rule SD <= eps C(S*) / 2 holds once eta^UB <= eps (C_H(S) - eta^UB) / 2. */
double orc_log_sets(uint64_t n, uint32_t k)
{
    /* log-sum-exp of ln C(n, j), j = 0 .. min(k, n) */
    const uint64_t top = k < n ? k : n;
    double mx = -INFINITY;
    for (uint64_t j = 0; j <= top; j++) {
        double x = lgamma((double)n + 1.0) - lgamma((double)j + 1.0) - lgamma((double)(n - j) + 1.0);
        if (x > mx) mx = x;
    }
    double acc = 0.0;
    for (uint64_t j = 0; j <= top; j++) {
        double x = lgamma((double)n + 1.0) - lgamma((double)j + 1.0) - lgamma((double)(n - j) + 1.0);
        acc += exp(x - mx);
    }
    return mx + log(acc);
}

void orc_hedge_bound(uint64_t m, uint64_t cov, uint64_t n, uint32_t k, double eps, double delta_i,
                     orc_bound_out *o)
{
    memset(o, 0, sizeof(*o));
    const double C = (double)cov / (double)m;
    const double eta = sqrt((log(2.0) + orc_log_sets(n, k) + log(1.0 / delta_i)) / (2.0 * (double)m));
    o->c_hat = C;
    o->eta = eta;
    o->certified = eta <= eps * (C - eta) / 2.0;
}

/* ------------------------------------------------------------------ */
/* Algorithm 1 (progressive sampling), readings R1 and R10. */
/* ---- triangle hyperedges (Sec. 3.1) ---- */

static int adjacent(const orc_graph *g, uint32_t u, uint32_t v)
{
    for (uint64_t e = g->row_ptr[u]; e < g->row_ptr[u + 1]; e++)
        if (g->col_idx[e] == v) return 1;
    return 0;
}

uint64_t orc_row_triangles(const orc_graph *g, uint32_t a, uint32_t *tri, uint64_t cap)
{
    if (g->directed) return UINT64_MAX;
    uint64_t T = 0;
    for (uint64_t e = g->row_ptr[a]; e < g->row_ptr[a + 1]; e++) {
        const uint32_t b = g->col_idx[e];
        if (b <= a) continue;
        for (uint64_t f = e + 1; f < g->row_ptr[a + 1]; f++) {
            const uint32_t c = g->col_idx[f];   /* c > b: rows ascend */
            if (!adjacent(g, b, c)) continue;
            if (T < cap) {
                tri[3 * T] = a;
                tri[3 * T + 1] = b;
                tri[3 * T + 2] = c;
            }
            T++;
        }
    }
    return T;
}

uint64_t orc_triangles(const orc_graph *g, uint32_t *tri, uint64_t cap)
{
    if (g->directed) return UINT64_MAX;
    uint64_t T = 0;
    for (uint32_t a = 0; a < g->n; a++)
        T += orc_row_triangles(g, a, tri ? tri + 3 * T : NULL, T < cap ? cap - T : 0);
    return T;
}

int orc_sample_triangles(const orc_graph *g, uint64_t seed, uint32_t instance,
                         uint64_t first, uint64_t count, uint64_t *he_off,
                         uint32_t *he_nodes)
{
    const uint64_t T = orc_triangles(g, NULL, 0);
    if (T == UINT64_MAX || T == 0) return -1;
    uint32_t *all = malloc(sizeof(uint32_t) * 3 * T);
    if (!all) return -1;
    orc_triangles(g, all, T);
    he_off[0] = 0;
    for (uint64_t i = 0; i < count; i++) {
        orc_stream st;
        orc_stream_init(&st, seed, first + i, instance, 5);
        const uint64_t r = orc_bounded(&st, T);
        memcpy(he_nodes + 3 * i, all + 3 * r, 3 * sizeof(uint32_t));
        he_off[i + 1] = 3 * (i + 1);
    }
    free(all);
    return 0;
}

/* kappa-path hyperedges (Sec. 3.1 names the space: the node sets of simple
 * paths of length at most kappa; the paper gives no sampler).  Reading, the
 * random simple walk of the kappa-path centrality: from the stream (seed,
 * sample, instance, tag 6) draw the start s = bounded(n) and the length
 * l = 1 + bounded(kappa); then, l times, move from the current node v to
 * the r-th (r = bounded(f)) of v's f out-neighbours that are not yet on the
 * walk, in ascending id; stop early when f = 0.  The hyperedge is the walk
 * after s (at most kappa nodes, the b <= kappa of Sec. 4.3). */
static int on_walk(uint32_t x, uint32_t s, const uint32_t *h, uint32_t len)
{
    if (x == s) return 1;
    for (uint32_t i = 0; i < len; i++)
        if (h[i] == x) return 1;
    return 0;
}

uint32_t orc_kpath(const orc_graph *g, uint32_t kappa, uint64_t seed, uint32_t instance,
                   uint64_t sample, uint32_t *h, uint32_t *s_out, uint32_t *l_out)
{
    orc_stream st;
    orc_stream_init(&st, seed, sample, instance, 6);
    const uint32_t s = (uint32_t)orc_bounded(&st, g->n);
    const uint32_t l = 1 + (uint32_t)orc_bounded(&st, kappa);
    if (s_out) *s_out = s;
    if (l_out) *l_out = l;
    uint32_t v = s, len = 0;
    while (len < l) {
        uint64_t f = 0;
        for (uint64_t e = g->row_ptr[v]; e < g->row_ptr[v + 1]; e++)
            f += !on_walk(g->col_idx[e], s, h, len);
        if (f == 0) break;
        uint64_t r = orc_bounded(&st, f);
        for (uint64_t e = g->row_ptr[v]; e < g->row_ptr[v + 1]; e++) {
            const uint32_t w = g->col_idx[e];
            if (on_walk(w, s, h, len)) continue;
            if (r == 0) {
                v = w;
                break;
            }
            r--;
        }
        h[len++] = v;
    }
    return len;
}

int orc_sample_kpaths(const orc_graph *g, uint32_t kappa, uint64_t seed, uint32_t instance,
                      uint64_t first, uint64_t count, uint64_t *he_off, uint32_t *he_nodes)
{
    if (kappa == 0 || g->n == 0) return -1;
    he_off[0] = 0;
    for (uint64_t i = 0; i < count; i++) {
        const uint32_t len = orc_kpath(g, kappa, seed, instance, first + i, he_nodes + he_off[i], NULL, NULL);
        he_off[i + 1] = he_off[i] + len;
    }
    return 0;
}

/* VC-dimension bounds of the range spaces Q_k of Sec. 4.3 (ranges: the
 * hyperedges met by a node set of at most k nodes).  Lemma vcboundgeneral:
 * with hyperedges of at most b nodes, VC(Q_1) <= d1 = floor(log2(2b)),
 * taken here as the largest j with 2^j <= 2b.  Lemma lemmavckbound:
 * VC(Q_k) <= 2 VC(Q_1) k log2(3k), floored.  And VC(Q_k) <= log2 |R_k| <=
 * floor(k log2 n), the union bound. */
int orc_vc_dims(uint64_t b, uint32_t k, uint64_t n, uint32_t *d1, uint64_t *dk_lemma, uint64_t *dk_union)
{
    if (b == 0 || k == 0 || n == 0) return -1;
    uint32_t j = 0;
    while (j < 63 && ((uint64_t)1 << (j + 1)) <= b) j++;   /* then 2^j <= b < 2^(j+1): floor(log2(2b)) = j + 1 */
    *d1 = j + 1;
    *dk_lemma = (uint64_t)floor(2.0 * (double)(*d1) * (double)k * log2(3.0 * (double)k));
    *dk_union = (uint64_t)floor((double)k * log2((double)n));
    return 0;
}

uint64_t orc_next_sample_size(uint64_t m_i, double c_hat, double eps, double delta_next,
                              uint32_t growth_num, uint32_t growth_den, uint64_t m_max,
                              uint32_t schedule)
{
    u128 geo = ((u128)m_i * growth_num + growth_den - 1) / growth_den;
    uint64_t next = geo > m_max ? m_max : (uint64_t)geo;
    if (schedule != 1 || !(c_hat > 0.0)) return next;
    /* the optimistic eta, sqrt(2L/m) + L/(3m), is at most the target
     * T = eps*c_hat/a exactly when y = 1/sqrt(m) is at most the positive
     * root of (L/3) y^2 + sqrt(2L) y - T = 0, that is
     * y = 2T / (sqrt(2L) + sqrt(2L + 4LT/3)); hence m = (1/y)^2 */
    const double a = 1.0 - exp(-1.0);
    const double L = log(5.0 / delta_next);
    const double T = eps * c_hat / a;
    const double inv_y = (sqrt(2.0 * L) + sqrt(2.0 * L + 4.0 * L * T / 3.0)) / (2.0 * T);
    const double m = inv_y * inv_y;
    const uint64_t opt = m < (double)m_max ? (uint64_t)ceil(m) : m_max;
    return opt > next ? opt : next;
}

int orc_progressive(const orc_graph *g, uint32_t c_bits, uint32_t k, uint32_t t,
                    double eps, double delta, uint64_t seed, uint32_t instance,
                    uint64_t m_init, uint64_t m_max, uint32_t growth_num,
                    uint32_t growth_den, uint32_t schedule, uint32_t space, uint32_t kappa,
                    uint32_t method, uint32_t *picks, orc_result *res, uint64_t *m_log,
                    uint32_t m_log_cap)
{
    const double a = 1.0 - exp(-1.0);
    if (k == 0 || t == 0 || !(eps > 0.0 && eps < a) || !(delta > 0.0 && delta < 1.0) ||
        m_init == 0 || m_max < m_init || growth_den == 0 || growth_num <= growth_den ||
        schedule > 2 || space > 3 || (space == 2 && kappa == 0) || method > 1)
        return -1;
    /* space 3: the bidirectional sampler; a lowered forward budget (a test
     * override) lowers the backward one too */
    side_state F, B;
    uint32_t *bscratch = NULL;
    uint32_t c_b = orc_count_bits_out(g);
    if (c_bits < orc_count_bits(g) && c_bits < c_b) c_b = c_bits;
    if (space == 3) {
        bscratch = malloc(sizeof(uint32_t) * g->n);
        if (!bscratch || side_alloc(&F, g->n) || side_alloc(&B, g->n)) return -1;
    }
    uint32_t *tri = NULL;
    uint64_t T = 0;
    if (space == 1) {
        T = orc_triangles(g, NULL, 0);
        if (T == UINT64_MAX || T == 0) return -1;
        tri = malloc(sizeof(uint32_t) * 3 * T);
        orc_triangles(g, tri, T);
    }
    uint64_t cap = 1024;
    uint64_t *he_off = malloc(sizeof(uint64_t) * (m_max + 1));
    uint32_t *he_nodes = malloc(sizeof(uint32_t) * cap);
    uint32_t *h = malloc(sizeof(uint32_t) * (g->n > kappa ? g->n : kappa));
    uint64_t *cov_cum = malloc(sizeof(uint64_t) * k);
    int64_t *topk = malloc(sizeof(int64_t) * t);
    bfs_state b;
    bfs_alloc(&b, g->n);
    he_off[0] = 0;
    uint64_t m_prev = 0, m_i = m_init;
    int rc = 1;
    memset(res, 0, sizeof(*res));
    for (uint32_t i = 1;; i++) {
        /* the fixed-size use bounds one sample with delta itself */
        const double delta_i = schedule == 2 ? delta : ldexp(delta, -(int)i);
        if (m_log && i <= m_log_cap) m_log[i - 1] = m_i;
        for (uint64_t s = m_prev; s < m_i; s++) {
            uint32_t len;
            if (space == 1) {
                orc_stream st;
                orc_stream_init(&st, seed, s, instance, 5);
                memcpy(h, tri + 3 * orc_bounded(&st, T), 3 * sizeof(uint32_t));
                len = 3;
            } else if (space == 2) {
                len = orc_kpath(g, kappa, seed, instance, s, h, NULL, NULL);
            } else if (space == 3) {
                len = bidir_one(g, c_bits, c_b, seed, instance, s, h, NULL, &F, &B, bscratch);
            } else {
                len = sample_one(g, c_bits, seed, instance, s, h, NULL, &b);
            }
            if (he_off[s] + len > cap) {
                while (he_off[s] + len > cap) cap *= 2;
                he_nodes = realloc(he_nodes, sizeof(uint32_t) * cap);
            }
            memcpy(he_nodes + he_off[s], h, sizeof(uint32_t) * len);
            he_off[s + 1] = he_off[s] + len;
        }
        uint32_t np = orc_greedy_cover(g->n, m_i, he_off, he_nodes, k, picks, cov_cum);
        uint64_t cov = np ? cov_cum[np - 1] : 0;
        orc_bound_out o;
        if (method == 1) {   /* HEDGE-P: the union bound, no AMCERA */
            orc_hedge_bound(m_i, cov, g->n, k, eps, delta_i, &o);
        } else {
            uint64_t dk;
            uint32_t bm;
            orc_mcera(g->n, m_i, he_off, he_nodes, seed, instance, t, k, topk, &dk, &bm);
            int64_t sum = 0;
            for (uint32_t j = 0; j < t; j++) sum += topk[j];
            orc_bound(m_i, cov, sum, t, dk, bm, eps, delta_i, &o);
        }
        res->n_picked = np;
        res->iterations = i;
        res->certified = o.certified;
        res->coverage = cov;
        res->m_final = m_i;
        res->c_hat = o.c_hat;
        res->amcera = o.amcera;
        res->wimpy = o.wimpy;
        res->xi = o.xi;
        res->nu = o.nu;
        res->rtilde = o.rtilde;
        res->r = o.r;
        res->eta = o.eta;
        if (o.certified) { rc = 0; break; }
        if (schedule == 2 || m_i >= m_max) { rc = 1; break; }
        m_prev = m_i;
        m_i = orc_next_sample_size(m_i, o.c_hat, eps, ldexp(delta, -(int)(i + 1)), growth_num,
                                   growth_den, m_max, schedule);
    }
    bfs_free(&b);
    if (space == 3) {
        side_free(&F);
        side_free(&B);
        free(bscratch);
    }
    free(he_off); free(he_nodes); free(h); free(cov_cum); free(topk); free(tri);
    return rc;
}
