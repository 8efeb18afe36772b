/*
 * centra_oracle.h -- plain, slow CPU oracle for the CentRA hot path
 * (Pellegrina, "Efficient Centrality Maximization with Rademacher Averages",
 * KDD 2023, arXiv 2306.03651).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists so that the tests, the smoke
 * check and the CPU-baseline leg of the benchmark can check the HIP path
 * against an independent implementation.  It shares no source with the HIP
 * path and no product code may link or call it.
 *
 * Every quantity is computed as the paper defines it, step by step, in the
 * paper's order:
 *   - hyperedge sampling for set betweenness (Sec. 3.1 definition of the
 *     hyperedge space; Sec. 5 sampling procedure), made deterministic with a
 *     counter-based generator (Philox4x64-10) and Lemire's bounded draw;
 *   - greedyCover(k, H) (Sec. 3.1 greedy algorithm, Algorithm 1 greedy step);
 *   - the per-node Rademacher sums r_j^u, the per-trial supremum r_j and the
 *     AMCERA (Sec. 4.1 definition; Algorithm 1 AMCERA steps);
 *   - the approximate wimpy variance (Sec. 4.1 definition);
 *   - xi, nu, R~, R, eta (Theorem bound_dev, eq. epsrade) and the stopping
 *     condition of Algorithm 1;
 *   - the progressive loop (Algorithm 1).
 *
 * Readings of points the paper leaves open are listed next to the function
 * that takes them.  Pins (checks against something other than this code) live
 * in tests/test_oracle_*.py.
 */
#ifndef CENTRA_ORACLE_H
#define CENTRA_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Philox4x64-10 block function (Salmon et al., SC'11).  ctr[4], key[2] in,
 * out[4] out. */
void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);

/* A Philox word stream: key = (seed, 0), counter = (block, c1, c2, c3); the
 * blocks b = 0, 1, 2, ... are consumed in order, four words each. */
typedef struct {
    uint64_t key[2];
    uint64_t ctr[4];
    uint64_t buf[4];
    int pos;
} orc_stream;

void orc_stream_init(orc_stream *st, uint64_t seed, uint64_t c1, uint64_t c2, uint64_t c3);
uint64_t orc_stream_next(orc_stream *st);

/* Lemire's unbiased bounded draw in [0, W), W >= 1 (ACM TOMACS 2019). */
uint64_t orc_bounded(orc_stream *st, uint64_t W);

/* Draws `count` bounded values from the stream (seed, c1, c2, c3) into out[]
 * (test hook for the bounded draw). */
void orc_bounded_many(uint64_t seed, uint64_t c1, uint64_t c2, uint64_t c3,
                      uint64_t W, uint64_t count, uint64_t *out);

/* Graph in CSR form.  Rows sorted ascending, no duplicate arcs, no self
 * loops.  For an undirected graph each edge appears as two arcs and the
 * in-neighbour rows are the out-neighbour rows (rrow_ptr == NULL). */
typedef struct {
    uint32_t n;
    uint32_t directed;
    uint64_t n_arcs;
    const uint32_t *row_ptr;   /* n+1 */
    const uint32_t *col_idx;   /* n_arcs */
    const uint32_t *rrow_ptr;  /* n+1, in-neighbours, or NULL if undirected */
    const uint32_t *rcol_idx;  /* n_arcs or NULL */
} orc_graph;

/* Checks the CSR contract; returns 0 if valid, a negative code otherwise. */
int orc_graph_check(const orc_graph *g);

/* C = 63 - bitlen(max in-degree): the bit budget of the normalised counts. */
uint32_t orc_count_bits(const orc_graph *g);

/* Per-sample diagnostics. */
typedef struct {
    uint32_t s, t;        /* the drawn pair */
    uint32_t dist;        /* d(s,t); 0xFFFFFFFF if t is unreachable */
    uint32_t len;         /* |h| */
    uint64_t arcs_scanned;   /* out-arcs scanned by the BFS */
    uint64_t nodes_visited;  /* nodes given a level by the BFS */
} orc_sample_info;

/* Draws sample number `sample` (global index) of instance `instance`:
 * a uniform ordered pair s != t, a BFS from s with normalised path counts,
 * and a uniformly random shortest s-t path by backtracking from t.  Writes
 * the internal nodes (t's neighbour first) to h (capacity n) and returns
 * |h|.  c_bits is the count bit budget (orc_count_bits, or a smaller test
 * override).  info may be NULL. */
uint32_t orc_sample_path(const orc_graph *g, uint32_t c_bits, uint64_t seed,
                         uint32_t instance, uint64_t sample, uint32_t *h,
                         orc_sample_info *info);

/* Samples [first, first+count) into a CSR-like hyperedge store: he_off has
 * count+1 entries relative to the first sample, he_nodes has capacity he_cap.
 * Returns the total number of nodes written, or UINT64_MAX if he_cap is too
 * small.  infos may be NULL. */
uint64_t orc_sample_paths(const orc_graph *g, uint32_t c_bits, uint64_t seed,
                          uint32_t instance, uint64_t first, uint64_t count,
                          uint64_t *he_off, uint32_t *he_nodes, uint64_t he_cap,
                          orc_sample_info *infos);

/* C_b = 63 - bitlen(max out-degree): the budget of the backward counts of
 * the bidirectional sampler (sums over out-neighbours). */
uint32_t orc_count_bits_out(const orc_graph *g);

/* The balanced bidirectional sampler (reading R16): samples [first,
 * first + count) of (seed, instance) from the stream with tag 7, stored as
 * orc_sample_paths does; c_f / c_b are the forward / backward count budgets
 * (orc_count_bits / orc_count_bits_out, or smaller test overrides).  The
 * hyperedge is the path's internal nodes, t's neighbour first. */
uint64_t orc_sample_paths_bidir(const orc_graph *g, uint32_t c_f, uint32_t c_b, uint64_t seed,
                                uint32_t instance, uint64_t first, uint64_t count, uint64_t *he_off,
                                uint32_t *he_nodes, uint64_t he_cap, orc_sample_info *infos);

/* BFS levels and normalised counts from s over the whole graph (test hook):
 * level[v] = d(s,v) or 0xFFFFFFFF, sigma[v] = normalised count (0 if
 * unreachable). */
void orc_bfs_counts(const orc_graph *g, uint32_t c_bits, uint32_t s,
                    uint32_t *level, uint64_t *sigma);

/* greedyCover(k, H): picks[r] and cov_cum[r] (number of hyperedges covered
 * after r+1 picks) for r < returned count (<= k). */
uint32_t orc_greedy_cover(uint32_t n, uint64_t m, const uint64_t *he_off,
                          const uint32_t *he_nodes, uint32_t k,
                          uint32_t *picks, uint64_t *cov_cum);

/* sigma_js in {-1, +1}. */
int orc_rademacher(uint64_t seed, uint32_t instance, uint64_t s, uint32_t j);

/* R[u*t + j] = sum over s < m with u in h_s of sigma_js. */
void orc_rade_sums(uint32_t n, uint64_t m, const uint64_t *he_off,
                   const uint32_t *he_nodes, uint64_t seed, uint32_t instance,
                   uint32_t t, int64_t *R);

/* AMCERA ingredients.  topk_sum[j] = sum of the min(k, #positive) largest
 * positive R[.][j]; deg_topk = sum of the k largest deg_H(u); b_max =
 * max |h|.  Returns the AMCERA = sum_j topk_sum[j] / (t*m). */
double orc_mcera(uint32_t n, uint64_t m, const uint64_t *he_off,
                 const uint32_t *he_nodes, uint64_t seed, uint32_t instance,
                 uint32_t t, uint32_t k, int64_t *topk_sum,
                 uint64_t *deg_topk, uint32_t *b_max);

/* Theorem bound_dev and the Algorithm 1 stopping condition. */
typedef struct {
    double c_hat;   /* C_H(S) = cov/m */
    double amcera;
    double wimpy;   /* approximate wimpy variance */
    double xi, nu, rtilde, r, eta;
    int certified;
} orc_bound_out;

void orc_bound(uint64_t m, uint64_t cov, int64_t sum_topk, uint32_t t,
               uint64_t deg_topk, uint32_t b_max, double eps, double delta_i,
               orc_bound_out *out);

/* Triangle hyperedges (Sec. 3.1: for the triangle centrality the space is
 * the node sets of the triangles of an undirected G, drawn uniformly).
 * Reading: the triangles {a < b < c} are ranked 0 .. T-1 in lexicographic
 * order of (a, b, c); sample number x draws r = bounded(T) from the Philox
 * stream (seed, x, instance, tag 5) and is the r-th triangle, hyperedge
 * (a, b, c).  orc_triangles writes the first min(T, cap) triangles in rank
 * order (3 ids each) and returns T; UINT64_MAX for a directed graph. */
/* The triangles {a < b < c} whose smallest node is a, in rank order (the
 * slice of orc_triangles' list for row a): writes the first min(count, cap). */
uint64_t orc_row_triangles(const orc_graph *g, uint32_t a, uint32_t *tri, uint64_t cap);
uint64_t orc_triangles(const orc_graph *g, uint32_t *tri, uint64_t cap);

/* Samples [first, first+count) triangle hyperedges: he_off[i] = 3i,
 * he_nodes holds 3*count ids.  Returns 0, or -1 for a directed graph or one
 * without triangles. */
int orc_sample_triangles(const orc_graph *g, uint64_t seed, uint32_t instance,
                         uint64_t first, uint64_t count, uint64_t *he_off,
                         uint32_t *he_nodes);

/* samplingSchedule of Algorithm 1 (Section 4).  Geometric (schedule 0):
 * min(ceil(m_i*num/den), m_max).  Adaptive (schedule 1): the larger of
 * that and the optimistic size, the m at which eta of Theorem bound_dev
 * with R = 0 and nu = 1 (sqrt(2L/m) + L/(3m), L = ln(5/delta_next)) equals
 * eps*c_hat/(1-1/e), rounded up and capped at m_max; c_hat = 0 gives no
 * optimistic size. */
uint64_t orc_next_sample_size(uint64_t m_i, double c_hat, double eps, double delta_next,
                              uint32_t growth_num, uint32_t growth_den, uint64_t m_max,
                              uint32_t schedule);

/* Algorithm 1.  schedule: 0 geometric, 1 adaptive (orc_next_sample_size),
 * 2 fixed: one iteration at m_init whose bound uses delta itself.  space:
 * 0 shortest paths (set betweenness), 1 triangles.  picks
 * has capacity k; m_log (optional) receives m_i of iterations 1 ..
 * min(iterations, m_log_cap).  Returns 0 if certified, 1 if not (m_max
 * reached, or the fixed iteration's test failed), negative on error. */
typedef struct {
    uint32_t n_picked, iterations;
    int certified;
    uint64_t coverage, m_final;
    double c_hat, amcera, wimpy, xi, nu, rtilde, r, eta;
} orc_result;

/* kappa-path hyperedges (Sec. 3.1; the sampler is a reading, see the C
 * file): orc_kpath writes sample `sample`'s walk after its start into h (at
 * most kappa ids), returns its length, and reports the start and the drawn
 * length l if asked.  orc_sample_kpaths: samples [first, first+count) into
 * he_off[count+1] / he_nodes (capacity count * kappa); -1 if kappa == 0. */
uint32_t orc_kpath(const orc_graph *g, uint32_t kappa, uint64_t seed, uint32_t instance,
                   uint64_t sample, uint32_t *h, uint32_t *s_out, uint32_t *l_out);
int orc_sample_kpaths(const orc_graph *g, uint32_t kappa, uint64_t seed, uint32_t instance,
                      uint64_t first, uint64_t count, uint64_t *he_off, uint32_t *he_nodes);

/* VC-dimension bounds of Sec. 4.3 for hyperedges of at most b nodes, k
 * picks and n nodes: d1 (Lemma vcboundgeneral), the bound of Lemma
 * lemmavckbound on VC(Q_k), and the union bound floor(k log2 n).
 * Returns 0, or -1 if b, k or n is 0. */
int orc_vc_dims(uint64_t b, uint32_t k, uint64_t n, uint32_t *d1, uint64_t *dk_lemma, uint64_t *dk_union);

/* space: 0 shortest paths, 1 triangles, 2 kappa-paths (kappa >= 1). */
/* HEDGE-P's bound (reading R17): ln of the number of node sets of at most
 * k nodes, and eta^UB with its stopping rule (o->eta, o->c_hat and
 * o->certified are set; the other fields are 0). */
double orc_log_sets(uint64_t n, uint32_t k);
void orc_hedge_bound(uint64_t m, uint64_t cov, uint64_t n, uint32_t k, double eps, double delta_i,
                     orc_bound_out *o);

int orc_progressive(const orc_graph *g, uint32_t c_bits, uint32_t k, uint32_t t,
                    double eps, double delta, uint64_t seed, uint32_t instance,
                    uint64_t m_init, uint64_t m_max, uint32_t growth_num,
                    uint32_t growth_den, uint32_t schedule, uint32_t space, uint32_t kappa,
                    uint32_t method, uint32_t *picks, orc_result *res, uint64_t *m_log,
                    uint32_t m_log_cap);   /* method 0: CentRA; 1: HEDGE-P (reading R17) */

#ifdef __cplusplus
}
#endif

#endif
