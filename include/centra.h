/*
 * centra.h -- C ABI of the MI355X (gfx950) implementation of the CentRA hot
 * path: progressive-sampling set-betweenness centrality maximisation with
 * Monte-Carlo Rademacher bounds (L. Pellegrina, "Efficient Centrality
 * Maximization with Rademacher Averages", KDD 2023, arXiv 2306.03651).
 *
 * Conventions (all entry points):
 *   - Plain C types only.  Pointers documented "device" are HIP device
 *     pointers (e.g. from torch.empty(..., device="cuda")); "host" pointers
 *     are ordinary memory.  The caller owns every buffer it passes and keeps
 *     it alive until the call returns.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *     Every entry point enqueues its work on `stream` and synchronises
 *     `stream` before returning, so outputs are ready on return -- except
 *     the stream-ordered calls (centra_sample_paths_append, centra_extend),
 *     which only enqueue: their outputs are ready when `stream` reaches
 *     them, and their device-side errors are reported by centra_check.
 *   - Return codes: CENTRA_OK (0) on success, CENTRA_NOT_CERTIFIED (1) from
 *     centra_progressive when the sample cap is reached, negative on error.
 *     The text of the last error is available from centra_last_error().  No
 *     C++ exception crosses this boundary.
 *   - A context is not thread safe: use one per host thread.  Work of one
 *     context runs on the HIP device given at creation.
 *   - Randomness is counter based: for the same (seed, instance) every
 *     hyperedge, Rademacher sign and result is a pure function of the
 *     inputs, independent of launch shape, batch split or timing.
 */
#ifndef CENTRA_H
#define CENTRA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#if defined(__GNUC__)
#define CENTRA_API __attribute__((visibility("default")))
#else
#define CENTRA_API
#endif

#define CENTRA_ABI_VERSION 11u

#define CENTRA_OK 0
#define CENTRA_NOT_CERTIFIED 1
#define CENTRA_STOPPED 2     /* centra_progressive_resumable stopped where asked */
#define CENTRA_EINVAL (-1)   /* invalid argument or malformed input */
#define CENTRA_ENOMEM (-2)   /* the context's HBM budget or the device is exhausted */
#define CENTRA_EHIP (-3)     /* HIP runtime error (text in centra_last_error) */
#define CENTRA_ENOSPC (-4)   /* a caller output buffer is too small */
#define CENTRA_ENOTSUP (-5)  /* unsupported configuration */

typedef struct centra_ctx centra_ctx;
typedef struct centra_graph centra_graph;

/* Returns CENTRA_ABI_VERSION of the built library. */
CENTRA_API uint32_t centra_abi_version(void);

/* Creates a context on HIP device `hip_device`.  `hbm_budget_bytes` bounds
 * the device memory the context allocates for its own workspaces (0 = no
 * bound beyond the device).  The sampler's per-BFS state is sized for as
 * many concurrent BFSs as the device runs, up to half of the device's
 * memory; with several contexts on one device, give each a budget.
 * Contexts are independent: different contexts may be used from different
 * host threads at the same time.  *out receives the context.
 * Placement: the sampler's speed depends on where the device allocator puts
 * the pages of that state's per-BFS node records (the same launch varies
 * by up to ~18% from one allocation to the next, and not within one).
 * When a synchronous sampling call first allocates at least 4 GiB of
 * records on a context, the context times a launch of the call's first
 * 65,536 work items on each of up to four allocations of them, holding two
 * at a time, and keeps the fastest; it stops once a step takes more than
 * 60 ms (a slow probe, or memory the device must clear first).  Results do
 * not depend on it.  The environment variable CENTRA_SLOT_SEARCH=0
 * turns this off; centra_context_log reports the times.  (Tests only:
 * the environment variable CENTRA_STAMP_START sets the context's first BFS
 * stamp, to exercise the sampler's 32-bit stamp wrap.)
 * Errors: CENTRA_EINVAL (out == NULL), CENTRA_EHIP (no such device). */
CENTRA_API int centra_create(int hip_device, size_t hbm_budget_bytes, centra_ctx **out);

/* Frees the context and every workspace it owns.  NULL is allowed. */
CENTRA_API void centra_destroy(centra_ctx *ctx);

/* Text of the last error reported on `ctx` ("" if none).  Valid until the
 * next call on ctx.  With ctx == NULL, the last error of a call without a
 * context (centra_create, centra_greedy_cover_noalloc) on this host thread. */
CENTRA_API const char *centra_last_error(const centra_ctx *ctx);

/* The context's log of one-time choices, one line each (the slot placement
 * search: each allocation's probe time and the one kept); "" if none or if
 * ctx == NULL.  Valid until the next call on ctx. */
CENTRA_API const char *centra_context_log(const centra_ctx *ctx);

/* ------------------------------------------------------------------ */
/* Graph G = (V, E) of the problem statement (Algorithm 1 input; Sec. 3.1),
 * in CSR form, device pointers, caller owned:
 *   row_ptr[n+1], col_idx[n_arcs]: out-neighbours of each node; rows sorted
 *     ascending; no duplicate arcs; no self loops; n_arcs < 2^32.
 *   rrow_ptr, rcol_idx: in-neighbours in the same form for a directed graph
 *     (directed = 1); NULL for an undirected graph (directed = 0), whose
 *     arcs come in both directions and whose in-rows are its out-rows. */
typedef struct {
    uint32_t n;
    uint32_t directed;
    uint64_t n_arcs;
    const uint32_t *row_ptr;
    const uint32_t *col_idx;
    const uint32_t *rrow_ptr;
    const uint32_t *rcol_idx;
} centra_csr;

/* Validates the CSR on the device and prepares the graph for sampling: the
 * maximum in-degree and the bit budget C = 63 - bitlen(max in-degree) of
 * the normalised shortest-path counts.  `count_bits_override`, if nonzero
 * and smaller than C, replaces C (tests only).  The CSR arrays must stay
 * alive until centra_graph_release.  *out receives the prepared graph.
 * Preparation also builds, in context memory, a relabelled copy of the
 * graph whose node order groups each node with its in-neighbour of largest
 * out-degree, so that nodes visited together by a BFS have nearby ids (the
 * sampler traverses that copy; every result is expressed in the caller's
 * ids and does not depend on the relabelling).  The environment variable
 * CENTRA_RELABEL=0 makes the sampler traverse the caller's CSR instead.
 * Errors: CENTRA_EINVAL (n < 2, unsorted row, duplicate, self loop, node id
 * out of range, inconsistent reverse CSR), CENTRA_ENOMEM, CENTRA_EHIP. */
CENTRA_API int centra_graph_prepare(centra_ctx *ctx, const centra_csr *csr, uint32_t count_bits_override,
                         centra_graph **out, void *stream);

/* Releases a prepared graph (not the caller's CSR arrays) and the context
 * memory it holds; call it before destroying its context.  NULL is allowed. */
CENTRA_API void centra_graph_release(centra_graph *g);

/* Host outputs: maximum in-degree and count bit budget C of the graph. */
CENTRA_API int centra_graph_info(const centra_graph *g, uint32_t *max_in_degree, uint32_t *count_bits);

/* Host output: a 64-bit fingerprint of the caller's graph, computed when
 * it was prepared: mix(n | directed << 32) + the sum over the arcs u -> v
 * of the out-CSR of mix(u << 32 | v), modulo 2^64, where mix is the
 * splitmix64 output function (z ^= z >> 30; z *= 0xBF58476D1CE4E5B9;
 * z ^= z >> 27; z *= 0x94D049BB133111EB; z ^= z >> 31).  Checkpoints
 * carry it. */
CENTRA_API int centra_graph_hash(const centra_graph *g, uint64_t *hash);

/* ------------------------------------------------------------------ */
/* sampleHEs for set betweenness (Algorithm 1 sampling step; hyperedge space
 * of Sec. 3.1; procedure of Sec. 5 with a single BFS from s instead of the
 * bidirectional BFS).  Draws samples [first_sample, first_sample + count)
 * of (seed, instance).  Sample number x: Philox4x64-10 stream with key
 * (seed, 0) and counter (block, x, instance, 0); s = bounded(n), t' =
 * bounded(n-1), t = t' + [t' >= s] (Lemire bounded draws); BFS from s with
 * normalised path counts up to t's level; a uniformly random shortest s-t
 * path by backtracking from t; the hyperedge is its internal nodes, t's
 * neighbour first (empty if t is unreachable or adjacent to s).
 *   he_off     device u64[count+1]: he_off[i] = offset of sample
 *              first_sample+i in he_nodes, he_off[0] = 0.
 *   he_nodes   device u32[he_cap]: node ids, sample after sample.
 *   he_needed  host u64 (may be NULL): receives he_off[count].
 *   st_out     optional device u32[2*count]: (s, t) of each sample.
 *   dist_out   optional device u32[count]: d(s,t), 0xFFFFFFFF if
 *              unreachable.
 * Errors: CENTRA_ENOSPC if he_cap < he_off[count] (then he_off is written
 * and *he_needed set; call again with a larger buffer), CENTRA_EINVAL,
 * CENTRA_ENOMEM, CENTRA_EHIP.
 * The environment variable CENTRA_SAMPLER_VARIANT selects another launch
 * shape of the sampling kernel, for tests: "lds" (an exact LDS visited
 * bitmap, 1024 threads, when it fits), "hbm512", "hbm256", "hbm128" (the
 * default) or "hbm64" (that many threads per BFS).  Results are the same. */
CENTRA_API int centra_sample_paths(centra_ctx *ctx, const centra_graph *g, uint64_t seed, uint32_t instance,
                        uint64_t first_sample, uint32_t count, uint64_t *he_off, uint32_t *he_nodes,
                        uint64_t he_cap, uint64_t *he_needed, uint32_t *st_out, uint32_t *dist_out,
                        void *stream);

/* sampleHEs for set betweenness by the balanced bidirectional search of
 * Sec. 5: the same hyperedge space and the same distribution (a uniform
 * ordered pair, then a uniformly random shortest path) as
 * centra_sample_paths, drawn from its own stream: Philox4x64-10 with key
 * (seed, 0) and counter (block, x, instance, 7); s, t as above; a search
 * from s over out-arcs and one from t over in-arcs, each level with
 * normalised counts (the forward budget C as above, the backward budget
 * 63 - bitlen(max out-degree); a count_bits_override lowers both), each
 * step expanding the side whose last level has fewer arcs to scan (the
 * forward side on ties); at the first level that meets the other side's
 * last level, a meeting node is drawn in ascending id with weight
 * sigma_f * sigma_b (the 128-bit product shifted so that the weights sum
 * below 2^63, clamped to >= 1), then the path is walked to t over the
 * backward counts (successors in row order) and to s over the forward
 * counts (predecessors in row order), one draw per step above level 1.
 * Arguments, outputs and errors as centra_sample_paths.  Its slot state is
 * 40 bytes per node per concurrent search. */
CENTRA_API int centra_sample_paths_bidir(centra_ctx *ctx, const centra_graph *g, uint64_t seed, uint32_t instance,
                              uint64_t first_sample, uint32_t count, uint64_t *he_off, uint32_t *he_nodes,
                              uint64_t he_cap, uint64_t *he_needed, uint32_t *st_out, uint32_t *dist_out,
                              void *stream);

/* greedyCover(k, H) (Sec. 3.1 greedy algorithm; Algorithm 1 greedy step):
 * k rounds; each adds the node covering the most not-yet-covered
 * hyperedges, lowest node id on ties, and stops early once that number is
 * 0.  The sample H is given as m hyperedges:
 *   he_off   device u64[m+1], he_off[0] = 0, non-decreasing;
 *   he_nodes device u32[he_off[m]], node ids < n, distinct within one
 *            hyperedge.
 * Outputs (device): picks u32[k], cov_cum u64[k] (hyperedges covered after
 * r+1 picks), n_picked u32[1] (entries written, <= k).
 * Errors: CENTRA_EINVAL (k == 0, n == 0, node id >= n), CENTRA_ENOMEM,
 * CENTRA_EHIP. */
CENTRA_API int centra_greedy_cover(centra_ctx *ctx, uint32_t n, uint64_t m, const uint64_t *he_off,
                        const uint32_t *he_nodes, uint32_t k, uint32_t *picks, uint64_t *cov_cum,
                        uint32_t *n_picked, void *stream);

/* centra_greedy_cover for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same inputs, outputs and results as centra_greedy_cover, on
 * the current HIP device and without a context; it calls no hipMalloc,
 * hipFree or other allocating routine.  Its workspaces (the incidence of
 * the sample, gains, the covered bitmap, round state) are carved from a
 * fixed array of CENTRA_NOALLOC_SCRATCH_BYTES in device memory that each
 * GPU the library runs on holds until the process ends.  The sizes must
 * fit it: about 28 n + 8 I + m / 8 + 16 k bytes (I = he_off[m], the
 * hyperedge entries), else CENTRA_ENOSPC with the sizes in
 * centra_last_error(NULL).  All calls on one GPU share that array: calls
 * that overlap on one GPU (two host threads, or two streams in flight)
 * race and give wrong results; serialise them.  Synchronises `stream`
 * before returning (it reads he_off[m] and the error word).
 * Errors: CENTRA_EINVAL (k == 0, n == 0, NULL pointer, node id >= n),
 * CENTRA_ENOTSUP (m >= 2^31), CENTRA_ENOSPC, CENTRA_EHIP. */
#define CENTRA_NOALLOC_SCRATCH_BYTES (64u << 20)
CENTRA_API int centra_greedy_cover_noalloc(uint32_t n, uint64_t m, const uint64_t *he_off, const uint32_t *he_nodes,
                                uint32_t k, uint32_t *picks, uint64_t *cov_cum, uint32_t *n_picked, void *stream);

/* AMCERA ingredients (Sec. 4.1 definitions of the AMCERA and the
 * approximate wimpy variance; Algorithm 1 AMCERA steps).  The sample is
 * given as for centra_greedy_cover; hyperedge i is sample number i.
 * sigma_ji = +1 iff bit (j mod 64) of word ((j mod 256) div 64) of the
 * Philox4x64-10 block with key (seed, 0) and counter (j div 256, i,
 * instance, 1) is set, else -1.  R[u][j] = sum over i with u in h_i of
 * sigma_ji (= m * r_j^u).
 * Outputs (device):
 *   topk_sum     i64[t]: sum of the min(k, #positive) largest positive
 *                R[.][j] (= m * r_j of Algorithm 1);
 *   deg_topk_sum u64[1]: sum of the k largest deg_H(u);
 *   b_max        u32[1]: max |h_i|;
 *   R_out        optional i32[n*t], R[u][j] at u*t + j.
 * AMCERA = sum_j topk_sum[j] / (t m); wimpy = b_max * deg_topk_sum / m.
 * Errors: CENTRA_EINVAL (t == 0 or t > 1024, k == 0, n == 0, m == 0,
 * m >= 2^31, node id >= n), CENTRA_ENOMEM, CENTRA_EHIP. */
CENTRA_API int centra_mcera(centra_ctx *ctx, uint32_t n, uint64_t m, const uint64_t *he_off,
                 const uint32_t *he_nodes, uint64_t seed, uint32_t instance, uint32_t t, uint32_t k,
                 int64_t *topk_sum, uint64_t *deg_topk_sum, uint32_t *b_max, int32_t *R_out,
                 void *stream);

/* ------------------------------------------------------------------ */
/* Stream-ordered calls.  They read nothing back to the host: the sizes
 * they need come from the caller (capacities), the sizes they produce stay
 * in device memory, and errors found on the device are raised into the
 * context's error word for centra_check.  A call may still wait for the
 * device when it has to grow one of the context's workspaces (allocation);
 * centra_reserve grows them ahead so that the calls after it only enqueue.
 * Calls on one context must be issued on one stream (or ordered by the
 * caller), as they share the context's workspaces. */

/* sampleHEs into a growing hyperedge store (Algorithm 1 sampling step; the
 * hyperedge space and the draws of centra_sample_paths, same results).
 * Samples [first_sample, first_sample + count) of (seed, instance) are
 * appended to the store after the entries already in it:
 *   he_off     device u64[count+1]: the store's offsets from the first new
 *              sample on (the caller passes store_off + first index);
 *              he_off[0] must hold the store's current size (entries) when
 *              the stream reaches the call (0 for an empty store); he_off[i]
 *              for i >= 1 receives the offset after new sample i-1.
 *   he_nodes   device u32[he_cap]: the whole store.
 *   he_total   device u64[1] (may be NULL): receives the store's new size,
 *              he_off[0] + entries of the new samples.
 * If the new size exceeds he_cap the new samples are stored as empty
 * hyperedges (he_off[i] = he_off[0]: the store stays consistent), *he_total
 * still receives the size they need, and centra_check reports
 * CENTRA_ENOSPC; the caller then grows the store and draws them again.
 * Not counted in centra_sampler_stats.  The staging area it uses holds
 * he_cap entries.
 * Errors (returned): CENTRA_EINVAL (NULL ctx, graph, he_off, or he_nodes
 * with he_cap > 0), CENTRA_ENOMEM, CENTRA_EHIP. */
CENTRA_API int centra_sample_paths_append(centra_ctx *ctx, const centra_graph *g, uint64_t seed, uint32_t instance,
                               uint64_t first_sample, uint32_t count, uint64_t *he_off, uint32_t *he_nodes,
                               uint64_t he_cap, uint64_t *he_total, void *stream);

/* One iteration's greedy and AMCERA steps on a sample that grows between
 * calls (Algorithm 1: greedyCover on the sample, then the AMCERA and the
 * wimpy-variance ingredients of Sec. 4.1), stream-ordered and incremental:
 * the context keeps the incidence of the store and the AMCERA counts, and
 * a call adds only the samples after m_prev.  Results equal those of
 * centra_greedy_cover and centra_mcera on samples [0, m). */
typedef struct {
    uint32_t n;                 /* nodes; every node id < n */
    uint32_t k;                 /* greedy rounds and top-k size, >= 1 */
    uint64_t m_prev;            /* samples [0, m_prev) of the store are unchanged since
                                   the previous centra_extend on this context (0: none
                                   are; the state is rebuilt) */
    uint64_t m;                 /* samples in the store now, 0 < m < 2^31, m >= m_prev */
    const uint64_t *he_off;     /* device u64[m+1]: the store's offsets, he_off[0] = 0,
                                   non-decreasing */
    const uint32_t *he_nodes;   /* device u32[he_cap]: the store's node ids */
    uint64_t he_cap;            /* entries he_nodes holds; he_off[m] must not exceed it
                                   (else the incidence is left empty and centra_check
                                   reports CENTRA_ENOSPC) */
    /* greedyCover outputs (device, as centra_greedy_cover); all NULL: skipped */
    uint32_t *picks;            /* u32[k] */
    uint64_t *cov_cum;          /* u64[k] */
    uint32_t *n_picked;         /* u32[1] */
    /* AMCERA (as centra_mcera); t = 0: skipped */
    uint32_t t;                 /* trials, <= 1024 */
    uint32_t instance;
    uint64_t seed;
    int64_t *topk_sum;          /* device i64[t] */
    uint64_t *deg_topk_sum;     /* device u64[1] */
    uint32_t *b_max;            /* device u32[1]: max |h_i| over samples [0, m) */
    int32_t *R_out;             /* optional device i32[n*t] */
} centra_extend_args;

/* Runs the steps of *a on `stream` without synchronising it.  State kept
 * from the previous call is reused when this call names the same store
 * (he_off, he_nodes, he_cap and n equal), m_prev covers what the state
 * holds, and, for the AMCERA, (seed, instance, t) are unchanged; otherwise
 * it is rebuilt from sample 0 (same results, more work).  Any other call
 * on the context that builds an incidence or AMCERA counts
 * (centra_greedy_cover, centra_mcera, centra_progressive) ends that state.
 * Errors (returned): CENTRA_EINVAL (NULL ctx or a, n == 0, k == 0, m == 0,
 * m < m_prev, NULL store pointers, greedy outputs partly NULL, t > 1024,
 * NULL AMCERA outputs with t > 0), CENTRA_ENOTSUP (m >= 2^31),
 * CENTRA_ENOMEM, CENTRA_EHIP.  Device-side: node ids >= n and decreasing
 * offsets (CENTRA_EINVAL), he_off[m] > he_cap (CENTRA_ENOSPC), reported
 * by centra_check. */
CENTRA_API int centra_extend(centra_ctx *ctx, const centra_extend_args *a, void *stream);

/* Grows the context's workspaces for stream-ordered calls up to the given
 * sizes, so that those calls only enqueue: sampling batches of up to
 * `batch` samples of graph g (NULL: no sampling) into a store of he_cap
 * entries, and centra_extend on n nodes, up to m_max samples, k picks, t
 * trials and 16 incidence segments (a longer run of extensions, or a
 * rebuild after 64 segments, may grow a workspace again).  Synchronises
 * `stream`.
 * Errors: CENTRA_EINVAL (NULL ctx, n == 0, g's node count != n,
 * t > 1024), CENTRA_ENOMEM, CENTRA_EHIP. */
CENTRA_API int centra_reserve(centra_ctx *ctx, const centra_graph *g, uint32_t n, uint32_t batch, uint64_t m_max,
                   uint64_t he_cap, uint32_t k, uint32_t t, void *stream);

/* Waits for `stream` and reports the errors that kernels of this context
 * raised since the last check (the stream-ordered calls' device-side
 * errors), clearing them: CENTRA_OK if none, else CENTRA_ENOSPC (only a
 * store capacity was exceeded), CENTRA_EINVAL (malformed input) or
 * CENTRA_EHIP, with the text in centra_last_error. */
CENTRA_API int centra_check(centra_ctx *ctx, void *stream);

/* Work and time of the sampling kernel, accumulated over every sampling
 * launch of the context since the last reset: centra_sample_paths and the
 * sampling steps of centra_progressive on either hyperedge space (the
 * triangle sampler's launches count only inside centra_progressive, which
 * synchronises anyway; for them arcs and nodes stay 0 and slots is 0).
 * kernel_ms is measured with HIP events recorded on the launch stream
 * immediately around each launch.
 * arcs counts every CSR entry the kernel scans (level expansions, the
 * checks around t, the backtrack is not included); nodes counts every node
 * given a level.  A re-launch after a staging overflow counts again.
 * Wide samples: a BFS about to expand a level of more than 65,536 nodes,
 * or a level of at least 4,096 nodes after scanning more than 2^21 CSR
 * entries (a flood of a skewed graph's reachable set; long narrow searches
 * such as grids stay), is handed from its workgroup to a device-wide BFS that redraws the sample level by level
 * with the whole GPU (same hyperedge).  kernel_ms, arcs and nodes stay
 * those of the workgroup kernel (a handed-over BFS's partial work
 * included); `wide` counts such samples, wide_ms is the wall time of their
 * device-wide BFSs (launches and the per-level synchronisation) and
 * wide_arcs the CSR entries those scanned (full levels).  Only the
 * synchronous single-graph launches do this (CENTRA_WIDE=0 turns it off;
 * tests only: CENTRA_WIDE_NODES lowers the level size that triggers it). */
typedef struct {
    uint64_t launches;
    double kernel_ms;
    uint64_t samples;
    uint64_t arcs;
    uint64_t nodes;
    uint64_t hyperedge_nodes;
    uint32_t lds_bitmap;   /* 1 if the last launch kept the visited bitmap in LDS */
    uint32_t slots;        /* workgroups (concurrent BFSs) of the last launch */
    uint64_t wide;         /* samples finished by the device-wide BFS */
    double wide_ms;
    uint64_t wide_arcs;
} centra_sampler_stats;

/* Copies the statistics to *out (host) and, if reset != 0, zeroes them. */
CENTRA_API int centra_sampler_stats_get(centra_ctx *ctx, centra_sampler_stats *out, int reset);

/* ------------------------------------------------------------------ */
/* Theorem bound_dev (eq. epsrade) with xi and the stopping condition of
 * Algorithm 1, in FP64 on the host:  a = 1 - 1/e, L = ln(5/delta_i),
 * C = cov/m, AMCERA = sum_topk/(t m), wimpy = b_max*deg_topk/m,
 * xi = sqrt((L/m)^2 + 2CL/(a m)) + L/m, nu = C/a + xi,
 * R~ = AMCERA + sqrt(4 wimpy L/(t m)), R = R~ + sqrt((L/m)^2 + 2L R~/m) + L/m,
 * eta = 2R + sqrt(2L(nu + 4R)/m) + L/(3m);
 * certified = a((a - eps) xi + eta) <= eps C.  All pointers host. */
typedef struct {
    double c_hat, amcera, wimpy, xi, nu, rtilde, r, eta;
    int certified;
} centra_bound_out;

/* Errors: CENTRA_EINVAL (m == 0, t == 0, delta_i outside (0,1), out NULL). */
CENTRA_API int centra_bound(uint64_t m, uint64_t cov, int64_t sum_topk, uint32_t t, uint64_t deg_topk,
                 uint32_t b_max, double eps, double delta_i, centra_bound_out *out);

/* HEDGE-P's bound (Sec. 5 describes HEDGE-P as Algorithm 1's iterations
 * with a union bound eta^UB in place of the AMCERA and HEDGE's stopping
 * rule SD <= eps C(S*) / 2; the paper does not print eta^UB, so this form is
 * this library's): with N_k = sum_{j <= k} C(n, j) node sets of at most k
 * nodes, Hoeffding's two-sided inequality and a union bound at confidence
 * delta_i give eta^UB = sqrt((ln(2 N_k) + ln(1 / delta_i)) / (2 m));
 * C(S*) >= C_H(S) - eta^UB on that event, so the rule holds once
 * eta^UB <= eps (C_H(S) - eta^UB) / 2 (out->certified).  ln N_k is summed
 * in FP64 from lgamma terms.  Writes out->c_hat = cov / m, out->eta and
 * out->certified; the other fields are 0.  Host only.
 * Errors: CENTRA_EINVAL (m, n or k is 0, delta_i outside (0,1), out NULL). */
CENTRA_API int centra_hedge_bound(uint64_t m, uint64_t cov, uint64_t n, uint32_t k, double eps, double delta_i,
                       centra_bound_out *out);

/* VC-dimension bounds of Sec. 4.3 for the range space Q_k (ranges: the
 * hyperedges met by a node set of at most k nodes), host only:
 *   d1       = floor(log2(2b)) >= VC(Q_1) when every hyperedge of the space
 *              has at most b nodes (Lemma vcboundgeneral; b = 3 for
 *              triangles, b <= kappa for kappa-paths, the vertex diameter
 *              for shortest paths);
 *   dk_lemma = floor(2 d1 k log2(3k)) >= VC(Q_k) (Lemma lemmavckbound);
 *   dk_union = floor(k log2 n) >= VC(Q_k) (the union bound);
 *   dk       = min(dk_lemma, dk_union).
 * The sample sizes of Theorem vcsamplecomplexity follow from dk only up to
 * a constant the paper does not give, so none is derived here.
 * Errors: CENTRA_EINVAL (b, k or n is 0, out NULL). */
typedef struct {
    uint32_t d1;
    uint64_t dk_lemma, dk_union, dk;
} centra_vc_out;
CENTRA_API int centra_vc_dims(uint64_t b, uint32_t k, uint64_t n, centra_vc_out *out);

/* ------------------------------------------------------------------ */
/* Triangle hyperedges: the hyperedge space of the triangle centrality
 * (Sec. 3.1: the node sets of the triangles of an undirected G, drawn
 * uniformly), the second space Algorithm 1 runs on (Sec. 4: the algorithm
 * is oblivious to sampleHEs).  The triangles {a < b < c} are ranked in
 * lexicographic order of (a, b, c); sample number x (global index) draws
 * r = bounded(T) from the Philox stream (seed, x, instance, tag 5) and is
 * the triangle of rank r, hyperedge (a, b, c).
 *
 * centra_triangle_count: *T receives the number of triangles (host).  The
 * per-graph triangle index is built on first use and kept with g: 12 bytes
 * per arc, plus 4 bytes per triangle for the ranked list of every
 * triangle's largest node when that list fits in an eighth of device memory
 * (samples then read it; otherwise each sample walks its arc's common
 * neighbours; CENTRA_TRIANGLE_LIST=0 in the environment forces the walk).
 * centra_sample_triangles: samples [first, first + count) into he_off
 * (device u64[count + 1], he_off[i] = 3 i) and he_nodes (device u32[3 count]).
 * Errors: CENTRA_ENOTSUP (directed graph), CENTRA_EINVAL (NULL argument;
 * sampling from a graph without triangles), CENTRA_ENOMEM, CENTRA_EHIP. */
CENTRA_API int centra_triangle_count(centra_ctx *ctx, const centra_graph *g, uint64_t *T, void *stream);
CENTRA_API int centra_sample_triangles(centra_ctx *ctx, const centra_graph *g, uint64_t seed, uint32_t instance,
                            uint64_t first, uint32_t count, uint64_t *he_off, uint32_t *he_nodes,
                            void *stream);

/* ------------------------------------------------------------------ */
/* kappa-path hyperedges: the hyperedge space of the kappa-path centrality
 * (Sec. 3.1: the node sets of simple paths of length at most kappa), a third
 * space for Algorithm 1 (Sec. 4: the algorithm is oblivious to sampleHEs).
 * The paper gives no sampler; sample number x (global index) is the random
 * simple walk of the kappa-path centrality, drawn from the Philox stream
 * (seed, x, instance, tag 6): start s = bounded(n), length
 * l = 1 + bounded(kappa), then l moves, each from the current node v to the
 * r-th (r = bounded(f)) of v's f out-neighbours not yet on the walk in
 * ascending id, stopping early when f = 0.  The hyperedge is the walk after
 * s: at most kappa nodes (b <= kappa, Sec. 4.3), in walk order.
 *
 * centra_sample_kpaths: samples [first, first + count) into he_off (device
 * u64[count + 1], relative to he_nodes) and he_nodes (device u32, capacity
 * count * kappa).  1 <= kappa <= CENTRA_MAX_KAPPA.  Synchronous.
 * Errors: CENTRA_EINVAL (NULL argument, kappa outside [1, 16]),
 * CENTRA_ENOMEM, CENTRA_EHIP. */
#define CENTRA_MAX_KAPPA 16u
CENTRA_API int centra_sample_kpaths(centra_ctx *ctx, const centra_graph *g, uint32_t kappa, uint64_t seed,
                         uint32_t instance, uint64_t first, uint32_t count, uint64_t *he_off,
                         uint32_t *he_nodes, void *stream);

/* ------------------------------------------------------------------ */
/* Algorithm 1 (CentRA).  Iteration i = 1, 2, ...: delta_i = delta / 2^i;
 * the sample is extended to m_i hyperedges (samples 0 .. m_i-1 of (seed,
 * instance)), then greedyCover, the AMCERA and the bound of Theorem
 * bound_dev; returns as soon as the stopping condition holds.  The sample
 * schedule (procedure samplingSchedule of Algorithm 1, Section 4):
 *   CENTRA_SCHEDULE_GEOMETRIC: m_1 = m_init,
 *     m_{i+1} = min(ceil(m_i * growth_num / growth_den), m_max);
 *   CENTRA_SCHEDULE_ADAPTIVE: the geometric step combined with the paper's
 *     optimistic guess, m_{i+1} = min(max(geometric step, m_opt), m_max),
 *     where m_opt = ceil(m) for the m > 0 solving
 *     sqrt(2 L / m) + L / (3 m) = eps * C_i / (1 - 1/e), i.e. eta of
 *     Theorem bound_dev with R = 0 and nu = 1 set equal to the largest
 *     value the stopping condition can accept; L = ln(5 / delta_{i+1}),
 *     C_i = coverage_i / m_i of the iteration just finished (m_opt = 0
 *     when C_i = 0); growth_num / growth_den = 6 / 5 is the paper's 1.2;
 *   CENTRA_SCHEDULE_FIXED: a single iteration at m = m_init whose bound
 *     uses delta itself (the fixed-sample-size use of Theorem bound_dev,
 *     Section 5), returning its stopping test.
 * The hyperedge space: CENTRA_SPACE_SHORTEST_PATHS (set betweenness,
 * centra_sample_paths), CENTRA_SPACE_TRIANGLES (triangle centrality,
 * centra_sample_triangles) or CENTRA_SPACE_KPATHS (kappa-path centrality,
 * centra_sample_kpaths with the params' kappa; kappa is ignored otherwise)
 * or CENTRA_SPACE_PATHS_BIDIR (set betweenness, centra_sample_paths_bidir).
 * The method: CENTRA_METHOD_CENTRA (the AMCERA and the bound of Theorem
 * bound_dev, the stopping condition of Algorithm 1) or
 * CENTRA_METHOD_HEDGE_P, the comparison method of Sec. 5: the same
 * iterations with the union bound of centra_hedge_bound in place of the
 * AMCERA (t is then unused) and its stopping rule; the result's eta is
 * eta^UB and its AMCERA fields are 0.
 * Inputs: k >= 1, 1 <= t <= 1024, eps in (0, 1-1/e), delta in (0,1),
 * 1 <= m_init <= m_max < 2^31, growth_num > growth_den >= 1, schedule and
 * space one of their values, 1 <= kappa <= CENTRA_MAX_KAPPA for
 * CENTRA_SPACE_KPATHS.
 * Work per iteration: only the new samples are drawn, and only their
 * entries are added to the node -> sample incidence (one segment per
 * iteration, at most 64 before one is rebuilt from sample 0) and to the
 * per-node Rademacher counts (the incremental computation of Section 4);
 * greedy and the per-trial top-k then run over the whole sample.
 * Synchronous: one host synchronisation per iteration. */
#define CENTRA_SCHEDULE_GEOMETRIC 0u
#define CENTRA_SCHEDULE_ADAPTIVE 1u
#define CENTRA_SCHEDULE_FIXED 2u
#define CENTRA_SPACE_SHORTEST_PATHS 0u
#define CENTRA_SPACE_TRIANGLES 1u
#define CENTRA_SPACE_KPATHS 2u
#define CENTRA_SPACE_PATHS_BIDIR 3u   /* shortest paths, bidirectional sampler */
#define CENTRA_METHOD_CENTRA 0u
#define CENTRA_METHOD_HEDGE_P 1u

typedef struct {
    uint32_t k, t;
    double eps, delta;
    uint64_t seed;
    uint32_t instance;
    uint64_t m_init, m_max;
    uint32_t growth_num, growth_den;
    uint32_t schedule;   /* CENTRA_SCHEDULE_* */
    uint32_t space;      /* CENTRA_SPACE_* */
    uint32_t kappa;      /* path length bound of CENTRA_SPACE_KPATHS */
    uint32_t method;     /* CENTRA_METHOD_* */
} centra_params;

typedef struct {
    uint32_t n_picked, iterations;
    int certified;
    uint64_t coverage, m_final;
    double c_hat, amcera, wimpy, xi, nu, rtilde, r, eta;
    double ms_sample, ms_cover, ms_mcera, ms_total;   /* device time per phase, summed */
} centra_result;

/* Per-iteration record (optional log). */
typedef struct {
    uint32_t i;
    uint64_t m;
    uint64_t coverage;
    int64_t sum_topk;
    uint64_t deg_topk;
    uint32_t b_max;
    double delta_i, amcera, wimpy, xi, nu, rtilde, r, eta;
    int certified;
    double ms_sample, ms_cover, ms_mcera;
    uint64_t arcs, nodes;   /* the iteration's sampling work (centra_sampler_stats
                               arcs and nodes; 0 for the triangle and k-path spaces;
                               the first iteration of a resume that redraws the
                               sample counts the redraw too) */
} centra_iteration;

/* picks: host u32[k] (receives result->n_picked entries); result: host.
 * log: optional host array of log_cap records (iteration i goes to
 * log[i-1] while i <= log_cap).
 * Returns CENTRA_OK if certified, CENTRA_NOT_CERTIFIED if m_max was reached
 * first (result and picks still filled), or an error. */
CENTRA_API int centra_progressive(centra_ctx *ctx, const centra_graph *g, const centra_params *params,
                       uint32_t *picks, centra_result *result, centra_iteration *log,
                       uint32_t log_cap, void *stream);

/* Checkpoint of Algorithm 1 after iteration i: everything iteration i + 1
 * depends on.  Samples, Rademacher signs and counts are functions of
 * (graph, seed, instance) and the sample indices, so the sample of m_i
 * hyperedges is redrawn on resume (or kept, on the same context). */
#define CENTRA_CHECKPOINT_VERSION 1u
typedef struct {
    uint32_t version;       /* CENTRA_CHECKPOINT_VERSION */
    uint32_t i;             /* iterations completed, >= 1 */
    uint64_t graph_hash;    /* centra_graph_hash of the graph */
    uint64_t params_hash;   /* centra_params_hash of the parameters */
    uint64_t m_i;           /* samples of iteration i */
    uint64_t m_next;        /* samples of iteration i + 1 (the schedule's state) */
    uint64_t entries;       /* hyperedge entries of samples [0, m_i), checked on resume */
} centra_checkpoint;

/* Host output: FNV-1a (64-bit) over the little-endian bytes of the fields
 * of *params in declaration order (k, t, eps and delta as their IEEE-754
 * bits, seed, instance, m_init, m_max, growth_num, growth_den, schedule,
 * space, kappa, method), each at its own width. */
CENTRA_API int centra_params_hash(const centra_params *params, uint64_t *hash);

/* centra_progressive that can stop and resume (same results as one
 * uninterrupted centra_progressive: picks, coverage, sample sizes, bound
 * values and iteration numbers).
 *   resume      host, may be NULL: start after iteration resume->i, at
 *               m = resume->m_next; its graph and parameter hashes must
 *               match.  On the context that wrote it (no other incidence
 *               or AMCERA build on the context since), the kept sample and
 *               counts are extended; elsewhere samples [0, m_next) are
 *               drawn anew and the entries of [0, m_i) are checked.
 *   ckpt        host, may be NULL: after every iteration that does not end
 *               the run, receives the checkpoint to resume after it.
 *   stop_after  0, or an iteration number: return CENTRA_STOPPED after the
 *               first iteration numbered >= stop_after that does not end
 *               the run (result, picks and *ckpt then hold its state).
 *   log         as centra_progressive: iteration i goes to log[i-1].
 * The fixed-size schedule has a single iteration and takes no resume.
 * Returns CENTRA_OK, CENTRA_NOT_CERTIFIED, CENTRA_STOPPED, or an error
 * (CENTRA_EINVAL also for a checkpoint of another graph, other parameters,
 * another version, inconsistent sizes, or a redrawn sample whose entries
 * differ). */
CENTRA_API int centra_progressive_resumable(centra_ctx *ctx, const centra_graph *g, const centra_params *params,
                                 const centra_checkpoint *resume, centra_checkpoint *ckpt,
                                 uint32_t stop_after, uint32_t *picks, centra_result *result,
                                 centra_iteration *log, uint32_t log_cap, void *stream);

/* ------------------------------------------------------------------ */
/* The batching and serving engine: Algorithm 1 (as centra_progressive with
 * the geometric schedule) for many queries at once, over sample pools kept
 * resident on the device.
 *
 * A pool is one prepared graph with one sample stream (seed, instance) and
 * one schedule m_0 = m_init, m_{j+1} = min(ceil(m_j growth_num /
 * growth_den), m_max); it keeps t Rademacher trials.  A query (k, t <= the
 * pool's t, eps, delta) on a pool runs iteration i = j + 1 at m_j with
 * delta_i = delta / 2^i, exactly as centra_progressive(k, t, eps, delta,
 * the pool's seed, instance, m_init, m_max, growth, CENTRA_SCHEDULE_
 * GEOMETRIC, CENTRA_SPACE_SHORTEST_PATHS) would: the same picks, coverage
 * and bound values, whatever else runs in the engine (samples and signs
 * are functions of their indices; the pool draws each sample once and
 * every query on it reuses it).
 *
 * centra_engine_run ticks until every submitted query is done.  A tick
 * admits the queries that have arrived (in submission order) while the
 * engine's device memory, pools and active queries, stays within
 * hbm_budget_bytes (0 = no bound; a query whose state cannot fit even
 * alone is refused with CENTRA_ENOMEM as its result); draws the samples
 * every active query's next iteration needs in one fused sampling launch
 * over all pools; builds the new levels (incidence segment, deg_H and
 * Rademacher sums of the pool's first m_j samples); runs the greedy rounds
 * of all active queries fused (the queries at one level of one pool share
 * one run with their largest k, as greedy's first k picks do not depend on
 * a larger k; one set of round launches serves every run, replayed from a
 * captured HIP graph unless CENTRA_ENGINE_NO_GRAPHS); runs their per-trial
 * top-k selections fused; and evaluates every query's bound on the host
 * (one synchronisation),
 * retiring certified queries and those at m_max.  realtime != 0: query
 * arrival times are seconds from the start of the run, admission waits for
 * them (continuous batching: arrivals join the running queries at the next
 * tick); realtime == 0: every query has arrived at the start (batch mode).
 * Admission reserves, for each pool with an active query, the memory of
 * the pool with every level of its schedule built and a greedy run's state
 * per level (projected from the mean hyperedge size of its first samples,
 * plus a tenth); a pool's first samples are drawn when its first query
 * arrives.
 * Before the first tick an autotuner times the fused sampling launch with
 * 128, 256 and 512 threads per BFS on the pools' first samples and keeps
 * the fastest, unless it beats 128 by under 2% (CENTRA_ENGINE_NO_TUNE:
 * 128; a cached choice may also be 64); the environment variable
 * CENTRA_TUNE_CACHE may name a file that keeps the choice per workload;
 * centra_engine_log returns the tuner's report.  Synchronous.
 * Level caches (unless CENTRA_ENGINE_NO_CACHE): the results of a level
 * depend only on its samples, so the engine keeps, per level of a pool,
 * the picks of a greedy run of the largest k submitted on the pool and the
 * per-trial (and degree) top-k sums for every k up to it (one selection of
 * each row's largest values, sorted and prefix-summed; up to k = 2,048),
 * and a later query at that level takes them from there: the same results,
 * without its own greedy run or selection.
 * Memory: a pool holds its samples, their incidence and per level j the
 * trial sums (n t 4 bytes) and deg_H; levels no queued or active query can
 * need are released (a later query on the pool rebuilds them).
 * Errors: CENTRA_EINVAL (bad argument; t of a query above its pool's;
 * arrivals out of order), CENTRA_ENOTSUP (a schedule of more than 64
 * levels), CENTRA_ENOMEM, CENTRA_EHIP. */
typedef struct centra_engine centra_engine;
#define CENTRA_ENGINE_NO_GRAPHS 1u
#define CENTRA_ENGINE_NO_TUNE 2u
#define CENTRA_ENGINE_NO_CACHE 4u

typedef struct {
    uint64_t seed;
    uint32_t instance;
    uint32_t t;                        /* Rademacher trials kept, 1..1024 */
    uint64_t m_init, m_max;            /* 1 <= m_init <= m_max < 2^31 */
    uint32_t growth_num, growth_den;   /* growth_num > growth_den >= 1 */
} centra_pool_params;

typedef struct {
    double arrival_s, admitted_s, finished_s;   /* seconds from the start of the run */
    uint32_t pool;
} centra_query_info;

typedef struct {
    uint64_t ticks, sampler_launches, samples, greedy_runs, greedy_launches, graph_replays, graphs_captured;
    double ms_sample, ms_levels, ms_greedy, ms_select;   /* device time per phase, summed */
    uint64_t peak_bytes;
    uint32_t peak_active, tuned_block;
} centra_engine_stats;

CENTRA_API int centra_engine_create(centra_ctx *ctx, size_t hbm_budget_bytes, uint32_t flags, centra_engine **out);
CENTRA_API void centra_engine_destroy(centra_engine *e);
/* The graph must stay prepared while the engine lives. */
CENTRA_API int centra_engine_add_pool(centra_engine *e, const centra_graph *g, const centra_pool_params *params,
                           uint32_t *pool_id);
/* Draws a pool's samples up to the first level of at least m samples and
 * builds its levels up to it, ahead of queries (sample sets made resident
 * before serving starts); the first call also runs the autotuner.  Levels
 * stay while queries are queued or active on the pool.  Synchronous. */
CENTRA_API int centra_engine_prefill(centra_engine *e, uint32_t pool_id, uint64_t m, void *stream);
/* arrival_s must not decrease from one submission to the next. */
CENTRA_API int centra_engine_submit(centra_engine *e, uint32_t pool_id, uint32_t k, uint32_t t, double eps,
                         double delta, double arrival_s, uint32_t *query_id);
CENTRA_API int centra_engine_run(centra_engine *e, int realtime, void *stream);
/* picks: host u32[k] (res->n_picked written); res, info: host (may be
 * NULL).  Returns the query's CENTRA_OK / CENTRA_NOT_CERTIFIED, or its
 * refusal (CENTRA_ENOMEM), or CENTRA_EINVAL if it has not finished. */
CENTRA_API int centra_engine_result(centra_engine *e, uint32_t query_id, uint32_t *picks, centra_result *res,
                         centra_query_info *info);
CENTRA_API int centra_engine_stats_get(centra_engine *e, centra_engine_stats *out);
CENTRA_API const char *centra_engine_log(const centra_engine *e);

#ifdef __cplusplus
}
#endif

#endif
