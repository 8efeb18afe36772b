// C ABI entry points (include/centra.h): context, graph preparation, the
// three device steps of an iteration, the host FP64 bound and the
// progressive loop of Algorithm 1.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <new>
#include <string>

#include "internal.hpp"

using namespace centra;

namespace {

thread_local std::string g_create_err;

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

hipStream_t as_stream(void* s) { return static_cast<hipStream_t>(s); }

// Error of a call without a context (centra_create, the allocation-free
// greedy): kept per host thread, read with centra_last_error(NULL).
int fail_free(int code, const char* msg) {
  g_create_err = msg;
  return code;
}

}  // namespace

namespace centra {

// Writes the Theorem bound_dev quantities (host FP64).
void bound_eval(uint64_t m, uint64_t cov, int64_t sum_topk, uint32_t t, uint64_t deg_topk, uint32_t b_max,
                double eps, double delta_i, centra_bound_out* o) {
  const double a = 1.0 - exp(-1.0);
  const double md = static_cast<double>(m);
  const double L = log(5.0 / delta_i);
  const double C = static_cast<double>(cov) / md;
  const double amcera = static_cast<double>(sum_topk) / (static_cast<double>(t) * md);
  const double wimpy = static_cast<double>(b_max) * static_cast<double>(deg_topk) / md;
  const double Lm = L / md;
  const double xi = sqrt(Lm * Lm + 2.0 * C * L / (a * md)) + Lm;
  const double nu = C / a + xi;
  const double rtilde = amcera + sqrt(4.0 * wimpy * L / (static_cast<double>(t) * md));
  const double r = rtilde + sqrt(Lm * Lm + 2.0 * L * rtilde / md) + Lm;
  const double eta = 2.0 * r + sqrt(2.0 * L * (nu + 4.0 * r) / md) + L / (3.0 * md);
  o->c_hat = C;
  o->amcera = amcera;
  o->wimpy = wimpy;
  o->xi = xi;
  o->nu = nu;
  o->rtilde = rtilde;
  o->r = r;
  o->eta = eta;
  o->certified = a * ((a - eps) * xi + eta) <= eps * C ? 1 : 0;
}

// ln of the number of node sets of at most k nodes, sum_{j <= k} C(n, j),
// by a log-sum-exp of lgamma terms; then HEDGE-P's union bound and rule.
static double log_node_sets(uint64_t n, uint32_t k) {
  const uint64_t top = k < n ? k : n;
  const double ln_n1 = lgamma(static_cast<double>(n) + 1.0);
  double mx = -INFINITY;
  for (uint64_t j = 0; j <= top; ++j) {
    const double x = ln_n1 - lgamma(static_cast<double>(j) + 1.0) - lgamma(static_cast<double>(n - j) + 1.0);
    if (x > mx) mx = x;
  }
  double acc = 0.0;
  for (uint64_t j = 0; j <= top; ++j) {
    const double x = ln_n1 - lgamma(static_cast<double>(j) + 1.0) - lgamma(static_cast<double>(n - j) + 1.0);
    acc += exp(x - mx);
  }
  return mx + log(acc);
}

void hedge_eval(uint64_t m, uint64_t cov, uint64_t n, uint32_t k, double eps, double delta_i, centra_bound_out* o) {
  memset(o, 0, sizeof(*o));
  const double C = static_cast<double>(cov) / static_cast<double>(m);
  const double eta = sqrt((log(2.0) + log_node_sets(n, k) + log(1.0 / delta_i)) / (2.0 * static_cast<double>(m)));
  o->c_hat = C;
  o->eta = eta;
  o->certified = eta <= eps * (C - eta) / 2.0 ? 1 : 0;
}

}  // namespace centra

namespace {

// Next sample size (samplingSchedule of Algorithm 1): the geometric step,
// and for the adaptive schedule the optimistic size when larger.  That size
// is where eta of Theorem bound_dev with R = 0 and nu = 1,
// sqrt(2L/m) + L/(3m), reaches T = eps * C / (1 - 1/e): with y = 1/sqrt(m)
// the quadratic (L/3) y^2 + sqrt(2L) y - T = 0 has the positive root
// y = 2T / (sqrt(2L) + sqrt(2L + 4LT/3)) (no cancellation), so m = (1/y)^2.
uint64_t next_sample_size(const centra_params* p, uint64_t m_i, double c_hat, double delta_next) {
  const unsigned __int128 geo =
      (static_cast<unsigned __int128>(m_i) * p->growth_num + p->growth_den - 1) / p->growth_den;
  uint64_t next = geo > p->m_max ? p->m_max : static_cast<uint64_t>(geo);
  if (p->schedule == CENTRA_SCHEDULE_ADAPTIVE && c_hat > 0.0) {
    const double a = 1.0 - exp(-1.0);
    const double L = log(5.0 / delta_next);
    const double T = p->eps * c_hat / a;
    const double inv_y = (sqrt(2.0 * L) + sqrt(2.0 * L + 4.0 * L * T / 3.0)) / (2.0 * T);
    const double m = inv_y * inv_y;
    const uint64_t opt = m < static_cast<double>(p->m_max) ? static_cast<uint64_t>(ceil(m)) : p->m_max;
    if (opt > next) next = opt;
  }
  return next;
}

float elapsed(hipEvent_t a, hipEvent_t b) {
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, a, b) != hipSuccess) ms = 0.f;
  return ms;
}

}  // namespace

extern "C" {

uint32_t centra_abi_version(void) { return CENTRA_ABI_VERSION; }

const char* centra_context_log(const centra_ctx* ctx) { return ctx ? ctx->log.c_str() : ""; }

int centra_create(int hip_device, size_t hbm_budget_bytes, centra_ctx** out) {
  g_create_err.clear();
  if (!out) {
    g_create_err = "centra_create: out is NULL";
    return CENTRA_EINVAL;
  }
  *out = nullptr;
  int count = 0;
  hipError_t e = hipGetDeviceCount(&count);
  if (e != hipSuccess || count == 0) {
    (void)hipGetLastError();
    g_create_err = "centra_create: no HIP device available";
    return CENTRA_EHIP;
  }
  if (hip_device < 0 || hip_device >= count) {
    g_create_err = "centra_create: device index out of range";
    return CENTRA_EINVAL;
  }
  DeviceGuard guard(hip_device);
  centra_ctx* ctx = new (std::nothrow) centra_ctx();
  if (!ctx) return CENTRA_ENOMEM;
  ctx->device = hip_device;
  ctx->budget = hbm_budget_bytes;
  // Test hook: CENTRA_STAMP_START sets the first BFS stamp, so that tests
  // can cross the 32-bit stamp wrap (a full record clear) within a few
  // hundred samples.
  if (const char* st = getenv("CENTRA_STAMP_START")) {
    const unsigned long v = strtoul(st, nullptr, 0);
    if (v >= 1 && v <= 0xFFFFFFFFul) ctx->stamp_next = static_cast<uint32_t>(v);
  }
  if (hipMalloc(reinterpret_cast<void**>(&ctx->d_flags), 256) != hipSuccess ||
      hipMemset(ctx->d_flags, 0, 256) != hipSuccess) {
    (void)hipGetLastError();
    g_create_err = "centra_create: device allocation failed";
    if (ctx->d_flags) (void)hipFree(ctx->d_flags);
    delete ctx;
    return CENTRA_ENOMEM;
  }
  for (auto& ev : ctx->ev) {
    if (hipEventCreate(&ev) != hipSuccess) {
      g_create_err = "centra_create: event creation failed";
      centra_destroy(ctx);
      return CENTRA_EHIP;
    }
  }
  *out = ctx;
  return CENTRA_OK;
}

void centra_destroy(centra_ctx* ctx) {
  if (!ctx) return;
  DeviceGuard guard(ctx->device);
  (void)hipDeviceSynchronize();
  DevBuf* bufs[] = {&ctx->slot_rec, &ctx->slot_q, &ctx->slot_praw, &ctx->slot_pinfo, &ctx->wide_ws,
                    &ctx->stage_nodes, &ctx->stage_pos,
                    &ctx->stage_len, &ctx->work_ctr, &ctx->scan_tmp, &ctx->deg, &ctx->inc_off,
                    &ctx->inc_cursor, &ctx->inc, &ctx->inc_node, &ctx->gain, &ctx->covered, &ctx->best,
                    &ctx->newcov, &ctx->words, &ctx->P, &ctx->Rtm, &ctx->topk_tmp, &ctx->misc,
                    &ctx->store_off, &ctx->store_nodes, &ctx->kp_len, &ctx->kp_stage, &ctx->inc_ws, &ctx->seg_deg, &ctx->multi_tab, &ctx->sel_rows, &ctx->ext_bmax, &ctx->bi_rec_f, &ctx->bi_rec_b, &ctx->bi_q_f,
                    &ctx->bi_q_b};
  for (DevBuf* b : bufs) release(ctx, *b);
  if (ctx->d_flags) (void)hipFree(ctx->d_flags);
  for (auto& ev : ctx->ev)
    if (ev) (void)hipEventDestroy(ev);
  delete ctx;
}

const char* centra_last_error(const centra_ctx* ctx) { return ctx ? ctx->err.c_str() : g_create_err.c_str(); }

int centra_graph_prepare(centra_ctx* ctx, const centra_csr* csr, uint32_t count_bits_override, centra_graph** out,
                         void* stream) {
  if (!ctx) return CENTRA_EINVAL;
  if (!csr || !out) return fail(ctx, CENTRA_EINVAL, "graph_prepare: NULL argument");
  *out = nullptr;
  if (csr->n < 2) return fail(ctx, CENTRA_EINVAL, "graph_prepare: n < 2");
  if (csr->n_arcs >= (1ull << 32)) return fail(ctx, CENTRA_ENOTSUP, "graph_prepare: n_arcs >= 2^32");
  if (!csr->row_ptr || (csr->n_arcs && !csr->col_idx))
    return fail(ctx, CENTRA_EINVAL, "graph_prepare: NULL CSR array");
  if (csr->directed && (!csr->rrow_ptr || (csr->n_arcs && !csr->rcol_idx)))
    return fail(ctx, CENTRA_EINVAL, "graph_prepare: directed graph without reverse CSR");
  DeviceGuard guard(ctx->device);
  centra_graph* g = new (std::nothrow) centra_graph();
  if (!g) return fail(ctx, CENTRA_ENOMEM, "graph_prepare: host allocation");
  g->ctx = ctx;
  g->n = csr->n;
  g->directed = csr->directed ? 1u : 0u;
  g->n_arcs = csr->n_arcs;
  g->row_ptr = csr->row_ptr;
  g->col_idx = csr->col_idx;
  g->in_ptr = csr->directed ? csr->rrow_ptr : csr->row_ptr;
  g->in_idx = csr->directed ? csr->rcol_idx : csr->col_idx;
  int rc = validate_graph(ctx, g, as_stream(stream));
  if (rc) {
    delete g;
    return rc;
  }
  if (count_bits_override && count_bits_override < g->count_bits) g->count_bits = count_bits_override;
  g->count_bits_override = count_bits_override;
  g->bfs_row_ptr = g->row_ptr;
  g->bfs_col_idx = g->col_idx;
  g->bfs_in_ptr = g->in_ptr;
  g->bfs_in_idx = g->in_idx;
  const char* rl = getenv("CENTRA_RELABEL");
  if (!(rl && !strcmp(rl, "0")) && (rc = relabel_graph(ctx, g, as_stream(stream)))) {
    delete g;
    return rc;
  }
  *out = g;
  return CENTRA_OK;
}

void centra_graph_release(centra_graph* g) {
  if (!g) return;
  if (g->ctx) {
    DeviceGuard guard(g->ctx->device);
    release_graph_buffers(g->ctx, g);
  }
  delete g;
}

int centra_graph_info(const centra_graph* g, uint32_t* max_in_degree, uint32_t* count_bits) {
  if (!g) return CENTRA_EINVAL;
  if (max_in_degree) *max_in_degree = g->max_in_degree;
  if (count_bits) *count_bits = g->count_bits;
  return CENTRA_OK;
}

int centra_sample_paths(centra_ctx* ctx, const centra_graph* g, uint64_t seed, uint32_t instance,
                        uint64_t first_sample, uint32_t count, uint64_t* he_off, uint32_t* he_nodes, uint64_t he_cap,
                        uint64_t* he_needed, uint32_t* st_out, uint32_t* dist_out, void* stream) {
  if (!ctx) return CENTRA_EINVAL;
  if (!g || !he_off) return fail(ctx, CENTRA_EINVAL, "sample_paths: NULL argument");
  DeviceGuard guard(ctx->device);
  hipStream_t s = as_stream(stream);
  uint64_t total = 0;
  int rc = sample_to_stage(ctx, g, seed, instance, first_sample, count, st_out, dist_out, &total, s);
  if (rc) return rc;
  if (he_needed) *he_needed = total;
  if (count == 0) {
    fill_u64(he_off, 0, 1, s);
    CENTRA_HIP(ctx, hipStreamSynchronize(s));
    return CENTRA_OK;
  }
  const bool fits = he_nodes && he_cap >= total;
  rc = stage_to_output(ctx, count, 0, he_off, fits ? he_nodes : nullptr, s);
  if (rc) return rc;
  CENTRA_HIP(ctx, hipStreamSynchronize(s));
  if (!fits) return fail(ctx, CENTRA_ENOSPC, "sample_paths: he_cap smaller than the sample");
  return CENTRA_OK;
}

int centra_sample_paths_bidir(centra_ctx* ctx, const centra_graph* g, uint64_t seed, uint32_t instance,
                              uint64_t first_sample, uint32_t count, uint64_t* he_off, uint32_t* he_nodes,
                              uint64_t he_cap, uint64_t* he_needed, uint32_t* st_out, uint32_t* dist_out,
                              void* stream) {
  if (!ctx) return CENTRA_EINVAL;
  if (!g || !he_off) return fail(ctx, CENTRA_EINVAL, "sample_paths_bidir: NULL argument");
  DeviceGuard guard(ctx->device);
  hipStream_t s = as_stream(stream);
  uint64_t total = 0;
  int rc = sample_bidir_to_stage(ctx, g, seed, instance, first_sample, count, st_out, dist_out, &total, s);
  if (rc) return rc;
  if (he_needed) *he_needed = total;
  if (count == 0) {
    fill_u64(he_off, 0, 1, s);
    CENTRA_HIP(ctx, hipStreamSynchronize(s));
    return CENTRA_OK;
  }
  const bool fits = he_nodes && he_cap >= total;
  rc = stage_to_output(ctx, count, 0, he_off, fits ? he_nodes : nullptr, s);
  if (rc) return rc;
  CENTRA_HIP(ctx, hipStreamSynchronize(s));
  if (!fits) return fail(ctx, CENTRA_ENOSPC, "sample_paths_bidir: he_cap smaller than the sample");
  return CENTRA_OK;
}

int centra_triangle_count(centra_ctx* ctx, const centra_graph* g, uint64_t* T, void* stream) {
  if (!ctx) return CENTRA_EINVAL;
  if (!g || !T) return fail(ctx, CENTRA_EINVAL, "triangle_count: NULL argument");
  DeviceGuard guard(ctx->device);
  return triangle_index(ctx, const_cast<centra_graph*>(g), T, as_stream(stream));
}

int centra_sample_triangles(centra_ctx* ctx, const centra_graph* g, uint64_t seed, uint32_t instance, uint64_t first,
                            uint32_t count, uint64_t* he_off, uint32_t* he_nodes, void* stream) {
  if (!ctx) return CENTRA_EINVAL;
  if (!g || !he_off || (count && !he_nodes)) return fail(ctx, CENTRA_EINVAL, "sample_triangles: NULL argument");
  DeviceGuard guard(ctx->device);
  hipStream_t s = as_stream(stream);
  int rc = sample_triangles_into(ctx, const_cast<centra_graph*>(g), seed, instance, first, count, he_off, 0, he_nodes,
                                 s);
  if (rc) return rc;
  CENTRA_HIP(ctx, hipStreamSynchronize(s));
  return check_flags(ctx, s, "sample_triangles");
}

int centra_sample_kpaths(centra_ctx* ctx, const centra_graph* g, uint32_t kappa, uint64_t seed, uint32_t instance,
                         uint64_t first, uint32_t count, uint64_t* he_off, uint32_t* he_nodes, void* stream) {
  if (!ctx) return CENTRA_EINVAL;
  if (!g || !he_off || (count && !he_nodes)) return fail(ctx, CENTRA_EINVAL, "sample_kpaths: NULL argument");
  DeviceGuard guard(ctx->device);
  hipStream_t s = as_stream(stream);
  int rc = kpath_count(ctx, g, kappa, seed, instance, first, count, he_off, s);
  if (!rc) rc = kpath_write(ctx, g, kappa, seed, instance, first, count, he_off, 0, he_nodes, s);
  if (rc) return rc;
  CENTRA_HIP(ctx, hipStreamSynchronize(s));
  return check_flags(ctx, s, "sample_kpaths");
}

// Checks the sample arguments; he_nodes may be NULL only if every hyperedge
// is empty (he_off[m] == 0), which is read from the device.
static int check_sample_args(centra_ctx* ctx, uint32_t n, uint64_t m, const uint64_t* he_off,
                             const uint32_t* he_nodes, const char* who, hipStream_t s) {
  if (n == 0) return fail(ctx, CENTRA_EINVAL, std::string(who) + ": n == 0");
  if (!he_off) return fail(ctx, CENTRA_EINVAL, std::string(who) + ": he_off is NULL");
  if (m >= (1ull << 31)) return fail(ctx, CENTRA_ENOTSUP, std::string(who) + ": m >= 2^31");
  if (!he_nodes) {
    uint64_t I = 0;
    CENTRA_HIP(ctx, hipMemcpyAsync(&I, he_off + m, 8, hipMemcpyDeviceToHost, s));
    CENTRA_HIP(ctx, hipStreamSynchronize(s));
    if (I) return fail(ctx, CENTRA_EINVAL, std::string(who) + ": he_nodes is NULL");
  }
  return CENTRA_OK;
}

int centra_greedy_cover(centra_ctx* ctx, uint32_t n, uint64_t m, const uint64_t* he_off, const uint32_t* he_nodes,
                        uint32_t k, uint32_t* picks, uint64_t* cov_cum, uint32_t* n_picked, void* stream) {
  if (!ctx) return CENTRA_EINVAL;
  if (k == 0) return fail(ctx, CENTRA_EINVAL, "greedy_cover: k == 0");
  if (!picks || !cov_cum || !n_picked) return fail(ctx, CENTRA_EINVAL, "greedy_cover: NULL output");
  DeviceGuard guard(ctx->device);
  hipStream_t s = as_stream(stream);
  int rc = check_sample_args(ctx, n, m, he_off, he_nodes, "greedy_cover", s);
  if (rc) return rc;
  if ((rc = build_incidence(ctx, n, 0, m, he_off, he_nodes, s))) return rc;
  if ((rc = check_flags(ctx, s, "greedy_cover"))) return rc;
  if ((rc = greedy_on_incidence(ctx, n, m, he_off, he_nodes, k, picks, cov_cum, n_picked, s))) return rc;
  CENTRA_HIP(ctx, hipStreamSynchronize(s));
  return CENTRA_OK;
}

int centra_greedy_cover_noalloc(uint32_t n, uint64_t m, const uint64_t* he_off, const uint32_t* he_nodes, uint32_t k,
                                uint32_t* picks, uint64_t* cov_cum, uint32_t* n_picked, void* stream) {
  g_create_err.clear();
  if (k == 0) return fail_free(CENTRA_EINVAL, "greedy_cover_noalloc: k == 0");
  if (n == 0) return fail_free(CENTRA_EINVAL, "greedy_cover_noalloc: n == 0");
  if (!he_off) return fail_free(CENTRA_EINVAL, "greedy_cover_noalloc: he_off is NULL");
  if (!picks || !cov_cum || !n_picked) return fail_free(CENTRA_EINVAL, "greedy_cover_noalloc: NULL output");
  if (m >= (1ull << 31)) return fail_free(CENTRA_ENOTSUP, "greedy_cover_noalloc: m >= 2^31");
  return greedy_cover_static(n, m, he_off, he_nodes, k, picks, cov_cum, n_picked, as_stream(stream), &g_create_err);
}

int centra_mcera(centra_ctx* ctx, uint32_t n, uint64_t m, const uint64_t* he_off, const uint32_t* he_nodes,
                 uint64_t seed, uint32_t instance, uint32_t t, uint32_t k, int64_t* topk_sum, uint64_t* deg_topk_sum,
                 uint32_t* b_max, int32_t* R_out, void* stream) {
  if (!ctx) return CENTRA_EINVAL;
  if (m == 0) return fail(ctx, CENTRA_EINVAL, "mcera: m == 0");
  if (t == 0 || t > 1024) return fail(ctx, CENTRA_EINVAL, "mcera: t must be in [1, 1024]");
  if (k == 0) return fail(ctx, CENTRA_EINVAL, "mcera: k == 0");
  if (!topk_sum || !deg_topk_sum || !b_max) return fail(ctx, CENTRA_EINVAL, "mcera: NULL output");
  DeviceGuard guard(ctx->device);
  hipStream_t s = as_stream(stream);
  int rc = check_sample_args(ctx, n, m, he_off, he_nodes, "mcera", s);
  if (rc) return rc;
  if ((rc = build_incidence(ctx, n, 0, m, he_off, he_nodes, s))) return rc;
  if ((rc = check_flags(ctx, s, "mcera"))) return rc;
  if ((rc = rade_words(ctx, seed, instance, 0, m, t, s))) return rc;
  if ((rc = mcera_on_incidence(ctx, n, m, ctx->inc_m0, he_off, t, k, topk_sum, deg_topk_sum, b_max, R_out, s))) return rc;
  CENTRA_HIP(ctx, hipStreamSynchronize(s));
  return CENTRA_OK;
}

int centra_sample_paths_append(centra_ctx* ctx, const centra_graph* g, uint64_t seed, uint32_t instance,
                               uint64_t first_sample, uint32_t count, uint64_t* he_off, uint32_t* he_nodes,
                               uint64_t he_cap, uint64_t* he_total, void* stream) {
  if (!ctx) return CENTRA_EINVAL;
  if (!g) return fail(ctx, CENTRA_EINVAL, "sample_paths_append: graph is NULL");
  if (!he_off) return fail(ctx, CENTRA_EINVAL, "sample_paths_append: he_off is NULL");
  if (!he_nodes && he_cap) return fail(ctx, CENTRA_EINVAL, "sample_paths_append: he_nodes is NULL");
  DeviceGuard guard(ctx->device);
  return sample_append(ctx, g, seed, instance, first_sample, count, he_off, he_nodes, he_cap, he_total,
                       as_stream(stream));
}

int centra_extend(centra_ctx* ctx, const centra_extend_args* a, void* stream) {
  if (!ctx) return CENTRA_EINVAL;
  if (!a) return fail(ctx, CENTRA_EINVAL, "extend: args are NULL");
  if (a->n == 0 || a->k == 0 || a->m == 0) return fail(ctx, CENTRA_EINVAL, "extend: n, k and m must be positive");
  if (a->m < a->m_prev) return fail(ctx, CENTRA_EINVAL, "extend: m < m_prev");
  if (a->m >= (1ull << 31)) return fail(ctx, CENTRA_ENOTSUP, "extend: m >= 2^31");
  if (!a->he_off || (!a->he_nodes && a->he_cap)) return fail(ctx, CENTRA_EINVAL, "extend: NULL store pointer");
  const int outs = (a->picks != nullptr) + (a->cov_cum != nullptr) + (a->n_picked != nullptr);
  if (outs != 0 && outs != 3) return fail(ctx, CENTRA_EINVAL, "extend: greedy outputs partly NULL");
  if (a->t > 1024) return fail(ctx, CENTRA_EINVAL, "extend: t > 1024");
  if (a->t && (!a->topk_sum || !a->deg_topk_sum || !a->b_max))
    return fail(ctx, CENTRA_EINVAL, "extend: NULL AMCERA output");
  DeviceGuard guard(ctx->device);
  hipStream_t s = as_stream(stream);
  const uint32_t n = a->n;
  const uint64_t m = a->m;
  const bool same = ctx->ext_off == a->he_off && ctx->ext_nodes == a->he_nodes && ctx->ext_cap == a->he_cap &&
                    ctx->ext_n == n;
  if (!same) ctx->mc_ok = false;
  // AMCERA counts of [0, mc_m) stay usable if those samples are unchanged
  bool keep_p = a->t && same && ctx->mc_ok && a->m_prev > 0 && ctx->mc_m <= a->m_prev && ctx->mc_m <= m &&
                ctx->mc_seed == a->seed && ctx->mc_instance == a->instance && ctx->mc_t == a->t;
  int rc;
  // incidence of samples [0, m): the segments already built, plus one for
  // the new samples
  if (a->m_prev > 0 && same && ctx->ext_inc && ctx->inc_m1 <= a->m_prev) {
    if (m > ctx->inc_m1 &&
        (rc = build_incidence(ctx, n, ctx->inc_m1, m, a->he_off, a->he_nodes, s, a->he_cap)))
      return rc;
  } else if ((rc = build_incidence(ctx, n, 0, m, a->he_off, a->he_nodes, s, a->he_cap))) {
    return rc;
  }
  ctx->ext_inc = true;
  ctx->ext_off = a->he_off;
  ctx->ext_nodes = a->he_nodes;
  ctx->ext_cap = a->he_cap;
  ctx->ext_n = n;
  if (a->picks &&
      (rc = greedy_on_incidence(ctx, n, m, a->he_off, a->he_nodes, a->k, a->picks, a->cov_cum, a->n_picked, s)))
    return rc;
  if (a->t) {
    // the counts extend from mc_m only if it starts a segment (the entries
    // of samples [mc_m, m) are then contiguous in the incidence)
    if (keep_p && ctx->mc_m != m) {
      bool boundary = false;
      for (uint32_t g = 0; g < ctx->inc_nseg; ++g) boundary = boundary || ctx->inc_seg_m0[g] == ctx->mc_m;
      keep_p = boundary;
    }
    const uint64_t from = keep_p ? ctx->mc_m : 0;
    if ((rc = mcera_reserve(ctx, n, m, a->t, s))) return rc;
    if ((rc = rade_words(ctx, a->seed, a->instance, from, m, a->t, s))) return rc;
    uint32_t* bm = static_cast<uint32_t*>(ctx->ext_bmax.ptr);
    if ((rc = mcera_on_incidence(ctx, n, m, from, a->he_off, a->t, a->k, a->topk_sum, a->deg_topk_sum, bm, a->R_out,
                                 s)))
      return rc;
    CENTRA_HIP(ctx, hipMemcpyAsync(a->b_max, bm, 4, hipMemcpyDeviceToDevice, s));
    ctx->mc_ok = true;
    ctx->mc_m = m;
    ctx->mc_seed = a->seed;
    ctx->mc_instance = a->instance;
    ctx->mc_t = a->t;
  }
  CENTRA_HIP(ctx, hipGetLastError());
  return CENTRA_OK;
}

int centra_reserve(centra_ctx* ctx, const centra_graph* g, uint32_t n, uint32_t batch, uint64_t m_max, uint64_t he_cap,
                   uint32_t k, uint32_t t, void* stream) {
  if (!ctx) return CENTRA_EINVAL;
  if (n == 0) return fail(ctx, CENTRA_EINVAL, "reserve: n == 0");
  if (g && g->n != n) return fail(ctx, CENTRA_EINVAL, "reserve: the graph's node count differs from n");
  if (t > 1024) return fail(ctx, CENTRA_EINVAL, "reserve: t > 1024");
  DeviceGuard guard(ctx->device);
  hipStream_t s = as_stream(stream);
  int rc;
  if (g && batch && (rc = sample_reserve(ctx, g, batch, he_cap, s))) return rc;
  if ((rc = incidence_reserve(ctx, n, he_cap, 16, s))) return rc;
  if (k && (rc = greedy_reserve(ctx, n, m_max, k, s))) return rc;
  if (t && (rc = mcera_reserve(ctx, n, m_max, t, s))) return rc;
  CENTRA_HIP(ctx, hipStreamSynchronize(s));
  return CENTRA_OK;
}

int centra_check(centra_ctx* ctx, void* stream) {
  if (!ctx) return CENTRA_EINVAL;
  DeviceGuard guard(ctx->device);
  return check_flags(ctx, as_stream(stream), "check");
}

int centra_sampler_stats_get(centra_ctx* ctx, centra_sampler_stats* out, int reset) {
  if (!ctx || !out) return CENTRA_EINVAL;
  *out = ctx->st;
  if (reset) ctx->st = centra_sampler_stats{};
  return CENTRA_OK;
}

int centra_hedge_bound(uint64_t m, uint64_t cov, uint64_t n, uint32_t k, double eps, double delta_i,
                       centra_bound_out* out) {
  if (!out || m == 0 || n == 0 || k == 0 || !(delta_i > 0.0 && delta_i < 1.0)) return CENTRA_EINVAL;
  hedge_eval(m, cov, n, k, eps, delta_i, out);
  return CENTRA_OK;
}

int centra_vc_dims(uint64_t b, uint32_t k, uint64_t n, centra_vc_out* out) {
  if (!out || b == 0 || k == 0 || n == 0) return CENTRA_EINVAL;
  // floor(log2(2b)) is the bit length of b
  out->d1 = 64u - static_cast<uint32_t>(__builtin_clzll(b));
  out->dk_lemma = static_cast<uint64_t>(floor(2.0 * double(out->d1) * double(k) * log2(3.0 * double(k))));
  out->dk_union = static_cast<uint64_t>(floor(double(k) * log2(double(n))));
  out->dk = out->dk_lemma < out->dk_union ? out->dk_lemma : out->dk_union;
  return CENTRA_OK;
}

int centra_bound(uint64_t m, uint64_t cov, int64_t sum_topk, uint32_t t, uint64_t deg_topk, uint32_t b_max,
                 double eps, double delta_i, centra_bound_out* out) {
  if (!out || m == 0 || t == 0 || !(delta_i > 0.0 && delta_i < 1.0)) return CENTRA_EINVAL;
  bound_eval(m, cov, sum_topk, t, deg_topk, b_max, eps, delta_i, out);
  return CENTRA_OK;
}

}  // extern "C"

namespace {

// FNV-1a (64-bit) over the little-endian bytes of each field.
struct Fnv {
  uint64_t h = 0xCBF29CE484222325ull;
  template <typename T>
  void add(T v) {
    unsigned char b[sizeof(T)];
    memcpy(b, &v, sizeof(T));
    for (unsigned char c : b) h = (h ^ c) * 0x100000001B3ull;
  }
};

uint64_t params_hash(const centra_params* p) {
  Fnv f;
  f.add(p->k);
  f.add(p->t);
  f.add(p->eps);
  f.add(p->delta);
  f.add(p->seed);
  f.add(p->instance);
  f.add(p->m_init);
  f.add(p->m_max);
  f.add(p->growth_num);
  f.add(p->growth_den);
  f.add(p->schedule);
  f.add(p->space);
  f.add(p->kappa);
  f.add(p->method);
  return f.h;
}

int progressive_run(centra_ctx* ctx, const centra_graph* g, const centra_params* p, const centra_checkpoint* from,
                    centra_checkpoint* ck, uint32_t stop_after, uint32_t* picks, centra_result* res,
                    centra_iteration* log, uint32_t log_cap, void* stream) {
  if (!ctx) return CENTRA_EINVAL;
  if (!g || !p || !picks || !res) return fail(ctx, CENTRA_EINVAL, "progressive: NULL argument");
  const double a = 1.0 - exp(-1.0);
  if (p->k == 0 || p->t == 0 || p->t > 1024) return fail(ctx, CENTRA_EINVAL, "progressive: bad k or t");
  if (!(p->eps > 0.0 && p->eps < a)) return fail(ctx, CENTRA_EINVAL, "progressive: eps outside (0, 1-1/e)");
  if (!(p->delta > 0.0 && p->delta < 1.0)) return fail(ctx, CENTRA_EINVAL, "progressive: delta outside (0, 1)");
  if (p->m_init == 0 || p->m_max < p->m_init || p->m_max >= (1ull << 31))
    return fail(ctx, CENTRA_EINVAL, "progressive: bad m_init / m_max");
  if (p->growth_den == 0 || p->growth_num <= p->growth_den)
    return fail(ctx, CENTRA_EINVAL, "progressive: growth must exceed 1");
  if (p->schedule > CENTRA_SCHEDULE_FIXED) return fail(ctx, CENTRA_EINVAL, "progressive: unknown schedule");
  if (p->space > CENTRA_SPACE_PATHS_BIDIR) return fail(ctx, CENTRA_EINVAL, "progressive: unknown hyperedge space");
  if (p->space == CENTRA_SPACE_KPATHS && (p->kappa == 0 || p->kappa > CENTRA_MAX_KAPPA))
    return fail(ctx, CENTRA_EINVAL, "progressive: kappa outside [1, 16]");
  if (p->method > CENTRA_METHOD_HEDGE_P) return fail(ctx, CENTRA_EINVAL, "progressive: unknown method");
  const bool hedge = p->method == CENTRA_METHOD_HEDGE_P;
  const bool tri = p->space == CENTRA_SPACE_TRIANGLES;
  const bool kp = p->space == CENTRA_SPACE_KPATHS;
  const bool fixed = p->schedule == CENTRA_SCHEDULE_FIXED;
  const uint64_t phash = params_hash(p);
  if (from) {
    if (from->version != CENTRA_CHECKPOINT_VERSION) return fail(ctx, CENTRA_EINVAL, "resume: checkpoint version");
    if (from->graph_hash != g->hash) return fail(ctx, CENTRA_EINVAL, "resume: checkpoint of another graph");
    if (from->params_hash != phash) return fail(ctx, CENTRA_EINVAL, "resume: checkpoint of other parameters");
    if (fixed) return fail(ctx, CENTRA_EINVAL, "resume: the fixed-size schedule has one iteration");
    if (from->i == 0 || from->i > 60 || from->m_i < p->m_init || from->m_i >= p->m_max ||
        from->m_next <= from->m_i || from->m_next > p->m_max)
      return fail(ctx, CENTRA_EINVAL, "resume: inconsistent checkpoint");
  }
  DeviceGuard guard(ctx->device);
  hipStream_t s = as_stream(stream);
  memset(res, 0, sizeof(*res));
  const uint32_t k = p->k, t = p->t, n = g->n;
  // continue the state this context holds, or start (over) from sample 0
  const bool keep = from && ctx->prog_ok && ctx->prog_g == g && ctx->prog_ghash == g->hash &&
                    ctx->prog_phash == phash && ctx->prog_i == from->i && ctx->prog_m == from->m_i &&
                    ctx->prog_entries == from->entries && ctx->prog_inc_gen == ctx->inc_gen &&
                    (hedge || ctx->prog_words_gen == ctx->words_gen);
  ctx->prog_ok = false;
  int rc;
  if ((rc = ensure(ctx, ctx->store_off, (p->m_max + 1) * 8, keep, s))) return rc;
  // device result block: picks u32[k] | cov_cum u64[k] | n_picked u32 | b_max u32 | deg_topk u64 | topk i64[t]
  const size_t o_cov = (size_t(k) * 4 + 7) & ~size_t(7);
  const size_t o_np = o_cov + size_t(k) * 8;
  const size_t o_bm = o_np + 4;
  const size_t o_dk = o_np + 8;
  const size_t o_tk = o_dk + 8;
  const size_t misc_bytes = o_tk + size_t(t) * 8;
  if ((rc = ensure(ctx, ctx->misc, misc_bytes, keep, s))) return rc;
  char* misc = static_cast<char*>(ctx->misc.ptr);
  uint64_t* store_off = static_cast<uint64_t*>(ctx->store_off.ptr);
  if (!keep) {
    fill_u64(store_off, 0, 1, s);
    fill_u64(reinterpret_cast<uint64_t*>(misc), 0, misc_bytes / 8, s);   // HEDGE-P leaves the AMCERA fields at 0
  }
  std::string host_block(misc_bytes, '\0');
  hipEvent_t* ev = ctx->ev;
  uint64_t m_prev = keep ? from->m_i : 0, m_i = from ? from->m_next : p->m_init, total_nodes = keep ? from->entries : 0;
  const bool redrawn = from && !keep;   // samples [0, from->m_i) drawn again: check their entries
  for (uint32_t i = from ? from->i + 1 : 1;; ++i) {
    // the fixed-size use bounds one sample with delta itself
    const double delta_i = fixed ? p->delta : ldexp(p->delta, -static_cast<int>(i));
    const uint64_t arcs0 = ctx->st.arcs, nodes0 = ctx->st.nodes;
    CENTRA_HIP(ctx, hipEventRecord(ev[0], s));
    uint64_t added = 0;
    const uint32_t cnt = static_cast<uint32_t>(m_i - m_prev);
    if (tri) {
      added = 3ull * cnt;
      if ((rc = ensure(ctx, ctx->store_nodes, (total_nodes + added + 1) * 4, true, s))) return rc;
      uint32_t* store_nodes = static_cast<uint32_t*>(ctx->store_nodes.ptr);
      if ((rc = sample_triangles_into(ctx, const_cast<centra_graph*>(g), p->seed, p->instance, m_prev, cnt,
                                      store_off + m_prev, total_nodes, store_nodes + total_nodes, s, true)))
        return rc;
    } else if (kp) {
      if ((rc = kpath_count(ctx, g, p->kappa, p->seed, p->instance, m_prev, cnt, store_off + m_prev, s, true)))
        return rc;
      CENTRA_HIP(ctx, hipMemcpyAsync(&added, store_off + m_i, 8, hipMemcpyDeviceToHost, s));
      CENTRA_HIP(ctx, hipStreamSynchronize(s));
      if ((rc = ensure(ctx, ctx->store_nodes, (total_nodes + added + 1) * 4, true, s))) return rc;
      uint32_t* store_nodes = static_cast<uint32_t*>(ctx->store_nodes.ptr);
      if ((rc = kpath_write(ctx, g, p->kappa, p->seed, p->instance, m_prev, cnt, store_off + m_prev, total_nodes,
                            store_nodes + total_nodes, s, true)))
        return rc;
    } else {
      if ((rc = p->space == CENTRA_SPACE_PATHS_BIDIR
                    ? sample_bidir_to_stage(ctx, g, p->seed, p->instance, m_prev, cnt, nullptr, nullptr, &added, s)
                    : sample_to_stage(ctx, g, p->seed, p->instance, m_prev, cnt, nullptr, nullptr, &added, s)))
        return rc;
      if ((rc = ensure(ctx, ctx->store_nodes, (total_nodes + added + 1) * 4, true, s))) return rc;
      uint32_t* store_nodes = static_cast<uint32_t*>(ctx->store_nodes.ptr);
      if ((rc = stage_to_output(ctx, cnt, total_nodes, store_off + m_prev, store_nodes + total_nodes, s))) return rc;
    }
    total_nodes += added;
    uint32_t* store_nodes = static_cast<uint32_t*>(ctx->store_nodes.ptr);
    CENTRA_HIP(ctx, hipEventRecord(ev[1], s));
    if ((rc = build_incidence(ctx, n, m_prev, m_i, store_off, store_nodes, s))) return rc;
    if ((rc = greedy_on_incidence(ctx, n, m_i, store_off, store_nodes, k, reinterpret_cast<uint32_t*>(misc),
                                  reinterpret_cast<uint64_t*>(misc + o_cov), reinterpret_cast<uint32_t*>(misc + o_np),
                                  s)))
      return rc;
    CENTRA_HIP(ctx, hipEventRecord(ev[2], s));
    if (!hedge) {   // HEDGE-P bounds the deviation without the AMCERA
      if ((rc = rade_words(ctx, p->seed, p->instance, m_prev, m_i, t, s))) return rc;
      if ((rc = mcera_on_incidence(ctx, n, m_i, ctx->inc_m0, store_off, t, k, reinterpret_cast<int64_t*>(misc + o_tk),
                                   reinterpret_cast<uint64_t*>(misc + o_dk), reinterpret_cast<uint32_t*>(misc + o_bm),
                                   nullptr, s)))
        return rc;
    }
    CENTRA_HIP(ctx, hipEventRecord(ev[3], s));
    uint64_t entries_then = 0;
    if (redrawn && m_prev == 0)
      CENTRA_HIP(ctx, hipMemcpyAsync(&entries_then, store_off + from->m_i, 8, hipMemcpyDeviceToHost, s));
    CENTRA_HIP(ctx, hipMemcpyAsync(&host_block[0], misc, misc_bytes, hipMemcpyDeviceToHost, s));
    CENTRA_HIP(ctx, hipStreamSynchronize(s));
    if ((rc = check_flags(ctx, s, "progressive"))) return rc;
    if (redrawn && m_prev == 0 && entries_then != from->entries)
      return fail(ctx, CENTRA_EINVAL, "resume: the redrawn sample does not match the checkpoint's entries");
    const char* hb = host_block.data();
    uint32_t np, bm;
    uint64_t dk;
    memcpy(&np, hb + o_np, 4);
    memcpy(&bm, hb + o_bm, 4);
    memcpy(&dk, hb + o_dk, 8);
    uint64_t cov = 0;
    if (np) memcpy(&cov, hb + o_cov + size_t(np - 1) * 8, 8);
    int64_t sum = 0;
    for (uint32_t j = 0; j < t; ++j) {
      int64_t x;
      memcpy(&x, hb + o_tk + size_t(j) * 8, 8);
      sum += x;
    }
    centra_bound_out o;
    if (hedge)
      hedge_eval(m_i, cov, n, k, p->eps, delta_i, &o);
    else
      bound_eval(m_i, cov, sum, t, dk, bm, p->eps, delta_i, &o);
    const double ms_s = elapsed(ev[0], ev[1]), ms_c = elapsed(ev[1], ev[2]), ms_m = elapsed(ev[2], ev[3]);
    if (tri || kp) {   // the space's sampler launches join the sampling-kernel statistics
      ctx->st.launches += kp ? 2 : 1;
      ctx->st.kernel_ms += elapsed(ev[4], ev[5]) + (kp ? elapsed(ev[6], ev[7]) : 0.f);
      ctx->st.samples += cnt;
      ctx->st.hyperedge_nodes += added;
      ctx->st.slots = 0;
    }
    memcpy(picks, hb, size_t(np) * 4);
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
    res->ms_sample += ms_s;
    res->ms_cover += ms_c;
    res->ms_mcera += ms_m;
    res->ms_total += ms_s + ms_c + ms_m;
    if (log && i <= log_cap) {
      centra_iteration& it = log[i - 1];
      it.i = i;
      it.m = m_i;
      it.coverage = cov;
      it.sum_topk = sum;
      it.deg_topk = dk;
      it.b_max = bm;
      it.delta_i = delta_i;
      it.amcera = o.amcera;
      it.wimpy = o.wimpy;
      it.xi = o.xi;
      it.nu = o.nu;
      it.rtilde = o.rtilde;
      it.r = o.r;
      it.eta = o.eta;
      it.certified = o.certified;
      it.ms_sample = ms_s;
      it.ms_cover = ms_c;
      it.ms_mcera = ms_m;
      it.arcs = ctx->st.arcs - arcs0;
      it.nodes = ctx->st.nodes - nodes0;
    }
    if (o.certified) return CENTRA_OK;
    if (fixed || m_i >= p->m_max) return CENTRA_NOT_CERTIFIED;
    const uint64_t m_next = next_sample_size(p, m_i, o.c_hat, ldexp(p->delta, -static_cast<int>(i + 1)));
    // the state after iteration i, for a resume on this context or elsewhere
    ctx->prog_ok = true;
    ctx->prog_g = g;
    ctx->prog_ghash = g->hash;
    ctx->prog_phash = phash;
    ctx->prog_i = i;
    ctx->prog_m = m_i;
    ctx->prog_entries = total_nodes;
    ctx->prog_inc_gen = ctx->inc_gen;
    ctx->prog_words_gen = ctx->words_gen;
    if (ck) *ck = centra_checkpoint{CENTRA_CHECKPOINT_VERSION, i, g->hash, phash, m_i, m_next, total_nodes};
    if (stop_after && i >= stop_after) return CENTRA_STOPPED;
    m_prev = m_i;
    m_i = m_next;
  }
}

}  // namespace

extern "C" {

int centra_progressive(centra_ctx* ctx, const centra_graph* g, const centra_params* p, uint32_t* picks,
                       centra_result* res, centra_iteration* log, uint32_t log_cap, void* stream) {
  return progressive_run(ctx, g, p, nullptr, nullptr, 0, picks, res, log, log_cap, stream);
}

int centra_progressive_resumable(centra_ctx* ctx, const centra_graph* g, const centra_params* p,
                                 const centra_checkpoint* resume, centra_checkpoint* ckpt, uint32_t stop_after,
                                 uint32_t* picks, centra_result* res, centra_iteration* log, uint32_t log_cap,
                                 void* stream) {
  return progressive_run(ctx, g, p, resume, ckpt, stop_after, picks, res, log, log_cap, stream);
}

int centra_params_hash(const centra_params* p, uint64_t* hash) {
  if (!p || !hash) return CENTRA_EINVAL;
  *hash = params_hash(p);
  return CENTRA_OK;
}

int centra_graph_hash(const centra_graph* g, uint64_t* hash) {
  if (!g || !hash) return CENTRA_EINVAL;
  *hash = g->hash;
  return CENTRA_OK;
}

}  // extern "C"
