// Host-side memory and undefined-behaviour check of the library: this
// program is linked with every library object built with AddressSanitizer
// and UndefinedBehaviorSanitizer on the host side only (device code is
// built as usual).  It drives the C ABI and checks its results against
// properties computed here on the host.
//
//   host_sanitize          the calls that need no GPU: the bound formulas
//                          (Theorem bound_dev, HEDGE-P, the VC-dimension
//                          bounds), the parameter hash, argument checks and
//                          centra_create on a machine without a device;
//   host_sanitize --gpu    also every device entry point on device 0: graph
//                          preparation (and a malformed CSR), the samplers
//                          of all four spaces, greedy cover with and without
//                          allocation, AMCERA, the stream-ordered append /
//                          extend chain, Algorithm 1 whole and stopped /
//                          resumed, and the multi-query engine.
//
// It prints "<N> failed checks" and returns 1 if N > 0.  It is test
// infrastructure, not part of the library.
#include <hip/hip_runtime_api.h>
#include <sanitizer/lsan_interface.h>
#include <unistd.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <set>
#include <vector>

#include "centra.h"

namespace {

int g_fail = 0;

void say(const char* what) {
  std::printf("%s\n", what);
  std::fflush(stdout);
}

#define CHECK(cond, ...)                                  \
  do {                                                    \
    if (!(cond)) {                                        \
      ++g_fail;                                           \
      std::printf("FAIL %s:%d: ", __FILE__, __LINE__);    \
      std::printf(__VA_ARGS__);                           \
      std::printf("\n");                                  \
      std::fflush(stdout);                                \
    }                                                     \
  } while (0)

struct HostGraph {
  uint32_t n = 0;
  bool directed = false;
  std::vector<std::set<uint32_t>> out, in;
  std::vector<uint32_t> row_ptr, col_idx, rrow_ptr, rcol_idx;

  void arc(uint32_t u, uint32_t v) {
    if (u == v) return;
    out[u].insert(v);
    in[v].insert(u);
    if (!directed) {
      out[v].insert(u);
      in[u].insert(v);
    }
  }
  void finish() {
    auto csr = [&](const std::vector<std::set<uint32_t>>& rows, std::vector<uint32_t>& rp, std::vector<uint32_t>& ci) {
      rp.assign(1, 0);
      ci.clear();
      for (const auto& r : rows) {
        ci.insert(ci.end(), r.begin(), r.end());
        rp.push_back(static_cast<uint32_t>(ci.size()));
      }
    };
    csr(out, row_ptr, col_idx);
    if (directed) csr(in, rrow_ptr, rcol_idx);
  }
  bool has_arc(uint32_t u, uint32_t v) const { return out[u].count(v) != 0; }
};

// An undirected grid with one diagonal per cell (so it has triangles) and a
// few long chords (so shortest paths vary in length and multiplicity).
HostGraph grid_graph(uint32_t R, uint32_t C) {
  HostGraph g;
  g.n = R * C;
  g.out.resize(g.n);
  g.in.resize(g.n);
  for (uint32_t r = 0; r < R; ++r)
    for (uint32_t c = 0; c < C; ++c) {
      const uint32_t u = r * C + c;
      if (c + 1 < C) g.arc(u, u + 1);
      if (r + 1 < R) g.arc(u, u + C);
      if (r + 1 < R && c + 1 < C) g.arc(u, u + C + 1);
      if (u % 7 == 0) g.arc(u, (u * 37 + 11) % g.n);
    }
  g.finish();
  return g;
}

// A directed graph: a cycle through every node plus three pseudo-random
// out-arcs per node.
HostGraph directed_graph(uint32_t n) {
  HostGraph g;
  g.n = n;
  g.directed = true;
  g.out.resize(n);
  g.in.resize(n);
  uint64_t x = 0x9E3779B97F4A7C15ull;
  for (uint32_t u = 0; u < n; ++u) {
    g.arc(u, (u + 1) % n);
    for (int j = 0; j < 3; ++j) {
      x = x * 6364136223846793005ull + 1442695040888963407ull;
      g.arc(u, static_cast<uint32_t>((x >> 33) % n));
    }
  }
  g.finish();
  return g;
}

template <typename T>
T* dev_alloc(size_t count) {
  void* p = nullptr;
  if (hipMalloc(&p, std::max<size_t>(count, 1) * sizeof(T)) != hipSuccess) return nullptr;
  (void)hipMemset(p, 0, std::max<size_t>(count, 1) * sizeof(T));
  return static_cast<T*>(p);
}

template <typename T>
T* dev_copy(const std::vector<T>& v) {
  T* p = dev_alloc<T>(v.size());
  if (p && !v.empty()) (void)hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
  return p;
}

template <typename T>
std::vector<T> host_copy(const T* p, size_t count) {
  std::vector<T> v(count);
  if (count) (void)hipMemcpy(v.data(), p, count * sizeof(T), hipMemcpyDeviceToHost);
  return v;
}

struct Sample {
  std::vector<uint64_t> off;
  std::vector<uint32_t> nodes;
  uint64_t m() const { return off.empty() ? 0 : off.size() - 1; }
};

// Offsets start at 0 and never decrease; node ids are < n and distinct
// within a hyperedge; no hyperedge is longer than max_len.
void check_sample(const Sample& s, uint32_t n, uint64_t max_len, const char* who) {
  CHECK(!s.off.empty() && s.off[0] == 0, "%s: he_off[0] != 0", who);
  bool ok = true;
  for (uint64_t i = 0; i < s.m() && ok; ++i) {
    if (s.off[i + 1] < s.off[i] || s.off[i + 1] - s.off[i] > max_len) ok = false;
    std::set<uint32_t> seen;
    for (uint64_t e = s.off[i]; ok && e < s.off[i + 1]; ++e)
      if (e >= s.nodes.size() || s.nodes[e] >= n || !seen.insert(s.nodes[e]).second) ok = false;
  }
  CHECK(ok, "%s: malformed hyperedges", who);
}

std::vector<uint64_t> degrees(const Sample& s, uint32_t n) {
  std::vector<uint64_t> d(n, 0);
  for (uint64_t e = 0; e < s.off.back(); ++e) ++d[s.nodes[e]];
  return d;
}

uint64_t covered_by(const Sample& s, const std::vector<uint32_t>& picks) {
  std::set<uint32_t> p(picks.begin(), picks.end());
  uint64_t c = 0;
  for (uint64_t i = 0; i < s.m(); ++i)
    for (uint64_t e = s.off[i]; e < s.off[i + 1]; ++e)
      if (p.count(s.nodes[e])) {
        ++c;
        break;
      }
  return c;
}

// ---------------------------------------------------------------- host only
void host_checks() {
  CHECK(centra_abi_version() == CENTRA_ABI_VERSION, "abi version");
  centra_bound_out b{};
  // Theorem bound_dev: the terms are non-negative and ordered
  // (rtilde >= AMCERA, r >= rtilde, eta >= 2r, nu >= C / (1 - 1/e)); a
  // larger sample lowers eta for the same empirical values.
  const uint64_t ms[] = {1, 2, 1000, 1000000, 1ull << 40};
  for (uint64_t m : ms)
    for (uint64_t cov : {uint64_t(0), m / 3, m})
      for (uint32_t t : {1u, 64u, 1024u}) {
        const int64_t sum_topk = static_cast<int64_t>(m / 10) * t;
        CHECK(centra_bound(m, cov, sum_topk, t, m, 5, 0.01, 0.1, &b) == CENTRA_OK, "bound rc");
        const double a = 1.0 - std::exp(-1.0);
        CHECK(std::isfinite(b.eta) && b.eta >= 2.0 * b.r && b.r >= b.rtilde && b.rtilde >= b.amcera &&
                  b.nu >= b.c_hat / a - 1e-12 && b.xi > 0.0 && b.c_hat >= 0.0 && b.c_hat <= 1.0,
              "bound terms out of order at m=%llu", (unsigned long long)m);
        centra_bound_out b2{};
        CHECK(centra_bound(2 * m, 2 * cov, 2 * sum_topk, t, 2 * m, 5, 0.01, 0.1, &b2) == CENTRA_OK, "bound rc");
        CHECK(b2.eta < b.eta, "eta does not shrink with the sample size");
      }
  CHECK(centra_bound(0, 0, 0, 1, 0, 0, 0.01, 0.1, &b) == CENTRA_EINVAL, "bound m = 0");
  CHECK(centra_bound(10, 0, 0, 0, 0, 0, 0.01, 0.1, &b) == CENTRA_EINVAL, "bound t = 0");
  CHECK(centra_bound(10, 0, 0, 1, 0, 0, 0.01, 1.0, &b) == CENTRA_EINVAL, "bound delta = 1");
  CHECK(centra_bound(10, 0, 0, 1, 0, 0, 0.01, 0.1, nullptr) == CENTRA_EINVAL, "bound NULL");

  // HEDGE-P: k >= n makes the union over all node sets 2^n.
  CHECK(centra_hedge_bound(1000, 500, 20, 50, 0.1, 0.1, &b) == CENTRA_OK, "hedge rc");
  const double want = std::sqrt((std::log(2.0) + 20.0 * std::log(2.0) + std::log(10.0)) / 2000.0);
  CHECK(std::fabs(b.eta - want) < 1e-12 * want, "hedge eta %.17g vs %.17g", b.eta, want);
  CHECK(centra_hedge_bound(1000, 500, 1u << 20, 100, 0.1, 0.1, &b) == CENTRA_OK && std::isfinite(b.eta), "hedge");
  CHECK(centra_hedge_bound(1000, 500, 0, 1, 0.1, 0.1, &b) == CENTRA_EINVAL, "hedge n = 0");

  // VC-dimension bounds: d1 = floor(log2(2b)) is the bit length of b.
  centra_vc_out v{};
  for (uint64_t bb : {uint64_t(1), uint64_t(2), uint64_t(3), uint64_t(1) << 40, ~uint64_t(0)}) {
    CHECK(centra_vc_dims(bb, 7, 1000, &v) == CENTRA_OK, "vc rc");
    uint32_t bits = 0;
    for (uint64_t x = bb; x; x >>= 1) ++bits;
    CHECK(v.d1 == bits && v.dk == std::min(v.dk_lemma, v.dk_union), "vc dims for b=%llu", (unsigned long long)bb);
  }
  CHECK(centra_vc_dims(0, 1, 10, &v) == CENTRA_EINVAL, "vc b = 0");

  centra_params p{};
  p.k = 5;
  p.t = 16;
  p.eps = 0.05;
  p.delta = 0.1;
  p.seed = 3;
  p.m_init = 1000;
  p.m_max = 8000;
  p.growth_num = 2;
  p.growth_den = 1;
  uint64_t h1 = 0, h2 = 0;
  CHECK(centra_params_hash(&p, &h1) == CENTRA_OK, "params hash");
  p.seed = 4;
  CHECK(centra_params_hash(&p, &h2) == CENTRA_OK && h1 != h2, "params hash ignores the seed");
  CHECK(centra_params_hash(nullptr, &h1) == CENTRA_EINVAL, "params hash NULL");

  // Entry points reject a NULL context or engine without touching a device.
  CHECK(centra_create(0, 0, nullptr) == CENTRA_EINVAL, "create NULL out");
  CHECK(std::strlen(centra_last_error(nullptr)) > 0, "create error text");
  CHECK(centra_graph_prepare(nullptr, nullptr, 0, nullptr, nullptr) == CENTRA_EINVAL, "prepare NULL");
  CHECK(centra_sample_paths(nullptr, nullptr, 0, 0, 0, 1, nullptr, nullptr, 0, nullptr, nullptr, nullptr,
                            nullptr) == CENTRA_EINVAL, "sample NULL");
  CHECK(centra_greedy_cover(nullptr, 1, 1, nullptr, nullptr, 1, nullptr, nullptr, nullptr, nullptr) == CENTRA_EINVAL,
        "greedy NULL");
  CHECK(centra_greedy_cover_noalloc(10, 1, nullptr, nullptr, 0, nullptr, nullptr, nullptr, nullptr) == CENTRA_EINVAL,
        "noalloc k = 0");
  CHECK(centra_mcera(nullptr, 1, 1, nullptr, nullptr, 0, 0, 1, 1, nullptr, nullptr, nullptr, nullptr, nullptr) ==
            CENTRA_EINVAL, "mcera NULL");
  CHECK(centra_progressive(nullptr, nullptr, &p, nullptr, nullptr, nullptr, 0, nullptr) == CENTRA_EINVAL,
        "progressive NULL");
  CHECK(centra_engine_create(nullptr, 0, 0, nullptr) == CENTRA_EINVAL, "engine NULL");
  CHECK(centra_graph_info(nullptr, nullptr, nullptr) == CENTRA_EINVAL, "graph info NULL");
  centra_graph_release(nullptr);
  centra_engine_destroy(nullptr);
  centra_destroy(nullptr);
  CHECK(std::strcmp(centra_context_log(nullptr), "") == 0 && std::strcmp(centra_engine_log(nullptr), "") == 0,
        "logs of NULL");
}

// -------------------------------------------------------------- device part
struct DevGraph {
  uint32_t *rp = nullptr, *ci = nullptr, *rrp = nullptr, *rci = nullptr;
  centra_graph* g = nullptr;
};

int prepare(centra_ctx* ctx, const HostGraph& h, DevGraph& d) {
  d.rp = dev_copy(h.row_ptr);
  d.ci = dev_copy(h.col_idx);
  if (h.directed) {
    d.rrp = dev_copy(h.rrow_ptr);
    d.rci = dev_copy(h.rcol_idx);
  }
  centra_csr c{h.n, h.directed ? 1u : 0u, h.col_idx.size(), d.rp, d.ci, d.rrp, d.rci};
  return centra_graph_prepare(ctx, &c, 0, &d.g, nullptr);
}

void release(DevGraph& d) {
  centra_graph_release(d.g);
  for (uint32_t* p : {d.rp, d.ci, d.rrp, d.rci})
    if (p) (void)hipFree(p);
}

// Draws `count` shortest-path samples (or bidirectional ones), first into a
// buffer that is too small (CENTRA_ENOSPC with the size needed), then into
// one that fits; checks each hyperedge against d(s, t) and the graph.
Sample paths(centra_ctx* ctx, const HostGraph& h, const DevGraph& d, uint32_t count, bool bidir) {
  const char* who = bidir ? "bidir" : "paths";
  auto call = bidir ? centra_sample_paths_bidir : centra_sample_paths;
  uint64_t* off = dev_alloc<uint64_t>(count + 1);
  uint32_t* small = dev_alloc<uint32_t>(4);
  uint32_t* st = dev_alloc<uint32_t>(2 * count);
  uint32_t* dist = dev_alloc<uint32_t>(count);
  uint64_t need = 0;
  int rc = call(ctx, d.g, 11, 0, 0, count, off, small, 4, &need, st, dist, nullptr);
  CHECK(rc == CENTRA_ENOSPC && need > 4, "%s: small buffer rc %d need %llu", who, rc, (unsigned long long)need);
  uint32_t* nodes = dev_alloc<uint32_t>(need);
  uint64_t need2 = 0;
  rc = call(ctx, d.g, 11, 0, 0, count, off, nodes, need, &need2, st, dist, nullptr);
  CHECK(rc == CENTRA_OK && need2 == need, "%s: rc %d", who, rc);
  Sample s{host_copy(off, count + 1), host_copy(nodes, need)};
  check_sample(s, h.n, h.n, who);
  const auto hst = host_copy(st, 2 * count);
  const auto hd = host_copy(dist, count);
  bool ok = true;
  for (uint32_t i = 0; i < count && ok; ++i) {
    const uint32_t src = hst[2 * i], dst = hst[2 * i + 1];
    const uint64_t len = s.off[i + 1] - s.off[i];
    if (src >= h.n || dst >= h.n || src == dst) ok = false;
    else if (hd[i] == 0xFFFFFFFFu) ok = len == 0;
    else if (hd[i] == 0 || len != hd[i] - 1) ok = false;
    else {
      // the path s, h[len-1], ..., h[0], t (t's neighbour first)
      uint32_t prev = dst;
      for (uint64_t e = s.off[i]; e < s.off[i + 1] && ok; ++e) {
        ok = h.has_arc(s.nodes[e], prev);
        prev = s.nodes[e];
      }
      ok = ok && h.has_arc(src, prev);
    }
  }
  CHECK(ok, "%s: a hyperedge is not a path of length d(s, t)", who);
  for (void* p : {(void*)off, (void*)small, (void*)st, (void*)dist, (void*)nodes}) (void)hipFree(p);
  return s;
}

struct Cover {
  std::vector<uint32_t> picks;
  std::vector<uint64_t> cov;
};

Cover greedy(centra_ctx* ctx, const Sample& s, uint32_t n, uint32_t k, bool noalloc) {
  uint64_t* off = dev_copy(s.off);
  uint32_t* nodes = dev_copy(s.nodes);
  uint32_t* picks = dev_alloc<uint32_t>(k);
  uint64_t* cov = dev_alloc<uint64_t>(k);
  uint32_t* np = dev_alloc<uint32_t>(1);
  const int rc = noalloc ? centra_greedy_cover_noalloc(n, s.m(), off, nodes, k, picks, cov, np, nullptr)
                         : centra_greedy_cover(ctx, n, s.m(), off, nodes, k, picks, cov, np, nullptr);
  CHECK(rc == CENTRA_OK, "greedy (noalloc %d) rc %d", int(noalloc), rc);
  const uint32_t got = host_copy(np, 1)[0];
  CHECK(got <= k, "greedy picked %u > k", got);
  Cover c{host_copy(picks, got), host_copy(cov, got)};
  for (void* p : {(void*)off, (void*)nodes, (void*)picks, (void*)cov, (void*)np}) (void)hipFree(p);
  return c;
}

void check_cover(const Cover& c, const Sample& s, uint32_t n) {
  // greedy's first pick is the node of largest degree in the sample, lowest
  // id on ties; the coverage of the picks is the last cumulative count
  const auto deg = degrees(s, n);
  const uint32_t best = static_cast<uint32_t>(std::max_element(deg.begin(), deg.end()) - deg.begin());
  CHECK(!c.picks.empty() && c.picks[0] == best, "first pick %u, want %u", c.picks.empty() ? 0u : c.picks[0], best);
  CHECK(std::set<uint32_t>(c.picks.begin(), c.picks.end()).size() == c.picks.size(), "repeated pick");
  CHECK(!c.cov.empty() && c.cov.back() == covered_by(s, c.picks), "coverage of the picks");
  CHECK(std::is_sorted(c.cov.begin(), c.cov.end()), "cumulative coverage decreases");
}

void mcera(centra_ctx* ctx, const Sample& s, uint32_t n) {
  const uint32_t t = 8, k = 5;
  uint64_t* off = dev_copy(s.off);
  uint32_t* nodes = dev_copy(s.nodes);
  int64_t* topk = dev_alloc<int64_t>(t);
  uint64_t* dk = dev_alloc<uint64_t>(1);
  uint32_t* bm = dev_alloc<uint32_t>(1);
  int32_t* R = dev_alloc<int32_t>(size_t(n) * t);
  const int rc = centra_mcera(ctx, n, s.m(), off, nodes, 7, 0, t, k, topk, dk, bm, R, nullptr);
  CHECK(rc == CENTRA_OK, "mcera rc %d", rc);
  auto deg = degrees(s, n);
  uint64_t b_max = 0;
  for (uint64_t i = 0; i < s.m(); ++i) b_max = std::max(b_max, s.off[i + 1] - s.off[i]);
  CHECK(host_copy(bm, 1)[0] == b_max, "b_max");
  std::vector<uint64_t> sorted = deg;
  std::sort(sorted.rbegin(), sorted.rend());
  uint64_t want = 0;
  for (uint32_t j = 0; j < k; ++j) want += sorted[j];
  CHECK(host_copy(dk, 1)[0] == want, "sum of the k largest degrees");
  // R[u][j] is a sum of deg(u) signs: |R| <= deg and R = deg (mod 2); the
  // top-k sums are sums of at most k positive entries of column j
  const auto hR = host_copy(R, size_t(n) * t);
  const auto hk = host_copy(topk, t);
  bool ok = true;
  for (uint32_t u = 0; u < n && ok; ++u)
    for (uint32_t j = 0; j < t && ok; ++j) {
      const int64_t r = hR[size_t(u) * t + j];
      ok = std::llabs(r) <= static_cast<int64_t>(deg[u]) && ((r - static_cast<int64_t>(deg[u])) % 2 == 0);
    }
  CHECK(ok, "Rademacher sums inconsistent with the degrees");
  for (uint32_t j = 0; j < t; ++j) {
    std::vector<int64_t> col;
    for (uint32_t u = 0; u < n; ++u)
      if (hR[size_t(u) * t + j] > 0) col.push_back(hR[size_t(u) * t + j]);
    std::sort(col.rbegin(), col.rend());
    int64_t w = 0;
    for (size_t q = 0; q < col.size() && q < k; ++q) w += col[q];
    CHECK(hk[j] == w, "top-k sum of trial %u", j);
  }
  for (void* p : {(void*)off, (void*)nodes, (void*)topk, (void*)dk, (void*)bm, (void*)R}) (void)hipFree(p);
}

void triangles(centra_ctx* ctx, const HostGraph& h, const DevGraph& d) {
  uint64_t T = 0, want = 0;
  const int rc = centra_triangle_count(ctx, d.g, &T, nullptr);
  if (h.directed) {
    CHECK(rc == CENTRA_ENOTSUP, "triangles on a directed graph rc %d", rc);
    return;
  }
  for (uint32_t a = 0; a < h.n; ++a)
    for (uint32_t b : h.out[a])
      if (b > a)
        for (uint32_t c : h.out[b])
          if (c > b && h.has_arc(a, c)) ++want;
  CHECK(rc == CENTRA_OK && T == want, "triangle count %llu, want %llu", (unsigned long long)T,
        (unsigned long long)want);
  const uint32_t count = 2000;
  uint64_t* off = dev_alloc<uint64_t>(count + 1);
  uint32_t* nodes = dev_alloc<uint32_t>(3 * count);
  CHECK(centra_sample_triangles(ctx, d.g, 5, 0, 0, count, off, nodes, nullptr) == CENTRA_OK, "sample triangles");
  const auto hn = host_copy(nodes, 3 * count);
  bool ok = host_copy(off, count + 1)[count] == 3ull * count;
  for (uint32_t i = 0; i < count && ok; ++i) {
    const uint32_t a = hn[3 * i], b = hn[3 * i + 1], c = hn[3 * i + 2];
    ok = a < b && b < c && c < h.n && h.has_arc(a, b) && h.has_arc(b, c) && h.has_arc(a, c);
  }
  CHECK(ok, "a sampled triple is not a triangle");
  (void)hipFree(off);
  (void)hipFree(nodes);
}

void kpaths(centra_ctx* ctx, const HostGraph& h, const DevGraph& d) {
  const uint32_t count = 3000, kappa = 4;
  uint64_t* off = dev_alloc<uint64_t>(count + 1);
  uint32_t* nodes = dev_alloc<uint32_t>(size_t(count) * kappa);
  CHECK(centra_sample_kpaths(ctx, d.g, kappa, 5, 0, 0, count, off, nodes, nullptr) == CENTRA_OK, "kpaths rc");
  CHECK(centra_sample_kpaths(ctx, d.g, 17, 5, 0, 0, count, off, nodes, nullptr) == CENTRA_EINVAL, "kappa 17");
  const auto ho = host_copy(off, count + 1);
  Sample s{ho, host_copy(nodes, ho[count])};
  check_sample(s, h.n, kappa, "kpaths");
  bool ok = true;
  for (uint32_t i = 0; i < count && ok; ++i)
    for (uint64_t e = s.off[i] + 1; e < s.off[i + 1] && ok; ++e) ok = h.has_arc(s.nodes[e - 1], s.nodes[e]);
  CHECK(ok, "a k-path walk leaves the graph");
  (void)hipFree(off);
  (void)hipFree(nodes);
}

// The stream-ordered chain: reserve, two appends, two extends (the second
// incremental), then one check; the picks equal centra_greedy_cover's on
// the same store.
void stream_chain(centra_ctx* ctx, const HostGraph& h, const DevGraph& d) {
  const uint32_t batch = 1500, k = 6, t = 8;
  const uint64_t cap = uint64_t(2) * batch * h.n;
  CHECK(centra_reserve(ctx, d.g, h.n, batch, 2 * batch, cap, k, t, nullptr) == CENTRA_OK, "reserve");
  uint64_t* off = dev_alloc<uint64_t>(2 * batch + 1);
  uint32_t* nodes = dev_alloc<uint32_t>(cap);
  uint32_t* picks = dev_alloc<uint32_t>(k);
  uint64_t* cov = dev_alloc<uint64_t>(k);
  uint32_t* np = dev_alloc<uint32_t>(1);
  int64_t* topk = dev_alloc<int64_t>(t);
  uint64_t* dk = dev_alloc<uint64_t>(1);
  uint32_t* bm = dev_alloc<uint32_t>(1);
  centra_extend_args a{};
  a.n = h.n;
  a.k = k;
  a.he_off = off;
  a.he_nodes = nodes;
  a.he_cap = cap;
  a.picks = picks;
  a.cov_cum = cov;
  a.n_picked = np;
  a.t = t;
  a.seed = 9;
  a.topk_sum = topk;
  a.deg_topk_sum = dk;
  a.b_max = bm;
  for (uint32_t b = 0; b < 2; ++b) {
    CHECK(centra_sample_paths_append(ctx, d.g, 21, 0, uint64_t(b) * batch, batch, off + uint64_t(b) * batch, nodes,
                                     cap, nullptr, nullptr) == CENTRA_OK, "append %u", b);
    a.m_prev = uint64_t(b) * batch;
    a.m = uint64_t(b + 1) * batch;
    CHECK(centra_extend(ctx, &a, nullptr) == CENTRA_OK, "extend %u", b);
  }
  CHECK(centra_check(ctx, nullptr) == CENTRA_OK, "check: %s", centra_last_error(ctx));
  const uint32_t got = host_copy(np, 1)[0];
  const std::vector<uint32_t> ext_picks = host_copy(picks, got);
  const auto ho = host_copy(off, 2 * batch + 1);
  Sample s{ho, host_copy(nodes, ho.back())};
  check_sample(s, h.n, h.n, "append");
  const Cover c = greedy(ctx, s, h.n, k, false);
  CHECK(c.picks == ext_picks, "extend's picks differ from greedy_cover's");
  for (void* p : {(void*)off, (void*)nodes, (void*)picks, (void*)cov, (void*)np, (void*)topk, (void*)dk, (void*)bm})
    (void)hipFree(p);
}

centra_params params(uint32_t space, uint32_t method) {
  centra_params p{};
  p.k = 6;
  p.t = 16;
  p.eps = 0.05;
  p.delta = 0.1;
  p.seed = 3;
  p.m_init = 1000;
  p.m_max = 16000;
  p.growth_num = 2;
  p.growth_den = 1;
  p.space = space;
  p.kappa = space == CENTRA_SPACE_KPATHS ? 4 : 0;
  p.method = method;
  return p;
}

void progressive(centra_ctx* ctx, const HostGraph& h, const DevGraph& d, const centra_params& p) {
  std::vector<uint32_t> picks(p.k), picks2(p.k);
  centra_result r{}, r2{};
  std::vector<centra_iteration> log(64), log2(64);
  const int rc = centra_progressive(ctx, d.g, &p, picks.data(), &r, log.data(), 64, nullptr);
  CHECK((rc == CENTRA_OK || rc == CENTRA_NOT_CERTIFIED) && r.iterations >= 1 && r.n_picked <= p.k &&
            r.coverage <= r.m_final && r.m_final <= p.m_max,
        "progressive space %u method %u rc %d: %s", p.space, p.method, rc, centra_last_error(ctx));
  for (uint32_t i = 0; i < r.n_picked; ++i) CHECK(picks[i] < h.n, "pick out of range");
  if (r.iterations < 2) return;
  centra_checkpoint ck{};
  int rs = centra_progressive_resumable(ctx, d.g, &p, nullptr, &ck, 1, picks2.data(), &r2, log2.data(), 64, nullptr);
  CHECK(rs == CENTRA_STOPPED && ck.i == 1 && ck.version == CENTRA_CHECKPOINT_VERSION, "stop after 1: rc %d", rs);
  centra_checkpoint bad = ck;
  bad.version = 7;
  CHECK(centra_progressive_resumable(ctx, d.g, &p, &bad, nullptr, 0, picks2.data(), &r2, log2.data(), 64,
                                     nullptr) == CENTRA_EINVAL, "checkpoint of another version accepted");
  rs = centra_progressive_resumable(ctx, d.g, &p, &ck, nullptr, 0, picks2.data(), &r2, log2.data(), 64, nullptr);
  CHECK(rs == rc && r2.n_picked == r.n_picked && r2.coverage == r.coverage && r2.m_final == r.m_final &&
            r2.eta == r.eta && std::equal(picks.begin(), picks.begin() + r.n_picked, picks2.begin()),
        "resumed run differs (space %u)", p.space);
}

void engine(centra_ctx* ctx, const DevGraph& a, const DevGraph& b, uint32_t flags) {
  centra_engine* e = nullptr;
  CHECK(centra_engine_create(ctx, 0, flags, &e) == CENTRA_OK && e, "engine create");
  if (!e) return;
  centra_pool_params pp{5, 0, 16, 1000, 16000, 2, 1};
  uint32_t pa = 0, pb = 0;
  CHECK(centra_engine_add_pool(e, a.g, &pp, &pa) == CENTRA_OK, "add pool a");
  pp.seed = 6;
  CHECK(centra_engine_add_pool(e, b.g, &pp, &pb) == CENTRA_OK, "add pool b");
  pp.t = 0;
  uint32_t junk = 0;
  CHECK(centra_engine_add_pool(e, a.g, &pp, &junk) == CENTRA_EINVAL, "pool with t = 0");
  CHECK(centra_engine_prefill(e, pa, 2000, nullptr) == CENTRA_OK, "prefill");
  std::vector<uint32_t> q(4);
  CHECK(centra_engine_submit(e, pa, 4, 16, 0.05, 0.1, 0.0, &q[0]) == CENTRA_OK, "submit");
  CHECK(centra_engine_submit(e, pb, 6, 8, 0.1, 0.1, 0.0, &q[1]) == CENTRA_OK, "submit");
  CHECK(centra_engine_submit(e, pa, 8, 16, 0.1, 0.05, 0.0, &q[2]) == CENTRA_OK, "submit");
  CHECK(centra_engine_submit(e, pb, 3, 4, 0.2, 0.1, 0.0, &q[3]) == CENTRA_OK, "submit");
  CHECK(centra_engine_run(e, 0, nullptr) == CENTRA_OK, "engine run: %s", centra_last_error(ctx));
  for (uint32_t id : q) {
    std::vector<uint32_t> picks(8);
    centra_result r{};
    centra_query_info info{};
    const int rc = centra_engine_result(e, id, picks.data(), &r, &info);
    CHECK((rc == CENTRA_OK || rc == CENTRA_NOT_CERTIFIED) && r.n_picked >= 1 && info.finished_s >= info.arrival_s,
          "engine result %u rc %d", id, rc);
  }
  centra_engine_stats st{};
  CHECK(centra_engine_stats_get(e, &st) == CENTRA_OK && st.greedy_runs >= 4, "engine stats");
  CHECK(centra_engine_log(e) != nullptr, "engine log");
  centra_engine_destroy(e);
}

void device_checks() {
  centra_ctx* ctx = nullptr;
  int rc = centra_create(0, 0, &ctx);
  CHECK(rc == CENTRA_OK && ctx, "create: %s", centra_last_error(nullptr));
  if (!ctx) return;
  const HostGraph hu = grid_graph(20, 20), hd = directed_graph(500);
  DevGraph du, dd;
  CHECK(prepare(ctx, hu, du) == CENTRA_OK, "prepare grid: %s", centra_last_error(ctx));
  CHECK(prepare(ctx, hd, dd) == CENTRA_OK, "prepare directed: %s", centra_last_error(ctx));
  uint32_t dmax = 0, cbits = 0;
  CHECK(centra_graph_info(dd.g, &dmax, &cbits) == CENTRA_OK, "graph info");
  size_t want_dmax = 0;
  for (const auto& r : hd.in) want_dmax = std::max(want_dmax, r.size());
  CHECK(dmax == want_dmax, "max in-degree %u, want %zu", dmax, want_dmax);

  // a malformed CSR (an unsorted row) is refused and the context stays usable
  {
    HostGraph bad = grid_graph(4, 4);
    std::swap(bad.col_idx[0], bad.col_idx[1]);
    DevGraph db;
    CHECK(prepare(ctx, bad, db) == CENTRA_EINVAL && db.g == nullptr, "unsorted row accepted");
    release(db);
  }
  for (const auto* pair : {&du, &dd}) {
    const HostGraph& h = pair == &du ? hu : hd;
    say(h.directed ? "device: directed graph" : "device: grid graph");
    const Sample s = paths(ctx, h, *pair, 3000, false);
    (void)paths(ctx, h, *pair, 3000, true);
    const Cover c = greedy(ctx, s, h.n, 8, false);
    check_cover(c, s, h.n);
    const Cover c2 = greedy(ctx, s, h.n, 8, true);
    CHECK(c2.picks == c.picks && c2.cov == c.cov, "allocation-free greedy differs");
    mcera(ctx, s, h.n);
    triangles(ctx, h, *pair);
    kpaths(ctx, h, *pair);
    stream_chain(ctx, h, *pair);
    say("device: samplers, cover, AMCERA and the stream-ordered chain done");
    for (uint32_t space : {CENTRA_SPACE_SHORTEST_PATHS, CENTRA_SPACE_TRIANGLES, CENTRA_SPACE_KPATHS,
                           CENTRA_SPACE_PATHS_BIDIR}) {
      if (space == CENTRA_SPACE_TRIANGLES && h.directed) continue;
      progressive(ctx, h, *pair, params(space, CENTRA_METHOD_CENTRA));
    }
    progressive(ctx, h, *pair, params(CENTRA_SPACE_SHORTEST_PATHS, CENTRA_METHOD_HEDGE_P));
  }
  centra_sampler_stats st{};
  CHECK(centra_sampler_stats_get(ctx, &st, 1) == CENTRA_OK && st.samples > 0, "sampler stats");
  say("device: Algorithm 1 runs done");
  engine(ctx, du, dd, 0);
  engine(ctx, du, dd, CENTRA_ENGINE_NO_GRAPHS | CENTRA_ENGINE_NO_TUNE | CENTRA_ENGINE_NO_CACHE);
  (void)centra_context_log(ctx);
  release(du);
  release(dd);
  centra_destroy(ctx);
}

}  // namespace

int main(int argc, char** argv) {
  const bool gpu = argc > 1 && std::strcmp(argv[1], "--gpu") == 0;
  host_checks();
  std::printf("host checks done\n");
  std::fflush(stdout);
  if (gpu) {
    device_checks();
    say("device checks done");
  } else {
    centra_ctx* ctx = nullptr;
    const int rc = centra_create(0, 0, &ctx);
    CHECK(rc == CENTRA_EHIP && ctx == nullptr, "create without a device: rc %d", rc);
  }
  std::printf("%d failed checks\n", g_fail);
  std::fflush(stdout);
  // Leaks are checked here, after the library has released everything; the
  // process then ends without the HIP runtime's own teardown, which frees
  // its allocations after the sanitizer's device allocator hook is gone.
  __lsan_do_leak_check();
  _exit(g_fail ? 1 : 0);
}
