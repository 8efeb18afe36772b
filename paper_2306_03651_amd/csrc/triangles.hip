// Triangle hyperedges on gfx950 (the triangle centrality's hyperedge space,
// Sec. 3.1: the node sets of the triangles of an undirected graph, drawn
// uniformly).
//
// Triangles {a < b < c} are ranked in lexicographic order of (a, b, c).  The
// index, built once per graph: for every arc a -> b with a < b the number of
// triangles {a, b, c} with c > b, i.e. |{c > b : c in N(a) and c in N(b)}|,
// and the exclusive prefix of those counts over the arcs in CSR order (which
// is (a, b) order).  Sample x draws r = bounded(T) from the Philox stream
// (seed, x, instance, tag 5); the arc whose prefix interval holds r gives
// (a, b), and c is the (r - prefix)-th common neighbour above b in ascending
// order.  Rows are ascending, so the entries of N(a) after b are exactly
// those above b.  One thread per arc and per sample: the per-arc work is an
// intersection of two sorted lists, walking the shorter one and binary
// searching the longer.  When the list of every triangle's c (4 bytes per
// triangle, in rank order) fits in an eighth of device memory it is kept
// with the index, and a sample is a binary search over the arcs plus one
// gather; otherwise the sample walks its arc's intersection.
#include "common.hpp"
#include "internal.hpp"

namespace centra {

// first index in [lo, hi) of idx with idx[i] > key
__device__ __forceinline__ uint32_t upper(const uint32_t* idx, uint32_t lo, uint32_t hi, uint32_t key) {
  while (lo < hi) {
    const uint32_t mid = lo + (hi - lo) / 2;
    if (idx[mid] <= key)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

__device__ __forceinline__ bool contains(const uint32_t* idx, uint32_t lo, uint32_t hi, uint32_t key) {
  const uint32_t p = upper(idx, lo, hi, key);
  return p > lo && idx[p - 1] == key;
}

// The common neighbours above b of arc e = (a, b): the lists A = N(a) after
// e and B = N(b) above b, both ascending.  Passes them to visit(c) in
// ascending order by walking the shorter list; stops after `limit` matches
// or at the end; returns the number visited.
template <typename Visit>
__device__ uint32_t common_above(const uint32_t* row_ptr, const uint32_t* col_idx, uint32_t a, uint32_t e, uint32_t b,
                                 uint32_t limit, Visit visit) {
  const uint32_t a0 = e + 1, a1 = row_ptr[a + 1];
  const uint32_t b1 = row_ptr[b + 1];
  const uint32_t b0 = upper(col_idx, row_ptr[b], b1, b);
  const bool walk_a = a1 - a0 <= b1 - b0;
  const uint32_t w0 = walk_a ? a0 : b0, w1 = walk_a ? a1 : b1;
  const uint32_t s0 = walk_a ? b0 : a0, s1 = walk_a ? b1 : a1;
  uint32_t found = 0;
  for (uint32_t i = w0; i < w1 && found < limit; ++i) {
    const uint32_t c = col_idx[i];
    if (contains(col_idx, s0, s1, c)) {
      ++found;
      visit(c);
    }
  }
  return found;
}

__global__ void k_arc_src(uint32_t n, const uint32_t* row_ptr, uint32_t* src) {
  const uint32_t v = (blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  if (v >= n) return;
  for (uint32_t e = row_ptr[v] + lane_id(); e < row_ptr[v + 1]; e += kWave) src[e] = v;
}

// Writes the c of every triangle of arc e at rank order: tri_c[prefix[e] + i].
__global__ void k_tri_list(uint64_t n_arcs, const uint32_t* row_ptr, const uint32_t* col_idx, const uint32_t* src,
                           const uint64_t* prefix, uint32_t* tri_c) {
  const uint64_t e = blockIdx.x * uint64_t(blockDim.x) + threadIdx.x;
  if (e >= n_arcs || prefix[e + 1] == prefix[e]) return;
  uint32_t* out = tri_c + prefix[e];
  common_above(row_ptr, col_idx, src[e], static_cast<uint32_t>(e), col_idx[e], kUnseen,
               [&](uint32_t c) { *out++ = c; });
}

__global__ void k_tri_count(uint64_t n_arcs, const uint32_t* row_ptr, const uint32_t* col_idx, const uint32_t* src,
                            uint32_t* cnt) {
  const uint64_t e = blockIdx.x * uint64_t(blockDim.x) + threadIdx.x;
  if (e >= n_arcs) return;
  const uint32_t a = src[e], b = col_idx[e];
  cnt[e] = b > a ? common_above(row_ptr, col_idx, a, static_cast<uint32_t>(e), b, kUnseen, [](uint32_t) {}) : 0u;
}

__global__ void k_tri_sample(uint32_t count, uint64_t first, uint64_t seed, uint32_t instance, uint64_t T,
                             uint64_t n_arcs, const uint64_t* prefix, const uint32_t* src, const uint32_t* row_ptr,
                             const uint32_t* col_idx, const uint32_t* tri_c, uint64_t base, uint64_t* he_off,
                             uint32_t* he_nodes) {
  const uint32_t x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x > count) return;
  he_off[x] = base + 3ull * x;
  if (x == count) return;
  WordStream st(seed, first + x, instance, 5);
  const uint64_t r = bounded(st, T);
  // the arc e with prefix[e] <= r < prefix[e + 1]
  uint64_t lo = 0, hi = n_arcs;
  while (lo + 1 < hi) {
    const uint64_t mid = lo + (hi - lo) / 2;
    if (prefix[mid] <= r)
      lo = mid;
    else
      hi = mid;
  }
  // (the largest such e has a triangle: a later arc with the same prefix
  // would also satisfy prefix <= r)
  const uint32_t e = static_cast<uint32_t>(lo);
  const uint32_t a = src[e], b = col_idx[e];
  uint32_t c = kUnseen;
  if (tri_c) {
    c = tri_c[r];
  } else {
    const uint32_t want = static_cast<uint32_t>(r - prefix[e]) + 1;
    common_above(row_ptr, col_idx, a, e, b, want, [&](uint32_t v) { c = v; });
  }
  he_nodes[3ull * x] = a;
  he_nodes[3ull * x + 1] = b;
  he_nodes[3ull * x + 2] = c;
}

// Builds the triangle index of an undirected graph once; *T receives the
// number of triangles.
int triangle_index(centra_ctx* ctx, centra_graph* g, uint64_t* T, hipStream_t s) {
  if (g->directed) return fail(ctx, CENTRA_ENOTSUP, "triangles: the graph is directed");
  if (g->tri_total != ~0ull) {
    *T = g->tri_total;
    return CENTRA_OK;
  }
  const uint64_t A = g->n_arcs;
  int rc;
  DevBuf cnt;
  if ((rc = ensure(ctx, g->tri_src, (A ? A : 1) * 4, false, s))) return rc;
  if ((rc = ensure(ctx, g->tri_prefix, (A + 1) * 8, false, s))) return rc;
  if ((rc = ensure(ctx, cnt, (A ? A : 1) * 4, false, s))) return rc;
  uint32_t* src = static_cast<uint32_t*>(g->tri_src.ptr);
  uint64_t* prefix = static_cast<uint64_t*>(g->tri_prefix.ptr);
  const uint64_t wthreads = uint64_t(g->n) * kWave;
  hipLaunchKernelGGL(k_arc_src, dim3(static_cast<unsigned>((wthreads + 255) / 256)), dim3(256), 0, s, g->n,
                     g->row_ptr, src);
  if (A)
    hipLaunchKernelGGL(k_tri_count, dim3(static_cast<unsigned>((A + 255) / 256)), dim3(256), 0, s, A, g->row_ptr,
                       g->col_idx, src, static_cast<uint32_t*>(cnt.ptr));
  if (hipGetLastError() != hipSuccess) {
    release(ctx, cnt);
    return fail(ctx, CENTRA_EHIP, "triangles: index launch failed");
  }
  rc = excl_scan_u32_to_u64(ctx, static_cast<uint32_t*>(cnt.ptr), prefix, A, s);
  uint64_t total = 0;
  if (!rc && hipMemcpyAsync(&total, prefix + A, 8, hipMemcpyDeviceToHost, s) == hipSuccess &&
      hipStreamSynchronize(s) == hipSuccess) {
    g->tri_total = total;
    *T = total;
  } else if (!rc) {
    rc = fail(ctx, CENTRA_EHIP, "triangles: index failed");
  }
  release(ctx, cnt);
  if (rc || total == 0) return rc;
  // the list of every triangle's c, when it fits (else samples walk;
  // CENTRA_TRIANGLE_LIST=0 forces the walk, for tests of that path)
  size_t free_b = 0, total_b = 0;
  if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
    (void)hipGetLastError();
    total_b = 0;
  }
  if (const char* v = getenv("CENTRA_TRIANGLE_LIST"))
    if (v[0] == '0') total_b = 0;
  if (total * 4 <= total_b / 8 && ensure(ctx, g->tri_c, total * 4, false, s) == CENTRA_OK) {
    hipLaunchKernelGGL(k_tri_list, dim3(static_cast<unsigned>((A + 255) / 256)), dim3(256), 0, s, A, g->row_ptr,
                       g->col_idx, src, prefix, static_cast<uint32_t*>(g->tri_c.ptr));
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess) {
      release(ctx, g->tri_c);
      return fail(ctx, CENTRA_EHIP, "triangles: list failed");
    }
  } else {
    ctx->err.clear();   // a refused list is not an error: samples walk instead
  }
  return CENTRA_OK;
}

int sample_triangles_into(centra_ctx* ctx, centra_graph* g, uint64_t seed, uint32_t instance, uint64_t first,
                          uint32_t count, uint64_t* he_off, uint64_t base, uint32_t* he_nodes, hipStream_t s) {
  uint64_t T = 0;
  int rc = triangle_index(ctx, g, &T, s);
  if (rc) return rc;
  if (T == 0) return fail(ctx, CENTRA_EINVAL, "triangles: the graph has no triangle");
  hipLaunchKernelGGL(k_tri_sample, dim3((count + 1 + 255) / 256), dim3(256), 0, s, count, first, seed, instance, T,
                     g->n_arcs, static_cast<const uint64_t*>(g->tri_prefix.ptr),
                     static_cast<const uint32_t*>(g->tri_src.ptr), g->row_ptr, g->col_idx,
                     static_cast<const uint32_t*>(g->tri_c.ptr), base, he_off, he_nodes);
  CENTRA_HIP(ctx, hipGetLastError());
  return CENTRA_OK;
}

}  // namespace centra
