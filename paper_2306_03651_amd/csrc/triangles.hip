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
// those above b.
//
// Each arc's common neighbours come from walking the shorter of its two
// ascending lists and searching the longer one, each search starting where
// the previous one ended.  An arc with at most kHeavy steps is walked by its
// own lane; longer ones (hub-hub arcs: 93% of the steps on a skewed graph)
// by the whole wave, 64 keys per step, with the matches placed in order by
// ballot.  The index also keeps every triangle's c in rank order when it
// fits in an eighth of device memory, so that a sample is a search over the
// arcs plus one gather:
//   - fused: one pass counts the matches and writes them into per-arc slots
//     sized by the walk length (4 bytes per step of all arcs);
//   - compact: a counting pass, then a second pass writes the matches at
//     the triangle prefix (4 bytes per triangle);
//   - walk (no list): each sample walks its arc's lists to its match.
// The first that fits is taken; CENTRA_TRIANGLE_LIST=0 forces the walk and
// CENTRA_TRIANGLE_LIST=compact the compact list (for tests of those paths).
//
// Finding r's arc.  A binary search over the whole prefix (8 bytes per arc)
// misses the cache at nearly every probe.  The index therefore keeps a
// directory of the ranks: with bucket width W (at most kDirBuckets
// buckets), dir[b] is the arc holding rank b W, and dir[nb] the arc holding
// rank T - 1.  Rank r's arc lies in [dir[b], dir[b+1]] for b = r / W, a few
// arcs, so the search there takes one or two lines.
#include <cstdlib>
#include <cstring>

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

constexpr uint32_t kHeavy = 64;   // an arc walked by one lane has at most this many steps
constexpr uint64_t kDirBuckets = 1ull << 22;   // rank directory size bound (16 MB)

// The two lists of arc e = (a, b): walk [w0, w1), search [s0, s1); empty
// unless a < b.  A = N(a) after e, B = N(b) above b; the shorter is walked.
struct ArcLists {
  uint32_t w0, w1, s0, s1;
};

__device__ __forceinline__ ArcLists arc_lists(const uint32_t* row_ptr, const uint32_t* col_idx, uint32_t a,
                                              uint32_t e, uint32_t b) {
  ArcLists L{0, 0, 0, 0};
  if (b <= a) return L;
  const uint32_t a0 = e + 1, a1 = row_ptr[a + 1];
  const uint32_t b1 = row_ptr[b + 1];
  const uint32_t b0 = upper(col_idx, row_ptr[b], b1, b);
  const bool walk_a = a1 - a0 <= b1 - b0;
  L.w0 = walk_a ? a0 : b0;
  L.w1 = walk_a ? a1 : b1;
  L.s0 = walk_a ? b0 : a0;
  L.s1 = walk_a ? b1 : a1;
  return L;
}

__device__ __forceinline__ uint32_t readlane_u32(uint32_t v, int l) {
  return static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(v), l));
}

__global__ void k_arc_src(uint32_t n, const uint32_t* row_ptr, uint32_t* src) {
  const uint32_t v = (blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  if (v >= n) return;
  for (uint32_t e = row_ptr[v] + lane_id(); e < row_ptr[v + 1]; e += kWave) src[e] = v;
}

// walk length of every arc (the capacity of its slot in the fused list)
__global__ void k_tri_cap(uint64_t n_arcs, const uint32_t* row_ptr, const uint32_t* col_idx, const uint32_t* src,
                          uint32_t* cap) {
  const uint64_t e = blockIdx.x * uint64_t(blockDim.x) + threadIdx.x;
  if (e >= n_arcs) return;
  const ArcLists L = arc_lists(row_ptr, col_idx, src[e], static_cast<uint32_t>(e), col_idx[e]);
  cap[e] = L.w1 - L.w0;
}

// cnt[e] = the number of common neighbours above b of arc e; with kWrite they
// are also written, ascending, at tri_c[out_off[e]...].
template <bool kWrite>
__global__ void __launch_bounds__(256) k_tri_arcs(uint64_t n_arcs, const uint32_t* row_ptr, const uint32_t* col_idx,
                                                  const uint32_t* src, const uint64_t* out_off, uint32_t* tri_c,
                                                  uint32_t* cnt) {
  const uint64_t e = blockIdx.x * uint64_t(blockDim.x) + threadIdx.x;
  const int lane = lane_id();
  ArcLists L{0, 0, 0, 0};
  if (e < n_arcs) L = arc_lists(row_ptr, col_idx, src[e], static_cast<uint32_t>(e), col_idx[e]);
  const uint32_t w = L.w1 - L.w0;
  const uint64_t off = kWrite && w ? out_off[e] : 0;
  uint32_t found = 0;
  if (w <= kHeavy) {
    uint32_t lo = L.s0;
    for (uint32_t i = L.w0; i < L.w1; ++i) {
      const uint32_t c = col_idx[i];
      const uint32_t p = upper(col_idx, lo, L.s1, c);
      if (p > lo && col_idx[p - 1] == c) {
        if (kWrite) tri_c[off + found] = c;
        ++found;
      }
      lo = p;
    }
  }
  // heavy arcs of this wave, one at a time, by all 64 lanes
  uint64_t heavy = __ballot(w > kHeavy);
  while (heavy) {
    const int h = __ffsll(static_cast<unsigned long long>(heavy)) - 1;
    heavy &= heavy - 1;
    const uint32_t w0 = readlane_u32(L.w0, h), w1 = readlane_u32(L.w1, h);
    const uint32_t s1 = readlane_u32(L.s1, h);
    const uint64_t hoff = kWrite ? (uint64_t(readlane_u32(static_cast<uint32_t>(off >> 32), h)) << 32) |
                                       readlane_u32(static_cast<uint32_t>(off), h)
                                 : 0;
    uint32_t lo = readlane_u32(L.s0, h), n = 0;
    for (uint32_t base = w0; base < w1; base += kWave) {
      const uint32_t i = base + lane;
      uint32_t c = 0, p = lo;
      bool hit = false;
      if (i < w1) {
        c = col_idx[i];
        p = upper(col_idx, lo, s1, c);
        hit = p > lo && col_idx[p - 1] == c;
      }
      const uint64_t m = __ballot(hit);
      if (kWrite && hit) tri_c[hoff + n + __popcll(m & ((1ull << lane) - 1))] = c;
      n += __popcll(m);
      // keys ascend across steps: the next search starts at the last key's place
      const uint32_t last = w1 - 1 - base < uint32_t(kWave) ? w1 - 1 - base : uint32_t(kWave - 1);
      lo = readlane_u32(p, static_cast<int>(last));
    }
    if (lane == h) found = n;
  }
  if (e < n_arcs) cnt[e] = found;
}

// The want-th (1-based) common neighbour above b of arc e, walking its lists
// (the sampler's path when no list is kept).
__device__ uint32_t nth_common(const uint32_t* row_ptr, const uint32_t* col_idx, uint32_t a, uint32_t e, uint32_t b,
                               uint32_t want) {
  const ArcLists L = arc_lists(row_ptr, col_idx, a, e, b);
  uint32_t lo = L.s0, found = 0;
  for (uint32_t i = L.w0; i < L.w1; ++i) {
    const uint32_t c = col_idx[i];
    const uint32_t p = upper(col_idx, lo, L.s1, c);
    if (p > lo && col_idx[p - 1] == c && ++found == want) return c;
    lo = p;
  }
  return kUnseen;
}

// dir[b] = the arc holding rank b W for the buckets starting in arc e, and
// dir[nb] = the arc holding rank T - 1 (every rank lies in exactly one arc
// with a positive count)
__global__ void k_tri_dir(uint64_t n_arcs, const uint64_t* prefix, uint64_t T, uint64_t W, uint64_t nb,
                          uint32_t* dir) {
  const uint64_t e = blockIdx.x * uint64_t(blockDim.x) + threadIdx.x;
  if (e >= n_arcs) return;
  const uint64_t c0 = prefix[e], c1 = prefix[e + 1];
  if (c1 == c0) return;
  for (uint64_t b = (c0 + W - 1) / W; b * W < c1; ++b) dir[b] = static_cast<uint32_t>(e);
  if (c0 <= T - 1 && T - 1 < c1) dir[nb] = static_cast<uint32_t>(e);
}

__global__ void k_tri_sample(uint32_t count, uint64_t first, uint64_t seed, uint32_t instance, uint64_t T,
                             uint64_t n_arcs, const uint64_t* prefix, const uint32_t* dir, uint64_t W,
                             const uint32_t* src, const uint32_t* row_ptr, const uint32_t* col_idx,
                             const uint64_t* list_off, const uint32_t* tri_c, uint64_t base, uint64_t* he_off,
                             uint32_t* he_nodes) {
  const uint32_t x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x > count) return;
  he_off[x] = base + 3ull * x;
  if (x == count) return;
  WordStream st(seed, first + x, instance, 5);
  const uint64_t r = bounded(st, T);
  // the arc e with prefix[e] <= r < prefix[e + 1]: prefix[lo] <= r and
  // prefix[hi] > r (or hi = n_arcs) hold throughout
  uint64_t lo = 0, hi = n_arcs;
  if (dir) {
    const uint64_t b = r / W;
    lo = dir[b];
    hi = uint64_t(dir[b + 1]) + 1;
  }
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
  const uint32_t c = list_off ? tri_c[list_off[e] + (r - prefix[e])]
                              : nth_common(row_ptr, col_idx, a, e, b, static_cast<uint32_t>(r - prefix[e]) + 1);
  he_nodes[3ull * x] = a;
  he_nodes[3ull * x + 1] = b;
  he_nodes[3ull * x + 2] = c;
}

static int read_u64(centra_ctx* ctx, const uint64_t* d, uint64_t* h, hipStream_t s) {
  CENTRA_HIP(ctx, hipGetLastError());
  CENTRA_HIP(ctx, hipMemcpyAsync(h, d, 8, hipMemcpyDeviceToHost, s));
  CENTRA_HIP(ctx, hipStreamSynchronize(s));
  return CENTRA_OK;
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
  if ((rc = ensure(ctx, g->tri_src, (A ? A : 1) * 4, false, s))) return rc;
  if ((rc = ensure(ctx, g->tri_prefix, (A + 1) * 8, false, s))) return rc;
  DevBuf cnt;
  if ((rc = ensure(ctx, cnt, (A ? A : 1) * 4, false, s))) return rc;
  uint32_t* src = static_cast<uint32_t*>(g->tri_src.ptr);
  uint64_t* prefix = static_cast<uint64_t*>(g->tri_prefix.ptr);
  uint32_t* cn = static_cast<uint32_t*>(cnt.ptr);
  const dim3 grid_a(static_cast<unsigned>((A + 255) / 256 ? (A + 255) / 256 : 1));
  const uint64_t wthreads = uint64_t(g->n) * kWave;
  hipLaunchKernelGGL(k_arc_src, dim3(static_cast<unsigned>((wthreads + 255) / 256)), dim3(256), 0, s, g->n,
                     g->row_ptr, src);
  // room for a list
  size_t free_b = 0, total_b = 0;
  if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
    (void)hipGetLastError();
    total_b = 0;
  }
  const char* mode = getenv("CENTRA_TRIANGLE_LIST");
  const uint64_t room = mode && mode[0] == '0' ? 0 : total_b / 8;
  const bool try_fused = !(mode && strcmp(mode, "compact") == 0);
  uint32_t* list = nullptr;
  const uint64_t* list_off = nullptr;
  g->tri_list_off = nullptr;
  if (A && room && try_fused) {
    uint64_t cap_total = 0;
    if (!(rc = ensure(ctx, g->tri_cap, (A + 1) * 8, false, s))) {
      hipLaunchKernelGGL(k_tri_cap, grid_a, dim3(256), 0, s, A, g->row_ptr, g->col_idx, src, cn);
      uint64_t* cap = static_cast<uint64_t*>(g->tri_cap.ptr);
      if (!(rc = excl_scan_u32_to_u64(ctx, cn, cap, A, s))) rc = read_u64(ctx, cap + A, &cap_total, s);
    }
    if (rc == CENTRA_EHIP) {
      release(ctx, cnt);
      return rc;
    }
    if (!rc && cap_total && cap_total * 4 <= room && ensure(ctx, g->tri_c, cap_total * 4, false, s) == CENTRA_OK) {
      list = static_cast<uint32_t*>(g->tri_c.ptr);
      list_off = static_cast<const uint64_t*>(g->tri_cap.ptr);
    } else {
      release(ctx, g->tri_cap);
      ctx->err.clear();   // no room for the fused list is not an error
    }
    rc = CENTRA_OK;
  }
  if (A) {
    if (list)
      hipLaunchKernelGGL(k_tri_arcs<true>, grid_a, dim3(256), 0, s, A, g->row_ptr, g->col_idx, src, list_off, list,
                         cn);
    else
      hipLaunchKernelGGL(k_tri_arcs<false>, grid_a, dim3(256), 0, s, A, g->row_ptr, g->col_idx, src, list_off, list,
                         cn);
  }
  uint64_t total = 0;
  if (!(rc = excl_scan_u32_to_u64(ctx, cn, prefix, A, s))) rc = read_u64(ctx, prefix + A, &total, s);
  if (!rc && !list && total && total * 4 <= room && ensure(ctx, g->tri_c, total * 4, false, s) == CENTRA_OK) {
    // compact list: a second pass writes the matches at the triangle prefix
    list = static_cast<uint32_t*>(g->tri_c.ptr);
    list_off = prefix;
    hipLaunchKernelGGL(k_tri_arcs<true>, grid_a, dim3(256), 0, s, A, g->row_ptr, g->col_idx, src, list_off, list,
                       cn);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess)
      rc = fail(ctx, CENTRA_EHIP, "triangles: list failed");
  }
  release(ctx, cnt);
  if (rc) {
    release(ctx, g->tri_c);
    release(ctx, g->tri_cap);
    return rc;
  }
  ctx->err.clear();   // a refused list is not an error: samples walk instead
  g->tri_dir_w = 0;
  if (total) {
    // the rank directory (optional: without it samples search the whole prefix)
    // Test hook: CENTRA_TRIANGLE_DIR_BUCKETS lowers the bucket bound, so
    // that small graphs get buckets wider than one rank.
    uint64_t max_buckets = kDirBuckets;
    if (const char* nb_env = getenv("CENTRA_TRIANGLE_DIR_BUCKETS")) {
      const unsigned long long v = strtoull(nb_env, nullptr, 0);
      if (v >= 1 && v < max_buckets) max_buckets = v;
    }
    const uint64_t W = (total + max_buckets - 1) / max_buckets;
    const uint64_t nb = (total + W - 1) / W;
    if (A < (1ull << 32) && ensure(ctx, g->tri_dir, (nb + 1) * 4, false, s) == CENTRA_OK) {
      hipLaunchKernelGGL(k_tri_dir, grid_a, dim3(256), 0, s, A, prefix, total, W, nb,
                         static_cast<uint32_t*>(g->tri_dir.ptr));
      if (hipGetLastError() == hipSuccess && hipStreamSynchronize(s) == hipSuccess) {
        g->tri_dir_w = W;
      } else {
        release(ctx, g->tri_dir);
        ctx->err.clear();
        (void)hipGetLastError();
      }
    } else {
      ctx->err.clear();
    }
  }
  if (total == 0) {
    release(ctx, g->tri_c);
    release(ctx, g->tri_cap);
    list_off = nullptr;
  }
  g->tri_list_off = list_off;
  g->tri_total = total;
  *T = total;
  return CENTRA_OK;
}

int sample_triangles_into(centra_ctx* ctx, centra_graph* g, uint64_t seed, uint32_t instance, uint64_t first,
                          uint32_t count, uint64_t* he_off, uint64_t base, uint32_t* he_nodes, hipStream_t s,
                          bool timed) {
  uint64_t T = 0;
  int rc = triangle_index(ctx, g, &T, s);
  if (rc) return rc;
  if (T == 0) return fail(ctx, CENTRA_EINVAL, "triangles: the graph has no triangle");
  if (timed) CENTRA_HIP(ctx, hipEventRecord(ctx->ev[4], s));
  hipLaunchKernelGGL(k_tri_sample, dim3((count + 1 + 255) / 256), dim3(256), 0, s, count, first, seed, instance, T,
                     g->n_arcs, static_cast<const uint64_t*>(g->tri_prefix.ptr),
                     g->tri_dir_w ? static_cast<const uint32_t*>(g->tri_dir.ptr) : nullptr, g->tri_dir_w,
                     static_cast<const uint32_t*>(g->tri_src.ptr), g->row_ptr, g->col_idx, g->tri_list_off,
                     static_cast<const uint32_t*>(g->tri_c.ptr), base, he_off, he_nodes);
  CENTRA_HIP(ctx, hipGetLastError());
  if (timed) CENTRA_HIP(ctx, hipEventRecord(ctx->ev[5], s));
  return CENTRA_OK;
}

}  // namespace centra
