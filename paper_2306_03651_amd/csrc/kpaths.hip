// kappa-path hyperedges on gfx950 (the kappa-path centrality's hyperedge
// space, Sec. 3.1: the node sets of simple paths of length at most kappa;
// the paper names the space but no sampler).
//
// Sample x is the random simple walk of the kappa-path centrality, drawn
// from the Philox stream (seed, x, instance, tag 6): the start
// s = bounded(n), the length l = 1 + bounded(kappa), then l times a move
// from the current node v to the r-th (r = bounded(f)) of v's f
// out-neighbours not yet on the walk, in ascending id, stopping early when
// f = 0.  The hyperedge is the walk after s (at most kappa nodes).
//
// One thread per walk.  A step never scans v's row: the walk's nodes (at
// most kappa + 1) are binary searched in the row, their positions sorted,
// and the r-th free entry is r's index shifted past every occupied position
// at or before it.  So a step costs O(kappa log deg(v)) loads whatever the
// degree, which matters on hubs, where degree-biased walks spend their
// steps.  One walk pass writes each walk's nodes to a staging slab of kappa
// entries and its length; a scan turns the lengths into offsets, and a
// streaming gather lays the nodes out in sample order.
#include "common.hpp"
#include "internal.hpp"

namespace centra {

constexpr uint32_t kMaxKappa = CENTRA_MAX_KAPPA;

// first index in [lo, hi) of idx with idx[i] >= key
__device__ __forceinline__ uint32_t lower_pos(const uint32_t* idx, uint32_t lo, uint32_t hi, uint32_t key) {
  while (lo < hi) {
    const uint32_t mid = lo + (hi - lo) / 2;
    if (idx[mid] < key)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

// Walk x: lens[x] = its length, its nodes at stage[x * kappa ...].
__global__ __launch_bounds__(256) void k_kpath(uint32_t count, uint64_t first, uint64_t seed, uint32_t instance,
                                               uint32_t n, uint32_t kappa, const uint32_t* row_ptr,
                                               const uint32_t* col_idx, uint32_t* lens, uint32_t* stage) {
  const uint32_t x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= count) return;
  WordStream st(seed, first + x, instance, 6);
  const uint32_t s = static_cast<uint32_t>(bounded(st, n));
  const uint32_t l = 1 + static_cast<uint32_t>(bounded(st, kappa));
  uint32_t walk[kMaxKappa + 1];
  uint32_t pos[kMaxKappa + 1];
  walk[0] = s;
  uint32_t len = 0, v = s;
  uint32_t* out = stage + size_t(x) * kappa;
  while (len < l) {
    const uint32_t lo = row_ptr[v], hi = row_ptr[v + 1];
    // row positions of the walk's nodes, ascending (insertion sort)
    uint32_t np = 0;
    for (uint32_t i = 0; i <= len; ++i) {
      const uint32_t w = walk[i];
      const uint32_t p = lower_pos(col_idx, lo, hi, w);
      if (p < hi && col_idx[p] == w) {
        uint32_t j = np++;
        while (j > 0 && pos[j - 1] > p) {
          pos[j] = pos[j - 1];
          --j;
        }
        pos[j] = p;
      }
    }
    const uint32_t f = (hi - lo) - np;
    if (f == 0) break;
    uint32_t idx = lo + static_cast<uint32_t>(bounded(st, f));
    for (uint32_t j = 0; j < np && pos[j] <= idx; ++j) ++idx;
    v = col_idx[idx];
    walk[++len] = v;
    out[len - 1] = v;
  }
  lens[x] = len;
}

// he_nodes[off[x] - off[0] + i] = stage[x * kappa + i], i < lens[x]: one
// thread per staged entry slot (coalesced reads of the slabs).
__global__ void k_kpath_gather(uint32_t count, uint32_t kappa, const uint32_t* lens, const uint32_t* stage,
                               const uint64_t* off, uint32_t* he_nodes) {
  const uint64_t e = blockIdx.x * uint64_t(blockDim.x) + threadIdx.x;
  const uint64_t x = e / kappa;
  if (x >= count) return;
  const uint32_t i = static_cast<uint32_t>(e - x * kappa);
  if (i < lens[x]) he_nodes[off[x] - off[0] + i] = stage[e];
}

__global__ void k_add_u64(uint64_t* a, uint64_t n, uint64_t add) {
  for (uint64_t i = blockIdx.x * uint64_t(blockDim.x) + threadIdx.x; i < n; i += uint64_t(gridDim.x) * blockDim.x)
    a[i] += add;
}

static dim3 grid_of(uint64_t threads) { return dim3(static_cast<unsigned>((threads + 255) / 256 ? (threads + 255) / 256 : 1)); }

int kpath_count(centra_ctx* ctx, const centra_graph* g, uint32_t kappa, uint64_t seed, uint32_t instance,
                uint64_t first, uint32_t count, uint64_t* off, hipStream_t s, bool timed) {
  if (kappa == 0 || kappa > kMaxKappa) return fail(ctx, CENTRA_EINVAL, "kappa-paths: kappa outside [1, 16]");
  int rc = ensure(ctx, ctx->kp_len, (size_t(count) + 1) * 4, false, s);
  if (rc) return rc;
  if ((rc = ensure(ctx, ctx->kp_stage, (size_t(count) * kappa + 1) * 4, false, s))) return rc;
  uint32_t* lens = static_cast<uint32_t*>(ctx->kp_len.ptr);
  if (timed) CENTRA_HIP(ctx, hipEventRecord(ctx->ev[4], s));
  if (count)
    hipLaunchKernelGGL(k_kpath, grid_of(count), dim3(256), 0, s, count, first, seed, instance, g->n, kappa, g->row_ptr,
                       g->col_idx, lens, static_cast<uint32_t*>(ctx->kp_stage.ptr));
  CENTRA_HIP(ctx, hipGetLastError());
  if (timed) CENTRA_HIP(ctx, hipEventRecord(ctx->ev[5], s));
  return excl_scan_u32_to_u64(ctx, lens, off, count, s);
}

int kpath_write(centra_ctx* ctx, const centra_graph* g, uint32_t kappa, uint64_t seed, uint32_t instance,
                uint64_t first, uint32_t count, uint64_t* off, uint64_t base, uint32_t* he_nodes, hipStream_t s,
                bool timed) {
  if (timed) CENTRA_HIP(ctx, hipEventRecord(ctx->ev[6], s));
  if (count)
    hipLaunchKernelGGL(k_kpath_gather, grid_of(uint64_t(count) * kappa), dim3(256), 0, s, count, kappa,
                       static_cast<const uint32_t*>(ctx->kp_len.ptr), static_cast<const uint32_t*>(ctx->kp_stage.ptr),
                       off, he_nodes);
  CENTRA_HIP(ctx, hipGetLastError());
  if (timed) CENTRA_HIP(ctx, hipEventRecord(ctx->ev[7], s));
  if (base) hipLaunchKernelGGL(k_add_u64, grid_of(uint64_t(count) + 1), dim3(256), 0, s, off, uint64_t(count) + 1, base);
  CENTRA_HIP(ctx, hipGetLastError());
  return CENTRA_OK;
}

}  // namespace centra
