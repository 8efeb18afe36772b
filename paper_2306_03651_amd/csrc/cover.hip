// Node -> sample incidence and greedyCover(k, H) on gfx950.
//
// The incidence is the transpose of the hyperedge lists, kept as segments,
// one per batch of samples [m0, m1) appended by the progressive loop (a
// single segment for a one-off call): segment g's offsets seg_off[g][u]
// give u's entries [seg_off[g][u], seg_off[g][u+1]) of inc (sample ids) and
// inc_node (= u); a segment's entries occupy the same index range of inc as
// its hyperedges' entries do of he_nodes.  deg[u] = deg_H(u) over every
// segment.  Appending a batch costs its own entries only, so a run whose
// sample doubles builds each entry once instead of about twice.  At most
// kMaxSegments segments are kept; the next append rebuilds one segment from
// sample 0.  The order of the samples inside a row is irrelevant to every
// consumer.
//
// Greedy keeps gain[u] = number of uncovered hyperedges containing u.  A
// round is two kernels: an argmax over gain packed as (gain << 32 | ~u),
// so the maximum key is the largest gain with the lowest id, each
// workgroup writing the maximum of its slice (no atomics on one word);
// then the covering pass, whose every workgroup first reduces those
// per-workgroup maxima to the pick and then walks its share of the picked
// node's incidence row, marking each newly covered sample in a bitmap
// (atomicOr decides which thread covers it) and decrementing the gain of
// every node of that hyperedge.  All updates
// are integer, so the picks are exactly those of the sequential greedy.
// The rounds run back to back on the stream; the picked node is read from
// device memory, so no host round trip happens between rounds.
#include "common.hpp"
#include "internal.hpp"

namespace centra {

__global__ void k_copy_u64(const uint64_t* src, uint64_t* dst, size_t n) {
  for (size_t i = blockIdx.x * size_t(blockDim.x) + threadIdx.x; i < n; i += size_t(gridDim.x) * blockDim.x)
    dst[i] = src[i];
}

static unsigned grid_for(uint64_t n, unsigned block, unsigned cap = 16384) {
  uint64_t g = (n + block - 1) / block;
  if (g > cap) g = cap;
  return g ? static_cast<unsigned>(g) : 1u;
}

// Per-workgroup aggregation of integer updates to a node-indexed array in
// an LDS hash table (open addressing, linear probing over kAggProbe slots).
// Hub nodes appear in a large fraction of the hyperedges; aggregating turns
// their per-hyperedge atomics into one global atomic per workgroup.  A node
// that finds no slot falls back to a direct global atomic.
constexpr uint32_t kAggBits = 11;
constexpr uint32_t kAggSize = 1u << kAggBits;
constexpr uint32_t kAggProbe = 8;

struct AggTable {
  uint32_t key[kAggSize];
  uint32_t cnt[kAggSize];
};

__device__ __forceinline__ void agg_init(AggTable& t) {
  for (uint32_t i = threadIdx.x; i < kAggSize; i += blockDim.x) {
    t.key[i] = kUnseen;
    t.cnt[i] = 0;
  }
}

// Adds 1 for node v; returns false if the table has no slot for v.
__device__ __forceinline__ bool agg_add(AggTable& t, uint32_t v) {
  const uint32_t h = (v * 0x9E3779B1u) >> (32 - kAggBits);
  for (uint32_t p = 0; p < kAggProbe; ++p) {
    const uint32_t slot = (h + p) & (kAggSize - 1);
    uint32_t k = t.key[slot];
    if (k == kUnseen) k = atomicCAS(&t.key[slot], kUnseen, v);
    if (k == kUnseen || k == v) {
      atomicAdd(&t.cnt[slot], 1u);
      return true;
    }
  }
  return false;
}

// Finds node v's slot (no insert); kUnseen if v has none.
__device__ __forceinline__ uint32_t agg_find(const AggTable& t, uint32_t v) {
  const uint32_t h = (v * 0x9E3779B1u) >> (32 - kAggBits);
  for (uint32_t p = 0; p < kAggProbe; ++p) {
    const uint32_t slot = (h + p) & (kAggSize - 1);
    if (t.key[slot] == v) return slot;
    if (t.key[slot] == kUnseen) return kUnseen;
  }
  return kUnseen;
}

// Transpose with per-workgroup range reservation: pass 1 counts this
// workgroup's entries per node, one atomic per node reserves a range of
// the node's row, pass 2 places the entries (the same grid-stride order in
// both passes).  Nodes without a slot reserve per entry.
__global__ void k_scatter_inc_agg(const uint64_t* he_off, const uint32_t* he_nodes, uint64_t m0, uint64_t m, uint32_t n,
                                  uint64_t* cursor, uint32_t* inc, uint32_t* inc_node) {
  __shared__ AggTable tab;
  __shared__ uint64_t base[kAggSize];
  agg_init(tab);
  __syncthreads();
  const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
  const uint64_t s0 = m0 + blockIdx.x * uint64_t(blockDim.x) + threadIdx.x;
  for (uint64_t s = s0; s < m; s += stride)
    for (uint64_t x = he_off[s]; x < he_off[s + 1]; ++x) {
      const uint32_t u = he_nodes[x];
      if (u < n) (void)agg_add(tab, u);
    }
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < kAggSize; i += blockDim.x) {
    if (tab.key[i] != kUnseen)
      base[i] = atomicAdd(reinterpret_cast<unsigned long long*>(&cursor[tab.key[i]]),
                          static_cast<unsigned long long>(tab.cnt[i]));
    tab.cnt[i] = 0;
  }
  __syncthreads();
  for (uint64_t s = s0; s < m; s += stride)
    for (uint64_t x = he_off[s]; x < he_off[s + 1]; ++x) {
      const uint32_t u = he_nodes[x];
      if (u >= n) continue;
      const uint32_t slot = agg_find(tab, u);
      const uint64_t p = slot != kUnseen
                             ? base[slot] + atomicAdd(&tab.cnt[slot], 1u)
                             : atomicAdd(reinterpret_cast<unsigned long long*>(&cursor[u]), 1ull);
      inc[p] = static_cast<uint32_t>(s);
      inc_node[p] = u;
    }
}

__global__ void k_count_deg_agg(const uint32_t* he_nodes, uint64_t I, uint32_t n, uint32_t* deg, uint32_t* flags) {
  __shared__ AggTable tab;
  agg_init(tab);
  __syncthreads();
  for (uint64_t e = blockIdx.x * uint64_t(blockDim.x) + threadIdx.x; e < I; e += uint64_t(gridDim.x) * blockDim.x) {
    const uint32_t u = he_nodes[e];
    if (u >= n) {
      atomicOr(flags, kErrNodeRange);
      continue;
    }
    if (!agg_add(tab, u)) atomicAdd(&deg[u], 1u);
  }
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < kAggSize; i += blockDim.x)
    if (tab.key[i] != kUnseen) atomicAdd(&deg[tab.key[i]], tab.cnt[i]);
}

__global__ void k_add_u32_to(const uint32_t* a, uint32_t n, uint32_t* acc) {
  for (uint32_t u = blockIdx.x * blockDim.x + threadIdx.x; u < n; u += gridDim.x * blockDim.x) acc[u] += a[u];
}

__global__ void k_offset_u64(uint64_t* a, uint64_t n, uint64_t add) {
  for (uint64_t i = blockIdx.x * uint64_t(blockDim.x) + threadIdx.x; i < n; i += uint64_t(gridDim.x) * blockDim.x)
    a[i] += add;
}

int build_incidence(centra_ctx* ctx, uint32_t n, uint64_t m0, uint64_t m1, const uint64_t* he_off,
                    const uint32_t* he_nodes, hipStream_t s) {
  if (m0 == 0 || ctx->inc_nseg >= kMaxSegments) {   // a new sample, or too many segments: start over
    ctx->inc_nseg = 0;
    m0 = 0;
  }
  uint64_t ends[2] = {0, 0};
  CENTRA_HIP(ctx, hipMemcpyAsync(&ends[0], he_off + m0, 8, hipMemcpyDeviceToHost, s));
  CENTRA_HIP(ctx, hipMemcpyAsync(&ends[1], he_off + m1, 8, hipMemcpyDeviceToHost, s));
  CENTRA_HIP(ctx, hipStreamSynchronize(s));
  const uint64_t I0 = ends[0], I1 = ends[1];
  const uint32_t g = ctx->inc_nseg;
  int rc;
  if ((rc = ensure(ctx, ctx->deg, size_t(n) * 4, g > 0, s))) return rc;
  if ((rc = ensure(ctx, ctx->seg_deg, size_t(n) * 4, false, s))) return rc;
  if ((rc = ensure(ctx, ctx->inc_off, (size_t(g) + 1) * (size_t(n) + 1) * 8, g > 0, s))) return rc;
  if ((rc = ensure(ctx, ctx->inc_cursor, size_t(n) * 8, false, s))) return rc;
  if ((rc = ensure(ctx, ctx->inc, (I1 ? I1 : 1) * 4, g > 0, s))) return rc;
  if ((rc = ensure(ctx, ctx->inc_node, (I1 ? I1 : 1) * 4, g > 0, s))) return rc;
  uint32_t* deg = static_cast<uint32_t*>(ctx->deg.ptr);
  uint32_t* sdeg = static_cast<uint32_t*>(ctx->seg_deg.ptr);
  uint64_t* off = static_cast<uint64_t*>(ctx->inc_off.ptr) + size_t(g) * (size_t(n) + 1);
  uint64_t* cur = static_cast<uint64_t*>(ctx->inc_cursor.ptr);
  if (g == 0) fill_u32(deg, 0, n, s);
  fill_u32(sdeg, 0, n, s);
  if (I1 > I0)
    hipLaunchKernelGGL(k_count_deg_agg, dim3(grid_for(I1 - I0, 256, 2048)), dim3(256), 0, s, he_nodes + I0, I1 - I0, n,
                       sdeg, ctx->d_flags);
  CENTRA_HIP(ctx, hipGetLastError());
  if ((rc = excl_scan_u32_to_u64(ctx, sdeg, off, n, s))) return rc;
  if (I0) hipLaunchKernelGGL(k_offset_u64, dim3(grid_for(uint64_t(n) + 1, 256)), dim3(256), 0, s, off, uint64_t(n) + 1, I0);
  hipLaunchKernelGGL(k_copy_u64, dim3(grid_for(n, 256)), dim3(256), 0, s, off, cur, size_t(n));
  if (m1 > m0)
    hipLaunchKernelGGL(k_scatter_inc_agg, dim3(grid_for(m1 - m0, 256, 2048)), dim3(256), 0, s, he_off, he_nodes, m0, m1,
                       n, cur, static_cast<uint32_t*>(ctx->inc.ptr), static_cast<uint32_t*>(ctx->inc_node.ptr));
  hipLaunchKernelGGL(k_add_u32_to, dim3(grid_for(n, 256)), dim3(256), 0, s, sdeg, n, deg);
  CENTRA_HIP(ctx, hipGetLastError());
  ctx->inc_nseg = g + 1;
  ctx->inc_m0 = m0;
  ctx->inc_I0 = I0;
  ctx->inc_I1 = I1;
  return CENTRA_OK;
}

// ---------------------------------------------------------------------------
__global__ void k_gain_init(const uint32_t* deg, uint32_t n, int32_t* gain) {
  for (uint32_t u = blockIdx.x * blockDim.x + threadIdx.x; u < n; u += gridDim.x * blockDim.x)
    gain[u] = static_cast<int32_t>(deg[u]);
}

constexpr int kArgBlock = 256;

constexpr unsigned kArgGrid = 512;   // workgroups of the argmax (and per-workgroup maxima)

// part[b] = the largest key of the slice of workgroup b (0 if the slice has
// no positive gain)
__global__ __launch_bounds__(kArgBlock) void k_argmax(const int32_t* gain, uint32_t n, uint64_t* part) {
  __shared__ uint64_t red[kArgBlock / kWave];
  uint64_t key = 0;
  for (uint32_t u = blockIdx.x * kArgBlock + threadIdx.x; u < n; u += gridDim.x * kArgBlock) {
    const int32_t g = gain[u];
    const uint64_t k = g > 0 ? (static_cast<uint64_t>(g) << 32) | (0xFFFFFFFFu - u) : 0ull;
    key = k > key ? k : key;
  }
  key = block_max_u64<kArgBlock>(key, red);
  if (threadIdx.x == 0) part[blockIdx.x] = key;
}

constexpr int kCoverBlock = 256;

// best = the round's pick (written by workgroup 0): the largest of the
// n_part per-workgroup maxima of the argmax.  The picked node's rows in the
// n_seg incidence segments are walked as one row (their concatenation), so
// the workgroups share it as they would a single segment's.
__global__ __launch_bounds__(kCoverBlock) void k_cover(const uint64_t* part, uint32_t n_part, uint64_t* best,
                                                       const uint64_t* seg_off, uint32_t n_seg, const uint32_t* inc,
                                                       const uint64_t* he_off, const uint32_t* he_nodes, uint32_t n,
                                                       uint32_t* covered, int32_t* gain, uint64_t* newcov) {
  __shared__ uint64_t red[kCoverBlock / kWave];
  __shared__ AggTable tab;
  __shared__ uint64_t seg_beg[kMaxSegments], seg_pre[kMaxSegments + 1];
  uint64_t key = 0;
  for (uint32_t i = threadIdx.x; i < n_part; i += kCoverBlock) key = part[i] > key ? part[i] : key;
  key = block_max_u64<kCoverBlock>(key, red);
  if (blockIdx.x == 0 && threadIdx.x == 0) *best = key;
  if ((key >> 32) == 0) return;
  const uint32_t u = 0xFFFFFFFFu - static_cast<uint32_t>(key);
  if (threadIdx.x < kWave) {   // segment starts and the prefix of the row lengths (n_seg <= 64)
    const uint32_t g = threadIdx.x;
    uint64_t b = 0, len = 0;
    if (g < n_seg) {
      const uint64_t* o = seg_off + size_t(g) * (size_t(n) + 1);
      b = o[u];
      len = o[u + 1] - b;
    }
    const uint64_t incl = wave_incl_scan_u64(len);
    if (g < n_seg) {
      seg_beg[g] = b;
      seg_pre[g + 1] = incl;
    }
    if (g == 0) seg_pre[0] = 0;
  }
  __syncthreads();
  const uint64_t row = seg_pre[n_seg];
  const uint64_t lead = blockIdx.x * uint64_t(kCoverBlock);
  if (lead >= row) return;   // uniform per workgroup: nothing of the row lands here
  agg_init(tab);
  __syncthreads();
  uint64_t cnt = 0;
  uint32_t g = 0;
  for (uint64_t q = lead + threadIdx.x; q < row; q += uint64_t(gridDim.x) * kCoverBlock) {
    while (q >= seg_pre[g + 1]) ++g;
    const uint32_t s = inc[seg_beg[g] + (q - seg_pre[g])];
    const uint32_t bit = 1u << (s & 31u);
    const uint32_t old = atomicOr(&covered[s >> 5], bit);
    if (old & bit) continue;
    ++cnt;
    for (uint64_t x = he_off[s]; x < he_off[s + 1]; ++x) {
      const uint32_t v = he_nodes[x];
      if (v < n && !agg_add(tab, v)) atomicSub(&gain[v], 1);
    }
  }
  cnt = block_sum_u64<kCoverBlock>(cnt, red);   // contains the barrier before the flush
  for (uint32_t i = threadIdx.x; i < kAggSize; i += kCoverBlock)
    if (tab.key[i] != kUnseen) atomicSub(&gain[tab.key[i]], static_cast<int32_t>(tab.cnt[i]));
  if (threadIdx.x == 0 && cnt) atomicAdd(reinterpret_cast<unsigned long long*>(newcov), cnt);
}

__global__ void k_greedy_finish(const uint64_t* best, const uint64_t* newcov, uint32_t k, uint32_t* picks,
                                uint64_t* cov_cum, uint32_t* n_picked) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  uint64_t cov = 0;
  uint32_t r = 0;
  for (; r < k; ++r) {
    const uint64_t key = best[r];
    if ((key >> 32) == 0) break;
    cov += newcov[r];
    picks[r] = 0xFFFFFFFFu - static_cast<uint32_t>(key);
    cov_cum[r] = cov;
  }
  *n_picked = r;
}

int greedy_on_incidence(centra_ctx* ctx, uint32_t n, uint64_t m, const uint64_t* he_off, const uint32_t* he_nodes,
                        uint32_t k, uint32_t* picks, uint64_t* cov_cum, uint32_t* n_picked, hipStream_t s) {
  int rc;
  if ((rc = ensure(ctx, ctx->gain, size_t(n) * 4, false, s))) return rc;
  if ((rc = ensure(ctx, ctx->covered, ((m + 31) / 32 + 1) * 4, false, s))) return rc;
  if ((rc = ensure(ctx, ctx->best, (size_t(k) + kArgGrid) * 8, false, s))) return rc;
  if ((rc = ensure(ctx, ctx->newcov, size_t(k) * 8, false, s))) return rc;
  int32_t* gain = static_cast<int32_t*>(ctx->gain.ptr);
  uint32_t* cov = static_cast<uint32_t*>(ctx->covered.ptr);
  uint64_t* best = static_cast<uint64_t*>(ctx->best.ptr);
  uint64_t* newcov = static_cast<uint64_t*>(ctx->newcov.ptr);
  hipLaunchKernelGGL(k_gain_init, dim3(grid_for(n, 256)), dim3(256), 0, s, static_cast<const uint32_t*>(ctx->deg.ptr),
                     n, gain);
  fill_u32(cov, 0, (m + 31) / 32 + 1, s);
  fill_u64(best, 0, k, s);
  fill_u64(newcov, 0, k, s);
  const unsigned ga = grid_for(n, kArgBlock, kArgGrid);
  uint64_t* part = best + k;
  const unsigned gc = 1024;
  const uint64_t* ioff = static_cast<const uint64_t*>(ctx->inc_off.ptr);
  const uint32_t* inc = static_cast<const uint32_t*>(ctx->inc.ptr);
  for (uint32_t r = 0; r < k; ++r) {
    hipLaunchKernelGGL(k_argmax, dim3(ga), dim3(kArgBlock), 0, s, gain, n, part);
    hipLaunchKernelGGL(k_cover, dim3(gc), dim3(kCoverBlock), 0, s, part, ga, best + r, ioff, ctx->inc_nseg, inc, he_off,
                       he_nodes, n, cov, gain, newcov + r);
  }
  hipLaunchKernelGGL(k_greedy_finish, dim3(1), dim3(64), 0, s, best, newcov, k, picks, cov_cum, n_picked);
  CENTRA_HIP(ctx, hipGetLastError());
  return CENTRA_OK;
}

}  // namespace centra
