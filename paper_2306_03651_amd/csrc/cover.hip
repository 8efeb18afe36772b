// Node -> sample incidence and greedyCover(k, H) on gfx950.
//
// The incidence is the transpose of the hyperedge lists: deg[u] =
// deg_H(u), inc_off (exclusive scan of deg), inc[p] = sample id and
// inc_node[p] = u for p in [inc_off[u], inc_off[u+1]).  The order of the
// samples inside a row is irrelevant to every consumer.
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
__global__ void k_scatter_inc_agg(const uint64_t* he_off, const uint32_t* he_nodes, uint64_t m, uint32_t n,
                                  uint64_t* cursor, uint32_t* inc, uint32_t* inc_node) {
  __shared__ AggTable tab;
  __shared__ uint64_t base[kAggSize];
  agg_init(tab);
  __syncthreads();
  const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
  const uint64_t s0 = blockIdx.x * uint64_t(blockDim.x) + threadIdx.x;
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

int build_incidence(centra_ctx* ctx, uint32_t n, uint64_t m, const uint64_t* he_off, const uint32_t* he_nodes,
                    hipStream_t s) {
  uint64_t I = 0;
  CENTRA_HIP(ctx, hipMemcpyAsync(&I, he_off + m, 8, hipMemcpyDeviceToHost, s));
  CENTRA_HIP(ctx, hipStreamSynchronize(s));
  int rc;
  if ((rc = ensure(ctx, ctx->deg, size_t(n) * 4, false, s))) return rc;
  if ((rc = ensure(ctx, ctx->inc_off, (size_t(n) + 1) * 8, false, s))) return rc;
  if ((rc = ensure(ctx, ctx->inc_cursor, size_t(n) * 8, false, s))) return rc;
  if ((rc = ensure(ctx, ctx->inc, (I ? I : 1) * 4, false, s))) return rc;
  if ((rc = ensure(ctx, ctx->inc_node, (I ? I : 1) * 4, false, s))) return rc;
  uint32_t* deg = static_cast<uint32_t*>(ctx->deg.ptr);
  uint64_t* off = static_cast<uint64_t*>(ctx->inc_off.ptr);
  uint64_t* cur = static_cast<uint64_t*>(ctx->inc_cursor.ptr);
  fill_u32(deg, 0, n, s);
  if (I)
    hipLaunchKernelGGL(k_count_deg_agg, dim3(grid_for(I, 256, 2048)), dim3(256), 0, s, he_nodes, I, n, deg,
                       ctx->d_flags);
  CENTRA_HIP(ctx, hipGetLastError());
  if ((rc = excl_scan_u32_to_u64(ctx, deg, off, n, s))) return rc;
  hipLaunchKernelGGL(k_copy_u64, dim3(grid_for(n, 256)), dim3(256), 0, s, off, cur, size_t(n));
  if (m)
    hipLaunchKernelGGL(k_scatter_inc_agg, dim3(grid_for(m, 256, 2048)), dim3(256), 0, s, he_off, he_nodes, m, n, cur,
                       static_cast<uint32_t*>(ctx->inc.ptr), static_cast<uint32_t*>(ctx->inc_node.ptr));
  CENTRA_HIP(ctx, hipGetLastError());
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
// n_part per-workgroup maxima of the argmax.
__global__ __launch_bounds__(kCoverBlock) void k_cover(const uint64_t* part, uint32_t n_part, uint64_t* best,
                                                       const uint64_t* inc_off, const uint32_t* inc,
                                                       const uint64_t* he_off, const uint32_t* he_nodes, uint32_t n,
                                                       uint32_t* covered, int32_t* gain, uint64_t* newcov) {
  __shared__ uint64_t red[kCoverBlock / kWave];
  __shared__ AggTable tab;
  uint64_t key = 0;
  for (uint32_t i = threadIdx.x; i < n_part; i += kCoverBlock) key = part[i] > key ? part[i] : key;
  key = block_max_u64<kCoverBlock>(key, red);
  if (blockIdx.x == 0 && threadIdx.x == 0) *best = key;
  if ((key >> 32) == 0) return;
  const uint32_t u = 0xFFFFFFFFu - static_cast<uint32_t>(key);
  const uint64_t b = inc_off[u], e = inc_off[u + 1];
  const uint64_t first = b + blockIdx.x * uint64_t(kCoverBlock);
  if (first >= e) return;   // uniform per workgroup: nothing of the row lands here
  agg_init(tab);
  __syncthreads();
  uint64_t cnt = 0;
  for (uint64_t p = first + threadIdx.x; p < e; p += uint64_t(gridDim.x) * kCoverBlock) {
    const uint32_t s = inc[p];
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
    hipLaunchKernelGGL(k_cover, dim3(gc), dim3(kCoverBlock), 0, s, part, ga, best + r, ioff, inc, he_off, he_nodes, n,
                       cov, gain, newcov + r);
  }
  hipLaunchKernelGGL(k_greedy_finish, dim3(1), dim3(64), 0, s, best, newcov, k, picks, cov_cum, n_picked);
  CENTRA_HIP(ctx, hipGetLastError());
  return CENTRA_OK;
}

}  // namespace centra
