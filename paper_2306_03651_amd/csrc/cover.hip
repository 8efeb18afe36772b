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
#include <mutex>
#include <string>

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
// Entries go to [he_off[m0], he_off[m]) of inc; nothing is written unless
// that range lies within the `limit` entries inc holds, and no write lands
// outside it whatever the offsets (decreasing offsets raise kErrOffsets).
__global__ void k_scatter_inc_agg(const uint64_t* he_off, const uint32_t* he_nodes, uint64_t m0, uint64_t m, uint32_t n,
                                  uint64_t limit, uint64_t* cursor, uint32_t* inc, uint32_t* inc_node,
                                  uint32_t* flags) {
  __shared__ AggTable tab;
  __shared__ uint64_t base[kAggSize];
  const uint64_t I0 = he_off[m0], I1 = he_off[m];
  if (I1 > limit || I0 > I1) return;   // uniform: k_count_deg_agg raised the error
  agg_init(tab);
  __syncthreads();
  const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
  const uint64_t s0 = m0 + blockIdx.x * uint64_t(blockDim.x) + threadIdx.x;
  for (uint64_t s = s0; s < m; s += stride) {
    const uint64_t b = he_off[s], e = he_off[s + 1];
    if (b > e) {
      atomicOr(flags, kErrOffsets);
      continue;
    }
    for (uint64_t x = b < I0 ? I0 : b; x < (e < I1 ? e : I1); ++x) {
      const uint32_t u = he_nodes[x];
      if (u < n) (void)agg_add(tab, u);
    }
  }
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < kAggSize; i += blockDim.x) {
    if (tab.key[i] != kUnseen)
      base[i] = atomicAdd(reinterpret_cast<unsigned long long*>(&cursor[tab.key[i]]),
                          static_cast<unsigned long long>(tab.cnt[i]));
    tab.cnt[i] = 0;
  }
  __syncthreads();
  for (uint64_t s = s0; s < m; s += stride) {
    const uint64_t b = he_off[s], e = he_off[s + 1];
    if (b > e) continue;
    for (uint64_t x = b < I0 ? I0 : b; x < (e < I1 ? e : I1); ++x) {
      const uint32_t u = he_nodes[x];
      if (u >= n) continue;
      const uint32_t slot = agg_find(tab, u);
      const uint64_t p = slot != kUnseen
                             ? base[slot] + atomicAdd(&tab.cnt[slot], 1u)
                             : atomicAdd(reinterpret_cast<unsigned long long*>(&cursor[u]), 1ull);
      if (p >= I1) {   // only with decreasing offsets (flagged above)
        atomicOr(flags, kErrOffsets);
        continue;
      }
      inc[p] = static_cast<uint32_t>(s);
      inc_node[p] = u;
    }
  }
}

// deg[u] += entries of u among he_nodes[he_off[m0], he_off[m1]) (the entry
// range is read on the device; a range beyond `limit` entries counts
// nothing and raises kErrCapacity).
__global__ void k_count_deg_agg(const uint64_t* he_off, uint64_t m0, uint64_t m1, const uint32_t* he_nodes, uint32_t n,
                                uint64_t limit, uint32_t* deg, uint32_t* flags) {
  __shared__ AggTable tab;
  const uint64_t I0 = he_off[m0], I1 = he_off[m1];
  if (I1 > limit || I0 > I1) {   // uniform over the grid
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(flags, I0 > I1 ? kErrOffsets : kErrCapacity);
    return;
  }
  agg_init(tab);
  __syncthreads();
  for (uint64_t e = I0 + blockIdx.x * uint64_t(blockDim.x) + threadIdx.x; e < I1; e += uint64_t(gridDim.x) * blockDim.x) {
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

// a[i] += *add for i < n (the addend read on the device).
__global__ void k_offset_u64(uint64_t* a, uint64_t n, const uint64_t* add) {
  const uint64_t x = *add;
  if (x == 0) return;
  for (uint64_t i = blockIdx.x * uint64_t(blockDim.x) + threadIdx.x; i < n; i += uint64_t(gridDim.x) * blockDim.x)
    a[i] += x;
}

// Launches the build of one incidence segment: samples [m0, m1), whose
// entries [he_off[m0], he_off[m1]) of he_nodes are located on the device
// (span_cap bounds their number, for the launch shapes only; inc and
// inc_node hold `limit` entries, and a segment reaching beyond them is
// left empty with kErrCapacity raised); its offsets go to `off` (absolute
// into inc), its degrees to sdeg, and deg accumulates them (cleared first
// when `first_segment`).  Launches only.
void incidence_segment(uint32_t n, uint64_t m0, uint64_t m1, uint64_t span_cap, uint64_t limit, const uint64_t* he_off,
                       const uint32_t* he_nodes, bool first_segment, uint32_t* deg, uint32_t* sdeg, uint64_t* off,
                       uint64_t* cur, uint32_t* inc, uint32_t* inc_node, uint64_t* scan_tiles, uint32_t* flags,
                       hipStream_t s) {
  if (first_segment) fill_u32(deg, 0, n, s);
  fill_u32(sdeg, 0, n, s);
  if (m1 > m0 && span_cap)
    hipLaunchKernelGGL(k_count_deg_agg, dim3(grid_for(span_cap, 256, 2048)), dim3(256), 0, s, he_off, m0, m1, he_nodes, n,
                       limit, sdeg, flags);
  excl_scan_u32_to_u64_ws(sdeg, off, n, scan_tiles, s);
  if (m0) hipLaunchKernelGGL(k_offset_u64, dim3(grid_for(uint64_t(n) + 1, 256)), dim3(256), 0, s, off, uint64_t(n) + 1,
                             he_off + m0);
  hipLaunchKernelGGL(k_copy_u64, dim3(grid_for(n, 256)), dim3(256), 0, s, off, cur, size_t(n));
  if (m1 > m0)
    hipLaunchKernelGGL(k_scatter_inc_agg, dim3(grid_for(m1 - m0, 256, 2048)), dim3(256), 0, s, he_off, he_nodes, m0, m1,
                       n, limit, cur, inc, inc_node, flags);
  hipLaunchKernelGGL(k_add_u32_to, dim3(grid_for(n, 256)), dim3(256), 0, s, sdeg, n, deg);
}

int build_incidence(centra_ctx* ctx, uint32_t n, uint64_t m0, uint64_t m1, const uint64_t* he_off,
                    const uint32_t* he_nodes, hipStream_t s, uint64_t entry_cap) {
  ctx->ext_inc = false;   // the extend calls' state is valid only after their own builds
  if (m0 == 0 || ctx->inc_nseg >= kMaxSegments) {   // a new sample, or too many segments: start over
    ctx->inc_nseg = 0;
    m0 = 0;
  }
  uint64_t I0 = 0, I1 = entry_cap;
  if (entry_cap == ~0ull) {   // sizes read from the device (one synchronisation)
    uint64_t ends[2] = {0, 0};
    CENTRA_HIP(ctx, hipMemcpyAsync(&ends[0], he_off + m0, 8, hipMemcpyDeviceToHost, s));
    CENTRA_HIP(ctx, hipMemcpyAsync(&ends[1], he_off + m1, 8, hipMemcpyDeviceToHost, s));
    CENTRA_HIP(ctx, hipStreamSynchronize(s));
    I0 = ends[0];
    I1 = ends[1];
  }
  const uint32_t g = ctx->inc_nseg;
  int rc;
  if ((rc = ensure(ctx, ctx->deg, size_t(n) * 4, g > 0, s))) return rc;
  if ((rc = ensure(ctx, ctx->seg_deg, size_t(n) * 4, false, s))) return rc;
  if ((rc = ensure(ctx, ctx->inc_off, (size_t(g) + 1) * (size_t(n) + 1) * 8, g > 0, s))) return rc;
  if ((rc = ensure(ctx, ctx->inc_cursor, size_t(n) * 8, false, s))) return rc;
  if ((rc = ensure(ctx, ctx->inc, (I1 ? I1 : 1) * 4, g > 0, s))) return rc;
  if ((rc = ensure(ctx, ctx->inc_node, (I1 ? I1 : 1) * 4, g > 0, s))) return rc;
  if ((rc = ensure(ctx, ctx->scan_tmp, scan_tile_words(n) * 8, false, s))) return rc;
  if (n <= kIncBucketMaxNodes) {
    if ((rc = ensure(ctx, ctx->inc_ws, incidence_ws_bytes(n, I1 - I0), false, s))) return rc;
    incidence_segment_bucketed(n, m0, m1, I1 - I0, I1, he_off, he_nodes, g == 0, static_cast<uint32_t*>(ctx->deg.ptr),
                               static_cast<uint32_t*>(ctx->seg_deg.ptr),
                               static_cast<uint64_t*>(ctx->inc_off.ptr) + size_t(g) * (size_t(n) + 1),
                               static_cast<uint64_t*>(ctx->inc_cursor.ptr), static_cast<uint32_t*>(ctx->inc.ptr),
                               static_cast<uint32_t*>(ctx->inc_node.ptr), ctx->inc_ws.ptr, ctx->d_flags, s);
  } else {
    incidence_segment(n, m0, m1, I1 - I0, I1, he_off, he_nodes, g == 0, static_cast<uint32_t*>(ctx->deg.ptr),
                      static_cast<uint32_t*>(ctx->seg_deg.ptr),
                      static_cast<uint64_t*>(ctx->inc_off.ptr) + size_t(g) * (size_t(n) + 1),
                      static_cast<uint64_t*>(ctx->inc_cursor.ptr), static_cast<uint32_t*>(ctx->inc.ptr),
                      static_cast<uint32_t*>(ctx->inc_node.ptr), static_cast<uint64_t*>(ctx->scan_tmp.ptr), ctx->d_flags,
                      s);
  }
  CENTRA_HIP(ctx, hipGetLastError());
  ctx->inc_nseg = g + 1;
  ++ctx->inc_gen;
  ctx->inc_m0 = m0;
  ctx->inc_span_cap = I1 - I0;
  ctx->inc_m1 = m1;
  ctx->inc_limit = I1;
  if (ctx->inc_seg_m0.size() < size_t(g) + 1) ctx->inc_seg_m0.resize(size_t(g) + 1);
  ctx->inc_seg_m0[g] = m0;
  return CENTRA_OK;
}

int incidence_reserve(centra_ctx* ctx, uint32_t n, uint64_t entries, uint32_t segments, hipStream_t s) {
  int rc;
  if ((rc = ensure(ctx, ctx->deg, size_t(n) * 4, true, s))) return rc;
  if ((rc = ensure(ctx, ctx->seg_deg, size_t(n) * 4, false, s))) return rc;
  if ((rc = ensure(ctx, ctx->inc_off, (size_t(segments) + 1) * (size_t(n) + 1) * 8, true, s))) return rc;
  if ((rc = ensure(ctx, ctx->inc_cursor, size_t(n) * 8, false, s))) return rc;
  if ((rc = ensure(ctx, ctx->inc, (entries ? entries : 1) * 4, true, s))) return rc;
  if ((rc = ensure(ctx, ctx->inc_node, (entries ? entries : 1) * 4, true, s))) return rc;
  if (n <= kIncBucketMaxNodes && (rc = ensure(ctx, ctx->inc_ws, incidence_ws_bytes(n, entries), false, s))) return rc;
  return ensure(ctx, ctx->scan_tmp, scan_tile_words(n) * 8, false, s);
}

// ---------------------------------------------------------------------------
__global__ void k_gain_init(const uint32_t* deg, uint32_t n, int32_t* gain) {
  for (uint32_t u = blockIdx.x * blockDim.x + threadIdx.x; u < n; u += gridDim.x * blockDim.x)
    gain[u] = static_cast<int32_t>(deg[u]);
}

constexpr int kArgBlock = 256;

constexpr unsigned kArgGrid = 512;   // workgroups of the argmax (and per-workgroup maxima)

constexpr int kArgUnroll = 4;       // 4-node groups a thread loads at once

__device__ __forceinline__ uint64_t gain_key(int32_t g, uint32_t u) {
  return g > 0 ? (static_cast<uint64_t>(g) << 32) | (0xFFFFFFFFu - u) : 0ull;
}

// The largest key (gain << 32 | ~u, 0 if no positive gain) of the slice
// of workgroup b of nb: the 4-node groups b*kArgBlock + i*nb*kArgBlock
// (gain is 16-byte aligned), kArgUnroll groups per thread loaded together
// so that their round trips overlap; workgroup 0 also takes the n % 4
// nodes past the last group.  The maximum of the keys does not depend on
// how the nodes are split.
__device__ __forceinline__ uint64_t argmax_slice(const int32_t* gain, uint32_t n, uint32_t b, uint32_t nb,
                                                 uint64_t* red) {
  uint64_t key = 0;
  const uint32_t nv = n >> 2;
  const int4* g4 = reinterpret_cast<const int4*>(gain);
  const uint32_t stride = nb * kArgBlock;
  for (uint32_t w = b * kArgBlock + threadIdx.x; w < nv; w += kArgUnroll * stride) {
    int4 x[kArgUnroll];
#pragma unroll
    for (int j = 0; j < kArgUnroll; ++j) {
      const uint32_t wj = w + j * stride;
      x[j] = wj < nv ? g4[wj] : make_int4(0, 0, 0, 0);
    }
#pragma unroll
    for (int j = 0; j < kArgUnroll; ++j) {
      const uint32_t u = (w + j * stride) * 4;   // groups past nv hold zeros: key 0
      uint64_t k = gain_key(x[j].x, u);
      k = max(k, gain_key(x[j].y, u + 1));
      k = max(k, gain_key(x[j].z, u + 2));
      k = max(k, gain_key(x[j].w, u + 3));
      key = max(key, k);
    }
  }
  if (b == 0 && threadIdx.x < (n & 3u)) {
    const uint32_t u = (nv << 2) + threadIdx.x;
    key = max(key, gain_key(gain[u], u));
  }
  return block_max_u64<kArgBlock>(key, red);
}

// part[b] = the largest key of the slice of workgroup b (0 if the slice has
// no positive gain)
__global__ __launch_bounds__(kArgBlock) void k_argmax(const int32_t* gain, uint32_t n, uint64_t* part) {
  __shared__ uint64_t red[kArgBlock / kWave];
  const uint64_t key = argmax_slice(gain, n, blockIdx.x, gridDim.x, red);
  if (threadIdx.x == 0) part[blockIdx.x] = key;
}

constexpr int kCoverBlock = 256;

// LDS of a covering walk.
struct CoverShared {
  AggTable tab;
  uint64_t red[kCoverBlock / kWave];
  uint64_t seg_beg[kMaxSegments], seg_pre[kMaxSegments + 1];
  uint32_t scan[kCoverBlock / kWave + 1];
  uint64_t hbeg[kCoverBlock];  // he_off of the step's newly covered samples
  uint32_t hoff[kCoverBlock];  // exclusive prefix of their hyperedge sizes
};

// The walk of one covering pass, workgroup b of nb, for the pick u: its
// share of u's incidence rows in the n_seg segments walked as one row
// (their concatenation), one entry per thread per step.  A step marks the
// newly covered samples among its entries, then the workgroup decrements
// the gains of all their nodes together (the concatenation of their
// hyperedges split evenly over the threads), so long hyperedges (paths of
// thousands of nodes) are spread over the workgroup instead of walked by
// one thread.
__device__ __forceinline__ void cover_walk(uint32_t u, const uint64_t* seg_off, uint32_t n_seg, const uint32_t* inc,
                                           const uint64_t* he_off, const uint32_t* he_nodes, uint32_t n,
                                           uint32_t* covered, int32_t* gain, uint64_t* newcov, uint32_t b, uint32_t nb,
                                           CoverShared& sh) {
  if (threadIdx.x < kWave) {   // segment starts and the prefix of the row lengths (n_seg <= 64)
    const uint32_t g = threadIdx.x;
    uint64_t rb = 0, len = 0;
    if (g < n_seg) {
      const uint64_t* o = seg_off + size_t(g) * (size_t(n) + 1);
      rb = o[u];
      len = o[u + 1] - rb;
    }
    const uint64_t incl = wave_incl_scan_u64(len);
    if (g < n_seg) {
      sh.seg_beg[g] = rb;
      sh.seg_pre[g + 1] = incl;
    }
    if (g == 0) sh.seg_pre[0] = 0;
  }
  __syncthreads();
  const uint64_t row = sh.seg_pre[n_seg];
  const uint64_t lead = b * uint64_t(kCoverBlock);
  if (lead >= row) {   // uniform per workgroup: nothing of the row lands here
    __syncthreads();   // seg_* are reused by the caller's next item
    return;
  }
  agg_init(sh.tab);
  __syncthreads();
  uint64_t cnt = 0;
  uint32_t g = 0;
  const uint64_t stride = uint64_t(nb) * kCoverBlock;
  for (uint64_t base = lead; base < row; base += stride) {   // uniform trip count
    const uint64_t q = base + threadIdx.x;
    uint32_t len = 0;
    uint64_t h0 = 0;
    if (q < row) {
      while (q >= sh.seg_pre[g + 1]) ++g;
      const uint32_t s = inc[sh.seg_beg[g] + (q - sh.seg_pre[g])];
      // the hyperedge's bounds are loaded before the covering atomic
      // returns, so the two round trips overlap
      h0 = he_off[s];
      const uint64_t h1 = he_off[s + 1];
      const uint32_t bit = 1u << (s & 31u);
      const uint32_t old = atomicOr(&covered[s >> 5], bit);
      if (!(old & bit)) {   // newly covered
        ++cnt;
        len = static_cast<uint32_t>(h1 - h0);
      }
    }
    uint32_t total;
    const uint32_t off = block_excl_scan_u32<kCoverBlock>(len, &total, sh.scan);
    sh.hbeg[threadIdx.x] = h0;
    sh.hoff[threadIdx.x] = off;
    __syncthreads();
    for (uint32_t e = threadIdx.x; e < total; e += kCoverBlock) {
      // the sample holding entry e: the last i with hoff[i] <= e and a
      // nonempty hyperedge (empty ones repeat their successor's offset)
      int lo = 0, hi = kCoverBlock - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (sh.hoff[mid] <= e)
          lo = mid;
        else
          hi = mid - 1;
      }
      const uint32_t v = he_nodes[sh.hbeg[lo] + (e - sh.hoff[lo])];
      if (v < n && !agg_add(sh.tab, v)) atomicSub(&gain[v], 1);
    }
    __syncthreads();
  }
  cnt = block_sum_u64<kCoverBlock>(cnt, sh.red);   // contains the barrier before the flush
  for (uint32_t i = threadIdx.x; i < kAggSize; i += kCoverBlock)
    if (sh.tab.key[i] != kUnseen) atomicSub(&gain[sh.tab.key[i]], static_cast<int32_t>(sh.tab.cnt[i]));
  if (threadIdx.x == 0 && cnt) atomicAdd(reinterpret_cast<unsigned long long*>(newcov), cnt);
  __syncthreads();   // the table and seg_* are reused by the caller's next item
}

// One covering pass, workgroup b of nb: reduces the n_part per-workgroup
// maxima to the round's pick (workgroup 0 writes it to *best), then walks
// its share of the pick's rows.
__device__ __forceinline__ void cover_pass(const uint64_t* part, uint32_t n_part, uint64_t* best, const uint64_t* seg_off,
                                           uint32_t n_seg, const uint32_t* inc, const uint64_t* he_off,
                                           const uint32_t* he_nodes, uint32_t n, uint32_t* covered, int32_t* gain,
                                           uint64_t* newcov, uint32_t b, uint32_t nb, CoverShared& sh) {
  static_assert(kArgGrid <= 2 * kCoverBlock, "two maxima per thread");
  const uint64_t p0 = threadIdx.x < n_part ? part[threadIdx.x] : 0ull;
  const uint64_t p1 = threadIdx.x + kCoverBlock < n_part ? part[threadIdx.x + kCoverBlock] : 0ull;
  const uint64_t key = block_max_u64<kCoverBlock>(p0 > p1 ? p0 : p1, sh.red);
  if (b == 0 && threadIdx.x == 0) *best = key;
  if ((key >> 32) == 0) return;
  cover_walk(0xFFFFFFFFu - static_cast<uint32_t>(key), seg_off, n_seg, inc, he_off, he_nodes, n, covered, gain, newcov,
             b, nb, sh);
}

// best = the round's pick (written by workgroup 0): the largest of the
// n_part per-workgroup maxima of the argmax.
__global__ __launch_bounds__(kCoverBlock) void k_cover(const uint64_t* part, uint32_t n_part, uint64_t* best,
                                                       const uint64_t* seg_off, uint32_t n_seg, const uint32_t* inc,
                                                       const uint64_t* he_off, const uint32_t* he_nodes, uint32_t n,
                                                       uint32_t* covered, int32_t* gain, uint64_t* newcov) {
  __shared__ CoverShared sh;
  cover_pass(part, n_part, best, seg_off, n_seg, inc, he_off, he_nodes, n, covered, gain, newcov, blockIdx.x, gridDim.x,
             sh);
}

// ---------------------------------------------------------------------------
// Greedy of many queries at once (the engine's fused rounds): blockIdx.y
// selects the query's descriptor; a query whose k is reached, or that is
// inactive (k = 0), leaves its workgroups at once.  The round number comes
// from device memory (round_base[0] + r_local), so a captured sequence of
// rounds can be replayed for the next rounds after the base is advanced.
//
// Candidate lists.  Gains only decrease, so once every node of gain >= tau
// has been collected into a list, every node outside the list stays below
// tau; while the list's largest gain is >= tau, the argmax over the list
// (largest gain, lowest id) is the argmax over all nodes, and a round reads
// the list's gains instead of all n.  A query cycles through three modes,
// decided after each round from device state:
//   full     every workgroup scans its slice of all n gains and adds a
//            histogram of them (8 bins per octave); after the round, tau is
//            the lowest bin bound whose bins and those above hold at most
//            kCandMax nodes (if any);
//   compact  a full scan that also appends every node of gain >= tau to the
//            list (at most kCandMax: gains were at most the histogram's);
//   list     one workgroup scans the list.
// The round after a list's largest gain falls below tau is full again.
constexpr uint32_t kCandMax = 8192;
constexpr uint32_t kGainBins = 256;
constexpr uint32_t kModeFull = 0, kModeCompact = 1, kModeList = 2;

// Bin of a positive gain: 8 bins per bit length, by the 3 bits below the
// leading one (nondecreasing in g).
__device__ __forceinline__ uint32_t gain_bin(uint32_t g) {
  const uint32_t bl = 32u - __clz(g);
  const uint32_t sub = bl >= 4 ? (g >> (bl - 4)) & 7u : (g << (4 - bl)) & 7u;
  return (bl - 1) * 8 + sub;
}

// Smallest gain of bin b (or of the next nonempty bin above it).
__device__ __forceinline__ uint32_t bin_min(uint32_t b) {
  const uint32_t bl = b / 8 + 1, sub = b % 8;
  if (bl >= 4) return (8u + sub) << (bl - 4);
  for (uint32_t g = 1; g < 16; ++g)
    if (gain_bin(g) >= b) return g;
  return 16;
}

__global__ __launch_bounds__(256) void k_greedy_init_multi(const GreedyDesc* d) {
  const GreedyDesc q = d[blockIdx.y];
  if (q.k == 0) return;
  const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
  const uint64_t i0 = blockIdx.x * uint64_t(blockDim.x) + threadIdx.x;
  for (uint64_t u = i0; u < q.n; u += stride) q.gain[u] = static_cast<int32_t>(q.deg[u]);
  for (uint64_t w = i0; w < (q.m + 31) / 32 + 1; w += stride) q.covered[w] = 0;
  for (uint64_t r = i0; r < q.k; r += stride) {
    q.best[r] = 0;
    q.newcov[r] = 0;
  }
  for (uint64_t b = i0; b < kGainBins; b += stride) q.hist[b] = 0;
  if (i0 == 0) {
    q.cst[0] = kModeFull;
    q.cst[1] = 0;
    q.cst[2] = 0;
  }
}

// Items (query, slice b of S): the argmax of every query's slices, or of its
// list (slice 0), grid-strided so that finished queries and list-mode
// slices cost one check each instead of a workgroup launch.
__global__ __launch_bounds__(kArgBlock) void k_argmax_multi(const GreedyDesc* d, uint32_t n_q, uint32_t S,
                                                            const uint32_t* round_base, uint32_t r_local) {
  __shared__ uint64_t red[kArgBlock / kWave];
  __shared__ uint32_t hist[kGainBins];
  const uint32_t r = round_base[0] + r_local;
  const uint64_t items = uint64_t(n_q) * S;
  for (uint64_t it = blockIdx.x; it < items; it += gridDim.x) {
    const GreedyDesc& q = d[it / S];
    const uint32_t b = static_cast<uint32_t>(it % S);
    if (r >= q.k) continue;
    const uint32_t mode = q.cst[0];
    if (mode == kModeList) {
      if (b != 0) continue;
      const uint32_t cnt = min(q.cst[2], kCandMax);
      uint64_t key = 0;
      for (uint32_t i = threadIdx.x; i < cnt; i += kArgBlock) {
        const uint32_t u = q.cand[i];
        const int32_t g = q.gain[u];
        const uint64_t k = g > 0 ? (static_cast<uint64_t>(g) << 32) | (0xFFFFFFFFu - u) : 0ull;
        key = k > key ? k : key;
      }
      key = block_max_u64<kArgBlock>(key, red);
      if (threadIdx.x == 0) q.part[0] = key;
      continue;
    }
    const uint32_t tau = q.cst[1];
    if (mode == kModeFull) {
      for (uint32_t i = threadIdx.x; i < kGainBins; i += kArgBlock) hist[i] = 0;
      __syncthreads();
    }
    uint64_t key = 0;
    for (uint32_t u = b * kArgBlock + threadIdx.x; u < q.n; u += S * kArgBlock) {
      const int32_t g = q.gain[u];
      if (g <= 0) continue;
      const uint64_t k = (static_cast<uint64_t>(g) << 32) | (0xFFFFFFFFu - u);
      key = k > key ? k : key;
      if (mode == kModeFull) {
        atomicAdd(&hist[gain_bin(static_cast<uint32_t>(g))], 1u);
      } else if (static_cast<uint32_t>(g) >= tau) {
        const uint32_t at = atomicAdd(&q.cst[2], 1u);
        if (at < kCandMax) q.cand[at] = u;
      }
    }
    key = block_max_u64<kArgBlock>(key, red);   // contains barriers
    if (threadIdx.x == 0) q.part[b] = key;
    if (mode == kModeFull) {
      for (uint32_t i = threadIdx.x; i < kGainBins; i += kArgBlock)
        if (hist[i]) atomicAdd(&q.hist[i], hist[i]);
      __syncthreads();
    }
  }
}

// One workgroup per query: the round's pick from the argmax maxima (S of
// them, or one in list mode), written to best[r]; 0 once a round found no
// positive gain.  cst[3] receives the pick's row length over the segments.
__global__ __launch_bounds__(256) void k_pick_multi(const GreedyDesc* d, uint32_t S, const uint32_t* round_base,
                                                    uint32_t r_local) {
  __shared__ uint64_t red[256 / kWave];
  const GreedyDesc& q = d[blockIdx.x];
  const uint32_t r = round_base[0] + r_local;
  if (r >= q.k) return;
  if (r > 0 && (q.best[r - 1] >> 32) == 0) {
    if (threadIdx.x == 0) q.best[r] = 0;
    return;
  }
  const uint32_t parts = q.cst[0] == kModeList ? 1u : S;
  uint64_t key = 0;
  for (uint32_t i = threadIdx.x; i < parts; i += 256) key = q.part[i] > key ? q.part[i] : key;
  key = block_max_u64<256>(key, red);
  uint64_t len = 0;
  if ((key >> 32) != 0) {
    const uint32_t u = 0xFFFFFFFFu - static_cast<uint32_t>(key);
    for (uint32_t g = threadIdx.x; g < q.n_seg; g += 256) {
      const uint64_t* o = q.seg_off + size_t(g) * (size_t(q.n) + 1);
      len += o[u + 1] - o[u];
    }
  }
  len = block_sum_u64<256>(len, red);
  if (threadIdx.x == 0) {
    q.best[r] = key;
    q.cst[3] = static_cast<uint32_t>(len < 0xFFFFFFFFull ? len : 0xFFFFFFFFull);
  }
}

// Items (query, part b of S): the covering walk of each query's pick.
__global__ __launch_bounds__(kCoverBlock) void k_cover_multi(const GreedyDesc* d, uint32_t n_q, uint32_t S,
                                                             const uint32_t* round_base, uint32_t r_local) {
  __shared__ CoverShared sh;
  const uint32_t r = round_base[0] + r_local;
  const uint64_t items = uint64_t(n_q) * S;
  for (uint64_t it = blockIdx.x; it < items; it += gridDim.x) {
    const GreedyDesc& q = d[it / S];
    const uint32_t b = static_cast<uint32_t>(it % S);
    if (r >= q.k) continue;
    const uint64_t key = q.best[r];
    if ((key >> 32) == 0) continue;
    if (uint64_t(b) * kCoverBlock >= q.cst[3]) continue;   // nothing of the row lands here
    cover_walk(0xFFFFFFFFu - static_cast<uint32_t>(key), q.seg_off, q.n_seg, q.inc, q.he_off, q.he_nodes, q.n,
               q.covered, q.gain, q.newcov + r, b, S, sh);
  }
}

// After a round: the next round's mode (see the candidate lists above).
__global__ __launch_bounds__(256) void k_greedy_post_multi(const GreedyDesc* d, const uint32_t* round_base,
                                                           uint32_t r_local) {
  __shared__ uint64_t red[256 / kWave];
  __shared__ uint32_t pick;
  const GreedyDesc& q = d[blockIdx.x];
  const uint32_t r = round_base[0] + r_local;
  if (r >= q.k) return;
  const uint32_t mode = q.cst[0];
  if (mode == kModeFull) {
    if (threadIdx.x == 0) {
      // lowest bin whose bins and those above hold at most kCandMax nodes
      uint32_t cum = 0, found = kGainBins;
      for (int b = kGainBins - 1; b >= 0; --b) {
        if (cum + q.hist[b] > kCandMax) break;
        cum += q.hist[b];
        found = static_cast<uint32_t>(b);
      }
      pick = cum > 0 && found < kGainBins ? found : kGainBins;
    }
    __syncthreads();
    if (threadIdx.x == 0 && pick < kGainBins) {
      q.cst[1] = bin_min(pick);
      q.cst[2] = 0;
      q.cst[0] = kModeCompact;
    }
    for (uint32_t b = threadIdx.x; b < kGainBins; b += 256) q.hist[b] = 0;
    return;
  }
  // list or compact: keep using the list while its largest gain is >= tau
  // (a list that overflowed is incomplete: never used)
  if (q.cst[2] > kCandMax) {
    if (threadIdx.x == 0) q.cst[0] = kModeFull;
    return;
  }
  const uint32_t cnt = q.cst[2];
  uint64_t mx = 0;
  for (uint32_t i = threadIdx.x; i < cnt; i += 256) {
    const int32_t g = q.gain[q.cand[i]];
    mx = g > 0 && static_cast<uint64_t>(g) > mx ? static_cast<uint64_t>(g) : mx;
  }
  mx = block_max_u64<256>(mx, red);
  if (threadIdx.x == 0) q.cst[0] = mx >= q.cst[1] && mx > 0 ? kModeList : kModeFull;
}

__global__ void k_round_advance(uint32_t* round_base, uint32_t by) {
  if (threadIdx.x == 0 && blockIdx.x == 0) round_base[0] += by;
}

__global__ void k_greedy_finish_multi(const GreedyDesc* d) {
  const GreedyDesc& q = d[blockIdx.x];
  if (q.k == 0 || threadIdx.x != 0) return;
  uint64_t cov = 0;
  uint32_t r = 0;
  for (; r < q.k; ++r) {
    const uint64_t key = q.best[r];
    if ((key >> 32) == 0) break;
    cov += q.newcov[r];
    q.picks[r] = 0xFFFFFFFFu - static_cast<uint32_t>(key);
    q.cov_cum[r] = cov;
  }
  *q.n_picked = r;
}

void greedy_multi_init(const GreedyDesc* d, uint32_t n_q, uint32_t max_n, hipStream_t s) {
  hipLaunchKernelGGL(k_greedy_init_multi, dim3(grid_for(max_n, 256, 1024), n_q), dim3(256), 0, s, d);
}

// Slices per query of the multi-query argmax: at least 16 nodes per thread,
// at most kArgGrid.
static uint32_t argmax_slices(uint32_t max_n) {
  return grid_for((uint64_t(max_n) + 15) / 16, kArgBlock, kArgGrid);
}

void greedy_multi_rounds(const GreedyDesc* d, uint32_t n_q, uint32_t max_n, uint32_t cover_grid, uint32_t* round_base,
                         uint32_t rounds, hipStream_t s) {
  const uint32_t Sa = argmax_slices(max_n);
  const unsigned ga = grid_for(uint64_t(n_q) * Sa, 1, 4096);
  const unsigned gc = grid_for(uint64_t(n_q) * cover_grid, 1, 4096);
  for (uint32_t r = 0; r < rounds; ++r) {
    hipLaunchKernelGGL(k_argmax_multi, dim3(ga), dim3(kArgBlock), 0, s, d, n_q, Sa, round_base, r);
    hipLaunchKernelGGL(k_pick_multi, dim3(n_q), dim3(256), 0, s, d, Sa, round_base, r);
    hipLaunchKernelGGL(k_cover_multi, dim3(gc), dim3(kCoverBlock), 0, s, d, n_q, cover_grid, round_base, r);
    hipLaunchKernelGGL(k_greedy_post_multi, dim3(n_q), dim3(256), 0, s, d, round_base, r);
  }
  hipLaunchKernelGGL(k_round_advance, dim3(1), dim3(64), 0, s, round_base, rounds);
}

void greedy_multi_finish(const GreedyDesc* d, uint32_t n_q, hipStream_t s) {
  hipLaunchKernelGGL(k_greedy_finish_multi, dim3(n_q), dim3(64), 0, s, d);
}

uint32_t greedy_cand_words() { return kCandMax; }
uint32_t greedy_hist_words() { return kGainBins; }

uint32_t greedy_part_words() { return kArgGrid; }

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

// Launches greedy's k rounds on an incidence of n_seg segments (offsets
// seg_off, entries inc, degrees deg): gain u32[n], covered u32[m/32 + 1],
// best u64[k + kArgGrid] and newcov u64[k] are the round state.  Launches
// only.
static void greedy_kernels(uint32_t n, uint64_t m, const uint64_t* he_off, const uint32_t* he_nodes, uint32_t k,
                           const uint32_t* deg, const uint64_t* seg_off, uint32_t n_seg, const uint32_t* inc,
                           int32_t* gain, uint32_t* cov, uint64_t* best, uint64_t* newcov, uint32_t* picks,
                           uint64_t* cov_cum, uint32_t* n_picked, hipStream_t s) {
  hipLaunchKernelGGL(k_gain_init, dim3(grid_for(n, 256)), dim3(256), 0, s, deg, n, gain);
  fill_u32(cov, 0, (m + 31) / 32 + 1, s);
  fill_u64(best, 0, k, s);
  fill_u64(newcov, 0, k, s);
  const unsigned ga = grid_for(n, kArgBlock, kArgGrid);
  uint64_t* part = best + k;
  const unsigned gc = 1024;
  for (uint32_t r = 0; r < k; ++r) {
    hipLaunchKernelGGL(k_argmax, dim3(ga), dim3(kArgBlock), 0, s, gain, n, part);
    hipLaunchKernelGGL(k_cover, dim3(gc), dim3(kCoverBlock), 0, s, part, ga, best + r, seg_off, n_seg, inc, he_off,
                       he_nodes, n, cov, gain, newcov + r);
  }
  hipLaunchKernelGGL(k_greedy_finish, dim3(1), dim3(64), 0, s, best, newcov, k, picks, cov_cum, n_picked);
}

int greedy_reserve(centra_ctx* ctx, uint32_t n, uint64_t m, uint32_t k, hipStream_t s) {
  int rc;
  if ((rc = ensure(ctx, ctx->gain, size_t(n) * 4, false, s))) return rc;
  if ((rc = ensure(ctx, ctx->covered, ((m + 31) / 32 + 1) * 4, false, s))) return rc;
  if ((rc = ensure(ctx, ctx->best, (size_t(k) + kArgGrid) * 8, false, s))) return rc;
  return ensure(ctx, ctx->newcov, size_t(k) * 8, false, s);
}

int greedy_on_incidence(centra_ctx* ctx, uint32_t n, uint64_t m, const uint64_t* he_off, const uint32_t* he_nodes,
                        uint32_t k, uint32_t* picks, uint64_t* cov_cum, uint32_t* n_picked, hipStream_t s) {
  int rc;
  if ((rc = ensure(ctx, ctx->gain, size_t(n) * 4, false, s))) return rc;
  if ((rc = ensure(ctx, ctx->covered, ((m + 31) / 32 + 1) * 4, false, s))) return rc;
  if ((rc = ensure(ctx, ctx->best, (size_t(k) + kArgGrid) * 8, false, s))) return rc;
  if ((rc = ensure(ctx, ctx->newcov, size_t(k) * 8, false, s))) return rc;
  greedy_kernels(n, m, he_off, he_nodes, k, static_cast<const uint32_t*>(ctx->deg.ptr),
                 static_cast<const uint64_t*>(ctx->inc_off.ptr), ctx->inc_nseg,
                 static_cast<const uint32_t*>(ctx->inc.ptr), static_cast<int32_t*>(ctx->gain.ptr),
                 static_cast<uint32_t*>(ctx->covered.ptr), static_cast<uint64_t*>(ctx->best.ptr),
                 static_cast<uint64_t*>(ctx->newcov.ptr), picks, cov_cum, n_picked, s);
  CENTRA_HIP(ctx, hipGetLastError());
  return CENTRA_OK;
}

// ---------------------------------------------------------------------------
// Greedy cover without allocation.  Every workspace of one greedy call (the
// single incidence segment, the round state, the scan tiles and an error
// word) is carved from `scratch`, a fixed array in device memory that each
// GPU holds for the life of the process.  Host code never passes the
// array's name to a kernel (on the host it is only a stand-in for the
// symbol): its device address is looked up once per device with
// hipGetSymbolAddress and kept in g_scratch_ptr.
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

static constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Bytes of scratch a greedy call on (n, m, I entries, k) carves.
size_t static_greedy_bytes(uint32_t n, uint64_t m, uint64_t I, uint32_t k) {
  const size_t N = n;
  return align256(4) + align256(N * 4) * 3 + align256((N + 1) * 8) + align256(N * 8) + align256((I ? I : 1) * 4) * 2 +
         align256(((m + 31) / 32 + 1) * 4) + align256((size_t(k) + kArgGrid) * 8) + align256(size_t(k) * 8) +
         align256(scan_tile_words(N) * 8);
}

int greedy_cover_static(uint32_t n, uint64_t m, const uint64_t* he_off, const uint32_t* he_nodes, uint32_t k,
                        uint32_t* picks, uint64_t* cov_cum, uint32_t* n_picked, hipStream_t s, std::string* err) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    *err = "greedy_cover_noalloc: no current HIP device";
    return CENTRA_EHIP;
  }
  char* base = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
      void* p = nullptr;
      e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !p) {
        *err = std::string("greedy_cover_noalloc: hipGetSymbolAddress failed: ") + hipGetErrorString(e);
        return CENTRA_EHIP;
      }
      g_scratch_ptr[dev] = p;
    }
    base = static_cast<char*>(g_scratch_ptr[dev]);
  }
  uint64_t I = 0;
  if ((e = hipMemcpyAsync(&I, he_off + m, 8, hipMemcpyDeviceToHost, s)) != hipSuccess ||
      (e = hipStreamSynchronize(s)) != hipSuccess) {
    *err = std::string("greedy_cover_noalloc: reading he_off[m]: ") + hipGetErrorString(e);
    return CENTRA_EHIP;
  }
  if (I && !he_nodes) {
    *err = "greedy_cover_noalloc: he_nodes is NULL";
    return CENTRA_EINVAL;
  }
  const size_t need = static_greedy_bytes(n, m, I, k);
  if (need > kStaticScratchBytes) {
    *err = "greedy_cover_noalloc: n = " + std::to_string(n) + ", m = " + std::to_string(m) + ", " +
           std::to_string(I) + " entries and k = " + std::to_string(k) + " need " + std::to_string(need) +
           " bytes of scratch; the fixed maximum is " + std::to_string(kStaticScratchBytes);
    return CENTRA_ENOSPC;
  }
  const size_t N = n;
  size_t at = 0;
  auto carve = [&](size_t bytes) {
    char* p = base + at;
    at += align256(bytes);
    return static_cast<void*>(p);
  };
  uint32_t* flags = static_cast<uint32_t*>(carve(4));
  uint32_t* deg = static_cast<uint32_t*>(carve(N * 4));
  uint32_t* sdeg = static_cast<uint32_t*>(carve(N * 4));
  int32_t* gain = static_cast<int32_t*>(carve(N * 4));
  uint64_t* off = static_cast<uint64_t*>(carve((N + 1) * 8));
  uint64_t* cur = static_cast<uint64_t*>(carve(N * 8));
  uint32_t* inc = static_cast<uint32_t*>(carve((I ? I : 1) * 4));
  uint32_t* inc_node = static_cast<uint32_t*>(carve((I ? I : 1) * 4));
  uint32_t* cov = static_cast<uint32_t*>(carve(((m + 31) / 32 + 1) * 4));
  uint64_t* best = static_cast<uint64_t*>(carve((size_t(k) + kArgGrid) * 8));
  uint64_t* newcov = static_cast<uint64_t*>(carve(size_t(k) * 8));
  uint64_t* tiles = static_cast<uint64_t*>(carve(scan_tile_words(N) * 8));
  // the array keeps the previous call's contents: the error word starts at 0
  // here, and every other region is written before it is read
  fill_u32(flags, 0, 1, s);
  incidence_segment(n, 0, m, I, I, he_off, he_nodes, true, deg, sdeg, off, cur, inc, inc_node, tiles, flags, s);
  greedy_kernels(n, m, he_off, he_nodes, k, deg, off, 1, inc, gain, cov, best, newcov, picks, cov_cum, n_picked, s);
  if ((e = hipGetLastError()) != hipSuccess) {
    *err = std::string("greedy_cover_noalloc: launch failed: ") + hipGetErrorString(e);
    return CENTRA_EHIP;
  }
  uint32_t f = 0;
  if ((e = hipMemcpyAsync(&f, flags, 4, hipMemcpyDeviceToHost, s)) != hipSuccess ||
      (e = hipStreamSynchronize(s)) != hipSuccess) {
    *err = std::string("greedy_cover_noalloc: ") + hipGetErrorString(e);
    return CENTRA_EHIP;
  }
  if (f & kErrNodeRange) {
    *err = "greedy_cover_noalloc: hyperedge node id out of range";
    return CENTRA_EINVAL;
  }
  if (f) {
    *err = "greedy_cover_noalloc: hyperedge offsets decrease";
    return CENTRA_EINVAL;
  }
  return CENTRA_OK;
}

}  // namespace centra
