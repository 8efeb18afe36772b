// Node -> sample incidence of one segment of the hyperedge store, built as
// a bucketed transpose (the greedy step and the AMCERA counts of Algorithm
// 1 read it: a node's row lists the samples whose hyperedges contain it).
//
// The entries of samples [m0, m1) (positions [he_off[m0], he_off[m1]) of
// he_nodes, read on the device) are moved in four passes, with no global
// atomic per entry:
//   1. per workgroup of a fixed grid, an LDS histogram of the entries' node
//      buckets (kBucketNodes consecutive node ids per bucket), written
//      bucket-major; a scan turns them into each (bucket, workgroup)'s
//      place in a bucket-ordered scratch array;
//   2. the same workgroups visit the same samples in the same order and
//      write each entry, (node, sample) in 8 bytes, to its bucket's run;
//   3. buckets are cut into items of at most kItem entries; per item, the
//      nodes' counts in LDS (a node's slot is its id within the bucket);
//      one global add per node present adds them to the segment degrees
//      (a bucket of one item has one add per node); a scan of the degrees
//      gives the rows;
//   4. per item again, one global add per node present reserves the item's
//      share of the node's row, and each entry is written at its place.
// Within a row the order of samples is not fixed (greedy and the counts
// only use the set).  Every access stays inside [he_off[m0], he_off[m1])
// of the store and inside the `limit` entries of the incidence; a segment
// reaching beyond them, or larger than span_cap, is skipped with an error
// bit, as are node ids >= n and decreasing offsets.
#include "common.hpp"
#include "internal.hpp"

namespace centra {

namespace {

constexpr uint32_t kBucketLog = 11;
constexpr uint32_t kBucketNodes = 1u << kBucketLog;
constexpr uint32_t kPartBlock = 256;
constexpr uint32_t kPartGrid = 512;        // workgroups of passes 1 and 2
constexpr uint32_t kItemBlock = 256;
constexpr uint32_t kItem = 16384;          // entries per item (at most)
constexpr uint32_t kItemGrid = 2048;

unsigned grid_of(uint64_t n, unsigned block, unsigned cap = 65535) {
  uint64_t g = (n + block - 1) / block;
  if (g > cap) g = cap;
  return g ? static_cast<unsigned>(g) : 1u;
}

// The segment's entry range, or false (uniform) when it is out of bounds.
__device__ __forceinline__ bool seg_range(const uint64_t* he_off, uint64_t m0, uint64_t m1, uint64_t limit,
                                          uint64_t span_cap, uint64_t* I0, uint64_t* I1) {
  *I0 = he_off[m0];
  *I1 = he_off[m1];
  return *I1 <= limit && *I0 <= *I1 && *I1 - *I0 <= span_cap;
}

// Pass 1: cnt[b * kPartGrid + blk] = entries of bucket b among the samples
// of workgroup blk (samples m0 + blk * kPartBlock + tid, strided by the
// grid).  An out-of-bounds segment counts nothing (and raises the error).
__global__ __launch_bounds__(kPartBlock) void k_inc_bucket_count(const uint64_t* he_off, const uint32_t* he_nodes,
                                                                 uint64_t m0, uint64_t m1, uint32_t n, uint64_t limit,
                                                                 uint64_t span_cap, uint32_t n_buckets, uint32_t* cnt,
                                                                 uint32_t* flags) {
  extern __shared__ uint32_t hist[];
  for (uint32_t b = threadIdx.x; b < n_buckets; b += kPartBlock) hist[b] = 0;
  __syncthreads();
  uint64_t I0, I1;
  const bool ok = seg_range(he_off, m0, m1, limit, span_cap, &I0, &I1);
  if (!ok && blockIdx.x == 0 && threadIdx.x == 0) atomicOr(flags, I0 > I1 ? kErrOffsets : kErrCapacity);
  if (ok) {
    const uint64_t stride = uint64_t(kPartGrid) * kPartBlock;
    for (uint64_t s = m0 + blockIdx.x * uint64_t(kPartBlock) + threadIdx.x; s < m1; s += stride) {
      const uint64_t b = he_off[s], e = he_off[s + 1];
      if (b > e) {
        atomicOr(flags, kErrOffsets);
        continue;
      }
      const uint64_t lo = b < I0 ? I0 : b, hi = e < I1 ? e : I1;
      for (uint64_t x = lo; x < hi; ++x) {
        const uint32_t u = he_nodes[x];
        if (u >= n) {
          atomicOr(flags, kErrNodeRange);
          continue;
        }
        atomicAdd(&hist[u >> kBucketLog], 1u);
      }
    }
  }
  __syncthreads();
  for (uint32_t b = threadIdx.x; b < n_buckets; b += kPartBlock) cnt[size_t(b) * kPartGrid + blockIdx.x] = hist[b];
}

// Pass 2: the same samples in the same order; entry (u, s) goes to
// tmp[pos[bucket(u) * kPartGrid + blk] + its rank] (rank by LDS cursor),
// packed as u << 32 | s.  Writes stay below tmp_cap.
__global__ __launch_bounds__(kPartBlock) void k_inc_partition(const uint64_t* he_off, const uint32_t* he_nodes,
                                                              uint64_t m0, uint64_t m1, uint32_t n, uint64_t limit,
                                                              uint64_t span_cap, uint32_t n_buckets,
                                                              const uint64_t* pos, uint64_t* tmp, uint64_t tmp_cap,
                                                              uint32_t* flags) {
  extern __shared__ unsigned long long cursor[];
  for (uint32_t b = threadIdx.x; b < n_buckets; b += kPartBlock) cursor[b] = pos[size_t(b) * kPartGrid + blockIdx.x];
  __syncthreads();
  uint64_t I0, I1;
  if (!seg_range(he_off, m0, m1, limit, span_cap, &I0, &I1)) return;   // uniform
  const uint64_t stride = uint64_t(kPartGrid) * kPartBlock;
  for (uint64_t s = m0 + blockIdx.x * uint64_t(kPartBlock) + threadIdx.x; s < m1; s += stride) {
    const uint64_t b = he_off[s], e = he_off[s + 1];
    if (b > e) continue;
    const uint64_t lo = b < I0 ? I0 : b, hi = e < I1 ? e : I1;
    for (uint64_t x = lo; x < hi; ++x) {
      const uint32_t u = he_nodes[x];
      if (u >= n) continue;
      const uint64_t p = atomicAdd(&cursor[u >> kBucketLog], 1ull);
      if (p < tmp_cap)
        tmp[p] = (uint64_t(u) << 32) | static_cast<uint32_t>(s);
      else
        atomicOr(flags, kErrOffsets);
    }
  }
}

// Items of each bucket: nitems[b] = ceil(entries of bucket b / kItem).
__global__ void k_inc_items(const uint64_t* pos, uint32_t n_buckets, uint32_t* nitems) {
  const uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= n_buckets) return;
  const uint64_t sz = pos[size_t(b + 1) * kPartGrid] - pos[size_t(b) * kPartGrid];
  nitems[b] = static_cast<uint32_t>((sz + kItem - 1) / kItem);
}

// Item q: its bucket (the last b with item_off[b] <= q) and entry range.
__device__ __forceinline__ void item_range(const uint64_t* item_off, uint32_t n_buckets, const uint64_t* pos,
                                           uint64_t q, uint32_t* bucket, uint64_t* e0, uint64_t* e1) {
  uint32_t lo = 0, hi = n_buckets - 1;
  while (lo < hi) {
    const uint32_t mid = (lo + hi + 1) >> 1;
    if (item_off[mid] <= q)
      lo = mid;
    else
      hi = mid - 1;
  }
  const uint64_t bs = pos[size_t(lo) * kPartGrid], be = pos[size_t(lo + 1) * kPartGrid];
  *bucket = lo;
  *e0 = bs + (q - item_off[lo]) * kItem;
  *e1 = *e0 + kItem < be ? *e0 + kItem : be;
}

// Passes 3 (PLACE = false) and 4 (PLACE = true) over the items, grid
// strided.  cnt[] counts the item's entries per node of its bucket (a
// node's slot is its id within the bucket).  Pass 3 adds each present
// node's count to sdeg (one global add per node per item); pass 4 reserves
// the node's share of its row with one add on cur, then places every entry
// at that base plus its rank among the node's entries of the item.
template <bool PLACE>
__global__ __launch_bounds__(kItemBlock) void k_inc_items_pass(const uint64_t* tmp, const uint64_t* pos,
                                                               const uint64_t* item_off, uint32_t n_buckets,
                                                               uint32_t* sdeg, uint64_t* cur, uint32_t* inc,
                                                               uint32_t* inc_node, uint64_t limit, uint32_t* flags) {
  __shared__ uint32_t cnt[kBucketNodes];
  __shared__ unsigned long long base[PLACE ? kBucketNodes : 1];
  const uint64_t items = item_off[n_buckets];
  for (uint64_t q = blockIdx.x; q < items; q += gridDim.x) {
    uint32_t bucket;
    uint64_t e0, e1;
    item_range(item_off, n_buckets, pos, q, &bucket, &e0, &e1);
    const uint32_t node0 = bucket << kBucketLog;
    for (uint32_t i = threadIdx.x; i < kBucketNodes; i += kItemBlock) cnt[i] = 0;
    __syncthreads();
    for (uint64_t e = e0 + threadIdx.x; e < e1; e += kItemBlock)
      atomicAdd(&cnt[static_cast<uint32_t>(tmp[e] >> 32) & (kBucketNodes - 1)], 1u);
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < kBucketNodes; i += kItemBlock) {
      const uint32_t c = cnt[i];
      if (!c) continue;
      if constexpr (PLACE) {
        base[i] = atomicAdd(reinterpret_cast<unsigned long long*>(&cur[node0 + i]), static_cast<unsigned long long>(c));
        cnt[i] = 0;   // now the rank counter
      } else {
        atomicAdd(&sdeg[node0 + i], c);
      }
    }
    if constexpr (PLACE) {
      __syncthreads();
      for (uint64_t e = e0 + threadIdx.x; e < e1; e += kItemBlock) {
        const uint64_t x = tmp[e];
        const uint32_t u = static_cast<uint32_t>(x >> 32);
        const uint32_t slot = u & (kBucketNodes - 1);
        const uint64_t p = base[slot] + atomicAdd(&cnt[slot], 1u);
        if (p < limit) {
          inc[p] = static_cast<uint32_t>(x);
          inc_node[p] = u;
        } else {
          atomicOr(flags, kErrOffsets);
        }
      }
    }
    __syncthreads();   // cnt and base are reused by the next item
  }
}

// a[i] += *add (the addend read on the device)
__global__ void k_inc_offset(uint64_t* a, uint64_t n, const uint64_t* add) {
  const uint64_t x = *add;
  if (x == 0) return;
  for (uint64_t i = blockIdx.x * uint64_t(blockDim.x) + threadIdx.x; i < n; i += uint64_t(gridDim.x) * blockDim.x)
    a[i] += x;
}

__global__ void k_inc_copy(const uint64_t* src, uint64_t* dst, uint64_t n) {
  for (uint64_t i = blockIdx.x * uint64_t(blockDim.x) + threadIdx.x; i < n; i += uint64_t(gridDim.x) * blockDim.x)
    dst[i] = src[i];
}

__global__ void k_inc_add(const uint32_t* a, uint32_t n, uint32_t* acc) {
  for (uint32_t u = blockIdx.x * blockDim.x + threadIdx.x; u < n; u += gridDim.x * blockDim.x) acc[u] += a[u];
}

uint32_t buckets_of(uint32_t n) { return (n + kBucketNodes - 1) / kBucketNodes; }

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Workspace layout: cnt u32[B * G] | pos u64[B * G + 1] | nitems u32[B] |
// item_off u64[B + 1] | scan tiles | tmp u64[span_cap]
struct IncWs {
  uint32_t* cnt;
  uint64_t* pos;
  uint32_t* nitems;
  uint64_t* item_off;
  uint64_t* tiles;
  uint64_t* tmp;
};

IncWs carve(void* ws, uint32_t n, uint64_t span_cap, size_t* total) {
  const size_t B = buckets_of(n), BG = B * kPartGrid;
  const size_t tile_n = scan_tile_words(BG > n ? BG : n);
  // addresses are formed as integers: ws is NULL when only the size is asked for
  const uintptr_t p = reinterpret_cast<uintptr_t>(ws);
  size_t o = 0;
  IncWs w{};
  w.cnt = reinterpret_cast<uint32_t*>(p + o);
  o += align256(BG * 4);
  w.pos = reinterpret_cast<uint64_t*>(p + o);
  o += align256((BG + 1) * 8);
  w.nitems = reinterpret_cast<uint32_t*>(p + o);
  o += align256(B * 4);
  w.item_off = reinterpret_cast<uint64_t*>(p + o);
  o += align256((B + 1) * 8);
  w.tiles = reinterpret_cast<uint64_t*>(p + o);
  o += align256(tile_n * 8);
  w.tmp = reinterpret_cast<uint64_t*>(p + o);
  o += align256((span_cap ? span_cap : 1) * 8);
  *total = o;
  return w;
}

}  // namespace

size_t incidence_ws_bytes(uint32_t n, uint64_t span_cap) {
  size_t total = 0;
  (void)carve(nullptr, n, span_cap, &total);
  return total;
}

void incidence_segment_bucketed(uint32_t n, uint64_t m0, uint64_t m1, uint64_t span_cap, uint64_t limit,
                                const uint64_t* he_off, const uint32_t* he_nodes, bool first_segment, uint32_t* deg,
                                uint32_t* sdeg, uint64_t* off, uint64_t* cur, uint32_t* inc, uint32_t* inc_node,
                                void* ws, uint32_t* flags, hipStream_t s) {
  size_t total = 0;
  const IncWs w = carve(ws, n, span_cap, &total);
  const uint32_t B = buckets_of(n);
  if (first_segment) fill_u32(deg, 0, n, s);
  fill_u32(sdeg, 0, n, s);
  const bool any = m1 > m0 && span_cap;
  if (any) {
    hipLaunchKernelGGL(k_inc_bucket_count, dim3(kPartGrid), dim3(kPartBlock), size_t(B) * 4, s, he_off, he_nodes, m0,
                       m1, n, limit, span_cap, B, w.cnt, flags);
    excl_scan_u32_to_u64_ws(w.cnt, w.pos, size_t(B) * kPartGrid, w.tiles, s);
    hipLaunchKernelGGL(k_inc_partition, dim3(kPartGrid), dim3(kPartBlock), size_t(B) * 8, s, he_off, he_nodes, m0, m1,
                       n, limit, span_cap, B, static_cast<const uint64_t*>(w.pos), w.tmp, span_cap, flags);
    hipLaunchKernelGGL(k_inc_items, dim3(grid_of(B, 256)), dim3(256), 0, s, static_cast<const uint64_t*>(w.pos), B,
                       w.nitems);
    excl_scan_u32_to_u64_ws(w.nitems, w.item_off, B, w.tiles, s);
    hipLaunchKernelGGL(k_inc_items_pass<false>, dim3(kItemGrid), dim3(kItemBlock), 0, s,
                       static_cast<const uint64_t*>(w.tmp), static_cast<const uint64_t*>(w.pos),
                       static_cast<const uint64_t*>(w.item_off), B, sdeg, static_cast<uint64_t*>(nullptr),
                       static_cast<uint32_t*>(nullptr), static_cast<uint32_t*>(nullptr), limit, flags);
  }
  excl_scan_u32_to_u64_ws(sdeg, off, n, w.tiles, s);
  if (m0)
    hipLaunchKernelGGL(k_inc_offset, dim3(grid_of(uint64_t(n) + 1, 256)), dim3(256), 0, s, off, uint64_t(n) + 1,
                       he_off + m0);
  hipLaunchKernelGGL(k_inc_copy, dim3(grid_of(n, 256)), dim3(256), 0, s, static_cast<const uint64_t*>(off), cur,
                     uint64_t(n));
  if (any)
    hipLaunchKernelGGL(k_inc_items_pass<true>, dim3(kItemGrid), dim3(kItemBlock), 0, s,
                       static_cast<const uint64_t*>(w.tmp), static_cast<const uint64_t*>(w.pos),
                       static_cast<const uint64_t*>(w.item_off), B, static_cast<uint32_t*>(nullptr), cur, inc,
                       inc_node, limit, flags);
  hipLaunchKernelGGL(k_inc_add, dim3(grid_of(n, 256)), dim3(256), 0, s, static_cast<const uint32_t*>(sdeg), n, deg);
}

}  // namespace centra
