// Context memory management, fill kernels and the device exclusive scan.
#include <stdio.h>

#include "common.hpp"
#include "internal.hpp"

namespace centra {

int fail(centra_ctx* ctx, int code, const std::string& msg) {
  if (ctx) ctx->err = msg;
  return code;
}

int hip_fail(centra_ctx* ctx, hipError_t e, const char* what) {
  char buf[512];
  snprintf(buf, sizeof(buf), "HIP error %d (%s) in %s", static_cast<int>(e), hipGetErrorString(e), what);
  return fail(ctx, e == hipErrorOutOfMemory ? CENTRA_ENOMEM : CENTRA_EHIP, buf);
}

int ensure(centra_ctx* ctx, DevBuf& b, size_t bytes, bool keep, hipStream_t s) {
  if (bytes <= b.bytes) return CENTRA_OK;
  // grow geometrically so repeated small extensions stay cheap
  size_t want = bytes;
  if (keep && b.bytes) want = bytes > b.bytes + b.bytes / 2 ? bytes : b.bytes + b.bytes / 2;
  want = (want + 255) & ~size_t(255);
  if (ctx->budget && ctx->allocated - b.bytes + want > ctx->budget) {
    if (ctx->allocated - b.bytes + bytes > ctx->budget)
      return fail(ctx, CENTRA_ENOMEM, "HBM budget exceeded");
    want = bytes;
  }
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, want);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(ctx, CENTRA_ENOMEM, "device allocation failed");
  }
  if (keep && b.ptr && b.bytes) {
    e = hipMemcpyAsync(p, b.ptr, b.bytes, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
      (void)hipFree(p);
      return hip_fail(ctx, e, "ensure/copy");
    }
  }
  if (b.ptr) {
    if (!keep) (void)hipStreamSynchronize(s);
    (void)hipFree(b.ptr);
  }
  ctx->allocated = ctx->allocated - b.bytes + want;
  b.ptr = p;
  b.bytes = want;
  return CENTRA_OK;
}

void release(centra_ctx* ctx, DevBuf& b) {
  if (b.ptr) (void)hipFree(b.ptr);
  ctx->allocated -= b.bytes;
  b.ptr = nullptr;
  b.bytes = 0;
}

__global__ void k_fill_u32(uint32_t* p, uint32_t v, size_t n) {
  for (size_t i = blockIdx.x * size_t(blockDim.x) + threadIdx.x; i < n; i += size_t(gridDim.x) * blockDim.x)
    p[i] = v;
}
__global__ void k_fill_u64(uint64_t* p, uint64_t v, size_t n) {
  for (size_t i = blockIdx.x * size_t(blockDim.x) + threadIdx.x; i < n; i += size_t(gridDim.x) * blockDim.x)
    p[i] = v;
}

static unsigned grid_for(size_t n, unsigned block) {
  size_t g = (n + block - 1) / block;
  if (g > 65536) g = 65536;
  return g ? static_cast<unsigned>(g) : 1u;
}

void fill_u32(uint32_t* p, uint32_t v, size_t n, hipStream_t s) {
  if (n) hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(n, 256)), dim3(256), 0, s, p, v, n);
}
void fill_u64(uint64_t* p, uint64_t v, size_t n, hipStream_t s) {
  if (n) hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(n, 256)), dim3(256), 0, s, p, v, n);
}

// ---------------------------------------------------------------------------
// Exclusive scan u32 -> u64 in three passes: per-tile sums, a single-block
// scan of the tile sums (looping over chunks with a carry), and the tile
// pass that writes the offsets.
constexpr int kScanBlock = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanBlock * kScanItems;

__global__ __launch_bounds__(kScanBlock) void k_scan_tile_sums(const uint32_t* in, size_t n, uint64_t* tile_sums) {
  __shared__ uint64_t red[kScanBlock / kWave];
  const size_t base = blockIdx.x * size_t(kScanTile);
  uint64_t acc = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    const size_t idx = base + size_t(i) * kScanBlock + threadIdx.x;
    if (idx < n) acc += in[idx];
  }
  acc = block_sum_u64<kScanBlock>(acc, red);
  if (threadIdx.x == 0) tile_sums[blockIdx.x] = acc;
}

__global__ __launch_bounds__(kScanBlock) void k_scan_tile_prefix(uint64_t* tile_sums, size_t tiles) {
  __shared__ uint64_t wsum[kScanBlock / kWave + 1];
  uint64_t carry = 0;
  const int lane = lane_id(), wid = threadIdx.x / kWave;
  for (size_t b = 0; b < tiles; b += kScanBlock) {
    const size_t i = b + threadIdx.x;
    const uint64_t v = i < tiles ? tile_sums[i] : 0;
    const uint64_t incl = wave_incl_scan_u64(v);
    if (lane == kWave - 1) wsum[wid] = incl;
    __syncthreads();
    uint64_t off = 0, tot = 0;
    for (int w = 0; w < kScanBlock / kWave; ++w) {
      if (w < wid) off += wsum[w];
      tot += wsum[w];
    }
    if (i < tiles) tile_sums[i] = carry + off + incl - v;
    carry += tot;
    __syncthreads();
  }
  if (threadIdx.x == 0) tile_sums[tiles] = carry;
}

__global__ __launch_bounds__(kScanBlock) void k_scan_tile_write(const uint32_t* in, size_t n,
                                                                const uint64_t* tile_prefix, uint64_t* out) {
  __shared__ uint64_t wsum[kScanBlock / kWave];
  const int lane = lane_id(), wid = threadIdx.x / kWave;
  // each thread owns kScanItems consecutive elements
  const size_t base = blockIdx.x * size_t(kScanTile) + size_t(threadIdx.x) * kScanItems;
  uint32_t v[kScanItems];
  uint64_t local = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    v[i] = base + i < n ? in[base + i] : 0u;
    local += v[i];
  }
  const uint64_t incl = wave_incl_scan_u64(local);
  if (lane == kWave - 1) wsum[wid] = incl;
  __syncthreads();
  uint64_t off = tile_prefix[blockIdx.x];
  for (int w = 0; w < wid; ++w) off += wsum[w];
  uint64_t run = off + incl - local;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    if (base + i < n) out[base + i] = run;
    run += v[i];
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) out[n] = tile_prefix[gridDim.x];
}

size_t scan_tile_words(size_t n) { return (n + kScanTile - 1) / kScanTile + 1; }

void excl_scan_u32_to_u64_ws(const uint32_t* in, uint64_t* out, size_t n, uint64_t* tile_sums, hipStream_t s) {
  if (n == 0) {
    fill_u64(out, 0, 1, s);
    return;
  }
  const size_t tiles = (n + kScanTile - 1) / kScanTile;
  hipLaunchKernelGGL(k_scan_tile_sums, dim3(tiles), dim3(kScanBlock), 0, s, in, n, tile_sums);
  hipLaunchKernelGGL(k_scan_tile_prefix, dim3(1), dim3(kScanBlock), 0, s, tile_sums, tiles);
  hipLaunchKernelGGL(k_scan_tile_write, dim3(tiles), dim3(kScanBlock), 0, s, in, n, tile_sums, out);
}

int excl_scan_u32_to_u64(centra_ctx* ctx, const uint32_t* in, uint64_t* out, size_t n, hipStream_t s) {
  int rc = ensure(ctx, ctx->scan_tmp, scan_tile_words(n) * sizeof(uint64_t), false, s);
  if (rc) return rc;
  excl_scan_u32_to_u64_ws(in, out, n, static_cast<uint64_t*>(ctx->scan_tmp.ptr), s);
  CENTRA_HIP(ctx, hipGetLastError());
  return CENTRA_OK;
}

int check_flags(centra_ctx* ctx, hipStream_t s, const char* where) {
  uint32_t f = 0;
  CENTRA_HIP(ctx, hipMemcpyAsync(&f, ctx->d_flags, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  CENTRA_HIP(ctx, hipStreamSynchronize(s));
  if (f) {
    fill_u32(ctx->d_flags, 0, 1, s);
    (void)hipStreamSynchronize(s);
    std::string msg = std::string(where) + ":";
    if (f & kErrNodeRange) msg += " hyperedge node id out of range;";
    if (f & kErrBacktrack) msg += " backtrack found no predecessor;";
    if (f & kErrGraph) msg += " malformed graph;";
    if (f & kErrCapacity) msg += " hyperedge store capacity exceeded;";
    if (f & kErrOffsets) msg += " hyperedge offsets decrease;";
    const int code = (f & kErrBacktrack) ? CENTRA_EHIP : (f & ~kErrCapacity) ? CENTRA_EINVAL : CENTRA_ENOSPC;
    return fail(ctx, code, msg);
  }
  return CENTRA_OK;
}

}  // namespace centra
