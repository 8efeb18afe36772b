// Device-side building blocks shared by the CentRA kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace centra {

constexpr uint32_t kUnseen = 0xFFFFFFFFu;
constexpr int kWave = 64;

// Error bits raised by kernels into the context's device flag word.
constexpr uint32_t kErrNodeRange = 1u;      // a hyperedge names a node >= n
constexpr uint32_t kErrBacktrack = 2u;      // no predecessor found (impossible on valid input)
constexpr uint32_t kErrGraph = 4u;          // malformed CSR
constexpr uint32_t kErrCapacity = 8u;       // a hyperedge store exceeds its stated capacity
constexpr uint32_t kErrOffsets = 16u;       // hyperedge offsets decrease

// ---------------------------------------------------------------------------
// Coherent accesses.  The per-BFS arrays are updated with device-scope
// atomics (performed in L2) by several waves at once; plain loads could be
// served from a stale line of the CU's vector L1, so every access to them
// goes through relaxed agent-scope atomic loads and stores.
__device__ __forceinline__ uint32_t ld_u32(const uint32_t* p) {
  return __hip_atomic_load(const_cast<uint32_t*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t ld_u64(const uint64_t* p) {
  return __hip_atomic_load(const_cast<uint64_t*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_u32(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_u64(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds, each two
// 64x64->128 products with the published multipliers; the key advances by
// the published Weyl constants after every round.
struct Block4 {
  uint64_t w0, w1, w2, w3;
};

__device__ __forceinline__ Block4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                               uint64_t k0, uint64_t k1) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t hi0 = __umul64hi(M0, c0), lo0 = M0 * c0;
    const uint64_t hi1 = __umul64hi(M1, c2), lo1 = M1 * c2;
    const uint64_t n0 = hi1 ^ c1 ^ k0;
    const uint64_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    k0 += W0;
    k1 += W1;
  }
  return Block4{c0, c1, c2, c3};
}

// Word stream with key (seed, 0) and counter (block, c1, c2, c3): blocks
// 0, 1, 2, ... consumed four words at a time.  Kept in registers; the
// selection avoids dynamic indexing (which would spill to scratch).
struct WordStream {
  uint64_t seed, c1, c2, c3;
  uint64_t next_block;
  uint32_t pos;
  Block4 buf;

  __device__ __forceinline__ WordStream(uint64_t seed_, uint64_t c1_, uint64_t c2_, uint64_t c3_)
      : seed(seed_), c1(c1_), c2(c2_), c3(c3_), next_block(0), pos(4), buf{0, 0, 0, 0} {}

  __device__ __forceinline__ uint64_t next() {
    if (pos == 4) {
      buf = philox4x64_10(next_block, c1, c2, c3, seed, 0);
      ++next_block;
      pos = 0;
    }
    const uint32_t p = pos++;
    return p == 0 ? buf.w0 : (p == 1 ? buf.w1 : (p == 2 ? buf.w2 : buf.w3));
  }
};

// Lemire's bounded draw in [0, W) (TOMACS 2019): high half of x*W, with the
// low half rejected below (2^64 - W) mod W.  W >= 1.
__device__ __forceinline__ uint64_t bounded(WordStream& st, uint64_t W) {
  uint64_t x = st.next();
  uint64_t lo = x * W;
  uint64_t hi = __umul64hi(x, W);
  if (lo < W) {
    const uint64_t thr = (0ull - W) % W;
    while (lo < thr) {
      x = st.next();
      lo = x * W;
      hi = __umul64hi(x, W);
    }
  }
  return hi;
}

// ---------------------------------------------------------------------------
// Wave (64-lane) helpers.
__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }

__device__ __forceinline__ uint64_t shfl_u64(uint64_t v, int src) {
  const uint32_t lo = __shfl(static_cast<uint32_t>(v), src, kWave);
  const uint32_t hi = __shfl(static_cast<uint32_t>(v >> 32), src, kWave);
  return (static_cast<uint64_t>(hi) << 32) | lo;
}
__device__ __forceinline__ uint64_t shfl_up_u64(uint64_t v, int d) {
  const uint32_t lo = __shfl_up(static_cast<uint32_t>(v), d, kWave);
  const uint32_t hi = __shfl_up(static_cast<uint32_t>(v >> 32), d, kWave);
  return (static_cast<uint64_t>(hi) << 32) | lo;
}
__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t v, int m) {
  const uint32_t lo = __shfl_xor(static_cast<uint32_t>(v), m, kWave);
  const uint32_t hi = __shfl_xor(static_cast<uint32_t>(v >> 32), m, kWave);
  return (static_cast<uint64_t>(hi) << 32) | lo;
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += shfl_xor_u64(v, m);
  return v;
}
__device__ __forceinline__ uint64_t wave_max_u64(uint64_t v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    const uint64_t o = shfl_xor_u64(v, m);
    v = o > v ? o : v;
  }
  return v;
}
// Workgroup-uniform values read from LDS or reduced across the block: the
// readfirstlane tells the compiler so, which keeps them (and what is derived
// from them) in scalar registers.  Only for values every lane holds equal.
__device__ __forceinline__ uint32_t uniform_u32(uint32_t x) {
  return static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(static_cast<int>(x)));
}
__device__ __forceinline__ uint64_t uniform_u64(uint64_t x) {
  return (uint64_t(uniform_u32(static_cast<uint32_t>(x >> 32))) << 32) | uniform_u32(static_cast<uint32_t>(x));
}

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, kWave);
  return v;
}
// Inclusive prefix sum over the 64 lanes.
__device__ __forceinline__ uint64_t wave_incl_scan_u64(uint64_t v) {
  const int lane = lane_id();
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const uint64_t o = shfl_up_u64(v, d);
    if (lane >= d) v += o;
  }
  return v;
}
__device__ __forceinline__ uint32_t wave_incl_scan_u32(uint32_t v) {
  const int lane = lane_id();
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const uint32_t o = __shfl_up(v, d, kWave);
    if (lane >= d) v += o;
  }
  return v;
}

// Block-wide exclusive scan of one u32 per thread; *total gets the sum.
// `scratch` holds BLOCK/64 + 1 words of LDS.  Contains barriers.
template <int BLOCK>
__device__ __forceinline__ uint32_t block_excl_scan_u32(uint32_t v, uint32_t* total, uint32_t* scratch) {
  constexpr int NW = BLOCK / kWave;
  const int lane = lane_id(), wid = threadIdx.x / kWave;
  const uint32_t incl = wave_incl_scan_u32(v);
  if (lane == kWave - 1) scratch[wid] = incl;
  __syncthreads();
  if (wid == 0) {
    uint32_t x = lane < NW ? scratch[lane] : 0u;
    const uint32_t xi = wave_incl_scan_u32(x);
    if (lane < NW) scratch[lane] = xi - x;   // exclusive wave offsets
    if (lane == NW - 1) scratch[NW] = xi;
  }
  __syncthreads();
  const uint32_t r = scratch[wid] + incl - v;
  *total = uniform_u32(scratch[NW]);
  __syncthreads();
  return r;
}

template <int BLOCK>
__device__ __forceinline__ uint64_t block_max_u64(uint64_t v, uint64_t* scratch) {
  constexpr int NW = BLOCK / kWave;
  const int lane = lane_id(), wid = threadIdx.x / kWave;
  v = wave_max_u64(v);
  if (lane == 0) scratch[wid] = v;
  __syncthreads();
  uint64_t r = 0;
#pragma unroll
  for (int i = 0; i < NW; ++i) r = scratch[i] > r ? scratch[i] : r;
  __syncthreads();
  return uniform_u64(r);
}

template <int BLOCK>
__device__ __forceinline__ uint64_t block_sum_u64(uint64_t v, uint64_t* scratch) {
  constexpr int NW = BLOCK / kWave;
  const int lane = lane_id(), wid = threadIdx.x / kWave;
  v = wave_sum_u64(v);
  if (lane == 0) scratch[wid] = v;
  __syncthreads();
  uint64_t r = 0;
#pragma unroll
  for (int i = 0; i < NW; ++i) r += scratch[i];
  __syncthreads();
  return uniform_u64(r);
}

__device__ __forceinline__ uint32_t bitlen64(uint64_t x) { return x ? 64u - __clzll(x) : 0u; }
__device__ __forceinline__ uint32_t bitlen32(uint32_t x) { return x ? 32u - __clz(x) : 0u; }

}  // namespace centra
