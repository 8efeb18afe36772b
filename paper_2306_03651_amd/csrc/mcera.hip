// AMCERA ingredients on gfx950: Rademacher sign words, the per-node trial
// sums R[u][j] = sum_{s : u in h_s} sigma_js, the per-trial sums of the k
// largest positive R[.][j], the k largest deg_H(u) and max |h|.
//
// Signs.  Sample s gets Wt = ceil(t/64) words; word w holds trials
// 64w .. 64w+63 and is word (w mod 4) of Philox block (w div 4, s,
// instance, 1), so bit (j mod 64) of word j div 64 is sigma_js.
//
// Trial sums.  R[u][j] = 2 P[u][j] - deg_H(u) with P[u][j] the number of
// samples of u's incidence row whose bit j is set.  A wave walks a span of
// the incidence (grouped by node); for each run of entries of one node
// inside a 64-entry batch it forms, for every trial bit j, the ballot of
// the lanes whose sign word has bit j set and adds its popcount to lane j's
// counter.  A node's counters are flushed with one coalesced row of atomic
// adds when the walk leaves the node (spans may split a node, hence the
// atomics; integer sums keep the result exact and order independent).
//
// Top-k.  For every trial row (plus one row of degrees) the k-th largest
// positive value is found by MSD radix selection: a histogram over the bit
// length, then 10-bit digit histograms below the leading bit, each with
// per-bin counts and sums; the answer is the sum of every value above the
// selected one plus the remaining copies of it.  Each pass splits every row
// over many workgroups, which build LDS histograms and merge them into the
// row's global histogram with atomics (a row on one workgroup would leave
// most CUs idle and serialise on a few LDS bins); a one-wave kernel per row
// then picks the digit with a wave scan and clears the histogram.
#include <vector>

#include "common.hpp"
#include "internal.hpp"

namespace centra {

__global__ void k_rade_words(uint64_t seed, uint32_t instance, uint64_t s0, uint64_t s1, uint32_t Wt,
                             uint64_t* words) {
  const uint32_t nblk = (Wt + 3) / 4;
  const uint64_t total = (s1 - s0) * nblk;
  for (uint64_t x = blockIdx.x * uint64_t(blockDim.x) + threadIdx.x; x < total;
       x += uint64_t(gridDim.x) * blockDim.x) {
    const uint64_t s = s0 + x / nblk;
    const uint32_t b = static_cast<uint32_t>(x % nblk);
    const Block4 r = philox4x64_10(b, s, instance, 1, seed, 0);
    uint64_t* dst = words + s * Wt + 4ull * b;
    const uint32_t avail = Wt - 4 * b;
    dst[0] = r.w0;
    if (avail > 1) dst[1] = r.w1;
    if (avail > 2) dst[2] = r.w2;
    if (avail > 3) dst[3] = r.w3;
  }
}

static unsigned grid_for(uint64_t n, unsigned block, unsigned cap = 16384) {
  uint64_t g = (n + block - 1) / block;
  if (g > cap) g = cap;
  return g ? static_cast<unsigned>(g) : 1u;
}

int rade_words(centra_ctx* ctx, uint64_t seed, uint32_t instance, uint64_t s0, uint64_t s1, uint32_t t,
               hipStream_t s) {
  const uint32_t Wt = (t + 63) / 64;
  ctx->mc_ok = false;   // the extend calls' AMCERA state is valid only after their own updates
  ++ctx->words_gen;
  int rc = ensure(ctx, ctx->words, size_t(s1) * Wt * 8, true, s);
  if (rc) return rc;
  if (s1 > s0)
    hipLaunchKernelGGL(k_rade_words, dim3(grid_for((s1 - s0) * ((Wt + 3) / 4), 256)), dim3(256), 0, s, seed,
                       instance, s0, s1, Wt, static_cast<uint64_t*>(ctx->words.ptr));
  CENTRA_HIP(ctx, hipGetLastError());
  return CENTRA_OK;
}

// ---------------------------------------------------------------------------
constexpr int kCountBlock = 256;
constexpr uint32_t kSpan = 64 * 16;   // incidence entries per wave

// P[u][j] += number of samples in u's incidence row whose sign bit j is set,
// for the trials 64g .. 64g+63 of word group g = blockIdx.y.  Each wave
// takes kSpan consecutive incidence entries (a node's entries are
// consecutive) and walks them one at a time: the entry's node and sign word
// are read into scalar registers (readlane) and lane j adds bit j of the
// word to its running count, flushed with one atomic per (node, lane) when
// the node changes.  The cost per entry is a few instructions whatever the
// row lengths; loads are 64 entries per step, coalesced for the incidence,
// one 8-byte gather per entry for the word.
__global__ __launch_bounds__(kCountBlock) void k_rade_count(const uint32_t* inc, const uint32_t* inc_node,
                                                            const uint64_t* he_off, uint64_t m0, uint64_t m1,
                                                            uint64_t limit, const uint64_t* words, uint32_t Wt,
                                                            uint32_t t, int32_t* P) {
  const int lane = lane_id();
  const uint32_t g = blockIdx.y;
  // the segment's entries [he_off[m0], he_off[m1]) of inc, read on the device
  const uint64_t I0 = he_off[m0], I = he_off[m1];
  if (I > limit || I0 > I) return;   // beyond the incidence (the build raised the error)
  const uint64_t wave = (blockIdx.x * uint64_t(kCountBlock) + threadIdx.x) / kWave;
  const uint64_t e0 = I0 + wave * kSpan;
  if (e0 >= I) return;
  const uint64_t e1 = e0 + kSpan < I ? e0 + kSpan : I;
  const uint32_t jt = 64 * g + lane;   // this lane's trial
  const bool live = jt < t;
  const uint32_t shift = lane & 31;
  const bool high = lane >= 32;
  uint32_t cur = kUnseen;
  uint32_t acc = 0;
  for (uint64_t base = e0; base < e1; base += kWave) {
    const uint64_t e = base + lane;
    const bool valid = e < e1;
    const uint32_t u = valid ? inc_node[e] : kUnseen;
    const uint64_t word = valid ? words[uint64_t(inc[e]) * Wt + g] : 0ull;
    const uint32_t wlo = static_cast<uint32_t>(word), whi = static_cast<uint32_t>(word >> 32);
    const uint32_t cnt = e1 - base < kWave ? static_cast<uint32_t>(e1 - base) : kWave;
    for (uint32_t i = 0; i < cnt; ++i) {
      const uint32_t ui = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(u), static_cast<int>(i)));
      const uint32_t lo = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(wlo), static_cast<int>(i)));
      const uint32_t hi = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(whi), static_cast<int>(i)));
      if (ui != cur) {
        if (cur != kUnseen && live && acc) atomicAdd(&P[uint64_t(cur) * t + jt], static_cast<int32_t>(acc));
        cur = ui;
        acc = 0;
      }
      acc += ((high ? hi : lo) >> shift) & 1u;
    }
  }
  if (cur != kUnseen && live && acc) atomicAdd(&P[uint64_t(cur) * t + jt], static_cast<int32_t>(acc));
}

// R[j][u] = 2 P[u][j] - deg[u] (trial-major for the selection) and, if
// requested, R_out[u][j] (node-major).  64 x 64 tiles through LDS.
__global__ __launch_bounds__(256) void k_rade_finish(const int32_t* P, const uint32_t* deg, uint32_t n, uint32_t t,
                                                     int32_t* Rtm, int32_t* R_out) {
  __shared__ int32_t tile[64][65];
  const uint32_t u0 = blockIdx.x * 64, j0 = blockIdx.y * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;   // 64 x 4
  for (int r = ty; r < 64; r += 4) {
    const uint32_t u = u0 + r, j = j0 + tx;
    int32_t v = 0;
    if (u < n && j < t) {
      v = 2 * P[uint64_t(u) * t + j] - static_cast<int32_t>(deg[u]);
      if (R_out) R_out[uint64_t(u) * t + j] = v;
    }
    tile[r][tx] = v;
  }
  __syncthreads();
  for (int r = ty; r < 64; r += 4) {
    const uint32_t j = j0 + r, u = u0 + tx;
    if (u < n && j < t) Rtm[uint64_t(j) * n + u] = tile[tx][r];
  }
}

// ---------------------------------------------------------------------------
constexpr int kSelBlock = 256;
constexpr int kDigitBits = 10;
constexpr uint32_t kBins = 1u << kDigitBits;   // also holds the 32 bit-length bins
constexpr int kDigitPasses = (30 + kDigitBits - 1) / kDigitBits;   // bits below the leading one

// Selection state of one row: the values still sought have bit length blen
// and their top pbits bits equal prefix; need of them are still to be taken
// and acc holds the sum of the values already taken.
// When done, the row's k largest are its values above tau and `ties`
// copies of tau (tau = 0, ties = 0: all of its positive values, fewer than
// k).
struct SelState {
  uint32_t prefix, pbits, blen, need, done, ties;
  int64_t acc;
  uint32_t tau, pad;
};

__global__ void k_sel_init(SelState* st, const SelRow* rows, uint32_t n_rows, uint32_t* hcnt, uint64_t* hsum) {
  const uint64_t nb = uint64_t(n_rows) * kBins;
  for (uint64_t i = blockIdx.x * uint64_t(blockDim.x) + threadIdx.x; i < nb; i += uint64_t(gridDim.x) * blockDim.x) {
    hcnt[i] = 0;
    hsum[i] = 0;
    if (i < n_rows) {
      const uint32_t k = rows[i].k;
      st[i] = SelState{1, 1, 0, k, k == 0 ? 1u : 0u, 0, 0, 0, 0};
    }
  }
}

// Pass `first`: bit lengths (bins 1..31) of the positive values; else the
// next digit of the values matching the row's prefix.  Block (x, r) takes
// values [x chunk, (x+1) chunk) of row r, chunk = ceil(n_r / gridDim.x).
__global__ __launch_bounds__(kSelBlock) void k_sel_hist(const SelRow* rows, const SelState* st, int first,
                                                        uint32_t* hcnt, uint64_t* hsum) {
  __shared__ uint32_t cnt[kBins];
  __shared__ uint64_t sum[kBins];
  const uint32_t r = blockIdx.y;
  const SelState s = st[r];
  if (s.done) return;
  const SelRow d = rows[r];
  const uint64_t chunk = (uint64_t(d.n) + gridDim.x - 1) / gridDim.x;
  const uint64_t i0 = uint64_t(blockIdx.x) * chunk;
  if (i0 >= d.n) return;
  const uint32_t B = s.blen, up = B - s.pbits;
  const uint32_t nb = first ? 5u : (up < uint32_t(kDigitBits) ? up : uint32_t(kDigitBits));
  const uint32_t shift = first ? 0u : up - nb;
  const uint32_t nbins = first ? 32u : 1u << nb;
  for (uint32_t b = threadIdx.x; b < nbins; b += kSelBlock) {
    cnt[b] = 0;
    sum[b] = 0;
  }
  __syncthreads();
  const int32_t* row = d.vals;
  const uint64_t i1 = i0 + chunk < d.n ? i0 + chunk : d.n;
  for (uint64_t i = i0 + threadIdx.x; i < i1; i += kSelBlock) {
    const int32_t x = row[i];
    if (x <= 0) continue;
    const uint32_t ux = static_cast<uint32_t>(x);
    uint32_t bin;
    if (first) {
      bin = bitlen32(ux);
    } else {
      if ((ux >> up) != s.prefix) continue;
      bin = (ux >> shift) & (nbins - 1u);
    }
    atomicAdd(&cnt[bin], 1u);
    atomicAdd(reinterpret_cast<unsigned long long*>(&sum[bin]), static_cast<unsigned long long>(ux));
  }
  __syncthreads();
  for (uint32_t b = threadIdx.x; b < nbins; b += kSelBlock) {
    if (cnt[b]) {
      atomicAdd(&hcnt[uint64_t(r) * kBins + b], cnt[b]);
      atomicAdd(reinterpret_cast<unsigned long long*>(&hsum[uint64_t(r) * kBins + b]),
                static_cast<unsigned long long>(sum[b]));
    }
  }
}

// One wave per row: walking the bins from the top, the bin where the count
// reaches `need` is the next digit (or bit length); the bins above it are
// taken whole.  Clears the row's histogram for the next pass.
__global__ __launch_bounds__(kWave) void k_sel_decide(SelState* st, int first, uint32_t* hcnt, uint64_t* hsum) {
  const uint32_t r = blockIdx.x;
  const int lane = lane_id();
  SelState s = st[r];
  if (s.done) return;
  const uint32_t up = s.blen - s.pbits;
  const uint32_t nb = first ? 5u : (up < uint32_t(kDigitBits) ? up : uint32_t(kDigitBits));
  const uint32_t nbins = first ? 32u : 1u << nb;
  const uint32_t per = nbins > uint32_t(kWave) ? nbins / kWave : 1u;
  uint32_t* C = hcnt + uint64_t(r) * kBins;
  uint64_t* S = hsum + uint64_t(r) * kBins;
  // lane L owns bins [hi - per, hi) with hi = nbins - L per (top bins first)
  const bool owns = uint32_t(lane) * per < nbins;
  const uint32_t hi = owns ? nbins - uint32_t(lane) * per : 0u;
  uint32_t c = 0;
  uint64_t sm = 0;
  for (uint32_t b = hi; b > hi - (owns ? per : 0u); --b) {
    c += C[b - 1];
    sm += S[b - 1];
  }
  const uint32_t c_incl = wave_incl_scan_u32(c);
  const uint64_t s_incl = wave_incl_scan_u64(sm);
  const uint32_t c_excl = c_incl - c;
  const uint64_t f = __ballot(owns && c_excl < s.need && c_incl >= s.need);
  if (f == 0) {
    // fewer than `need` values left (only in the first pass: fewer than k
    // positive values): all of them are taken
    if (lane == kWave - 1) {
      s.acc += static_cast<int64_t>(s_incl);
      s.done = 1;
      s.tau = 0;
      s.ties = 0;
      st[r] = s;
    }
  } else if (lane == __ffsll(static_cast<unsigned long long>(f)) - 1) {
    uint32_t rem = s.need - c_excl;
    int64_t acc = s.acc + static_cast<int64_t>(s_incl - sm);
    uint32_t d = hi - 1;
    for (uint32_t b = hi; b > hi - per; --b) {
      d = b - 1;
      if (C[d] < rem) {
        rem -= C[d];
        acc += static_cast<int64_t>(S[d]);
      } else {
        break;
      }
    }
    if (first) {
      s.blen = d;
      s.prefix = 1;
      s.pbits = 1;
    } else {
      s.prefix = (s.prefix << nb) | d;
      s.pbits += nb;
    }
    s.need = rem;
    s.acc = acc;
    if (s.pbits >= s.blen) {   // every bit fixed: the remaining copies of prefix
      s.acc += static_cast<int64_t>(s.need) * static_cast<int64_t>(s.prefix);
      s.tau = s.prefix;
      s.ties = s.need;
      s.done = 1;
    }
    st[r] = s;
  }
  for (uint32_t b = lane; b < nbins; b += kWave) {
    C[b] = 0;
    S[b] = 0;
  }
}

// b_max = max(b_max, largest |h| of samples [0, m) of he_off): one atomic
// per workgroup (an atomic per wave on the one word serialised the kernel).
constexpr int kBmaxBlock = 256;
__global__ __launch_bounds__(kBmaxBlock) void k_bmax(const uint64_t* he_off, uint64_t m, uint32_t* b_max) {
  __shared__ uint32_t red[kBmaxBlock / kWave];
  uint32_t mx = 0;
  for (uint64_t s = blockIdx.x * uint64_t(kBmaxBlock) + threadIdx.x; s < m; s += uint64_t(gridDim.x) * kBmaxBlock) {
    const uint64_t len = he_off[s + 1] - he_off[s];
    mx = len > mx ? static_cast<uint32_t>(len) : mx;
  }
  for (int o = 32; o >= 1; o >>= 1) {
    const uint32_t x = __shfl_xor(mx, o, kWave);
    mx = x > mx ? x : mx;
  }
  if (lane_id() == 0) red[threadIdx.x / kWave] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t r = 0;
    for (int i = 0; i < kBmaxBlock / kWave; ++i) r = red[i] > r ? red[i] : r;
    if (r) atomicMax(b_max, r);
  }
}

__global__ void k_sel_out(const SelState* st, const SelRow* rows, uint32_t n_rows) {
  for (uint32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < n_rows; r += gridDim.x * blockDim.x)
    if (rows[r].out) *rows[r].out = st[r].acc;
}

size_t select_ws_bytes(uint32_t n_rows) { return size_t(n_rows) * (sizeof(SelState) + kBins * 12); }

// The sum of the k largest positive values of every row (rows[r].k, 0 if
// there are none; rows[r].out receives it): MSD radix selection, each pass
// spread over about 2,048 workgroups.
void select_topk_rows(const SelRow* rows, uint32_t n_rows, uint32_t max_n, void* ws, hipStream_t s) {
  SelState* st = static_cast<SelState*>(ws);
  uint64_t* hsum = reinterpret_cast<uint64_t*>(st + n_rows);
  uint32_t* hcnt = reinterpret_cast<uint32_t*>(hsum + size_t(n_rows) * kBins);
  // about 2,048 workgroups per histogram pass, at least 4,096 values each
  uint32_t parts = 2048 / n_rows ? 2048 / n_rows : 1u;
  const uint32_t max_parts = (max_n + 4095) / 4096 ? (max_n + 4095) / 4096 : 1u;
  if (parts > max_parts) parts = max_parts;
  hipLaunchKernelGGL(k_sel_init, dim3(grid_for(uint64_t(n_rows) * kBins, 256)), dim3(256), 0, s, st, rows, n_rows, hcnt,
                     hsum);
  for (int pass = 0; pass <= kDigitPasses; ++pass) {
    hipLaunchKernelGGL(k_sel_hist, dim3(parts, n_rows), dim3(kSelBlock), 0, s, rows, st, pass == 0 ? 1 : 0, hcnt, hsum);
    hipLaunchKernelGGL(k_sel_decide, dim3(n_rows), dim3(kWave), 0, s, st, pass == 0 ? 1 : 0, hcnt, hsum);
  }
  hipLaunchKernelGGL(k_sel_out, dim3(grid_for(n_rows, 256, 64)), dim3(256), 0, s, st, rows, n_rows);
}

// Top-k sums of every row for every k <= K at once: after the selection
// at K, the row's values above its threshold are gathered (at most K of
// them), sorted in LDS together with the threshold's copies, and
// prefix-summed: out[r * K + i] = the sum of the i + 1 largest positive
// values (flat once they run out).
constexpr uint32_t kPrefixMax = 2048;

__global__ __launch_bounds__(kSelBlock) void k_sel_gather(const SelRow* rows, const SelState* st, uint32_t K,
                                                          uint32_t* gcount, int32_t* buf) {
  const uint32_t r = blockIdx.y;
  const SelRow d = rows[r];
  const uint32_t tau = st[r].tau;
  const uint64_t chunk = (uint64_t(d.n) + gridDim.x - 1) / gridDim.x;
  const uint64_t i0 = uint64_t(blockIdx.x) * chunk;
  const uint64_t i1 = i0 + chunk < d.n ? i0 + chunk : d.n;
  for (uint64_t i = i0 + threadIdx.x; i < i1; i += kSelBlock) {
    const int32_t x = d.vals[i];
    if (x <= 0 || static_cast<uint32_t>(x) <= tau) continue;
    const uint32_t at = atomicAdd(&gcount[r], 1u);
    if (at < K) buf[size_t(r) * K + at] = x;
  }
}

__global__ __launch_bounds__(kSelBlock) void k_sel_prefix(const SelState* st, const uint32_t* gcount,
                                                          const int32_t* buf, uint32_t K, uint32_t Kpad,
                                                          int64_t* out) {
  __shared__ int32_t v[kPrefixMax];
  __shared__ int64_t wsum[kSelBlock / kWave];
  const uint32_t r = blockIdx.x;
  const SelState s = st[r];
  const uint32_t g = gcount[r] < K ? gcount[r] : K;
  for (uint32_t i = threadIdx.x; i < Kpad; i += kSelBlock) {
    int32_t x = 0;
    if (i < g)
      x = buf[size_t(r) * K + i];
    else if (i < g + s.ties && i < K)
      x = static_cast<int32_t>(s.tau);
    v[i] = x;
  }
  __syncthreads();
  // bitonic sort, descending
  for (uint32_t size = 2; size <= Kpad; size <<= 1) {
    for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
      for (uint32_t i = threadIdx.x; i < Kpad; i += kSelBlock) {
        const uint32_t j = i ^ stride;
        if (j > i) {
          const bool desc = (i & size) == 0;
          const int32_t a = v[i], b = v[j];
          if (desc ? a < b : a > b) {
            v[i] = b;
            v[j] = a;
          }
        }
      }
      __syncthreads();
    }
  }
  // prefix sums: each thread sums Kpad / kSelBlock consecutive entries
  const uint32_t per = Kpad / kSelBlock ? Kpad / kSelBlock : 1u;
  const uint32_t b0 = threadIdx.x * per;
  int64_t loc = 0;
  for (uint32_t i = b0; i < b0 + per && i < Kpad; ++i) loc += v[i];
  const int64_t incl = static_cast<int64_t>(wave_incl_scan_u64(static_cast<uint64_t>(loc)));
  if (lane_id() == kWave - 1) wsum[threadIdx.x / kWave] = incl;
  __syncthreads();
  int64_t run = incl - loc;
  for (uint32_t w = 0; w < threadIdx.x / kWave; ++w) run += wsum[w];
  for (uint32_t i = b0; i < b0 + per && i < Kpad; ++i) {
    run += v[i];
    if (i < K) out[size_t(r) * K + i] = run;
  }
}

size_t select_prefix_ws_bytes(uint32_t n_rows, uint32_t K) {
  return select_ws_bytes(n_rows) + size_t(n_rows) * 4 + size_t(n_rows) * K * 4 + 256;
}

void select_prefix_rows(const SelRow* rows, uint32_t n_rows, uint32_t max_n, uint32_t K, void* ws, int64_t* out,
                        hipStream_t s) {
  select_topk_rows(rows, n_rows, max_n, ws, s);
  const SelState* st = static_cast<const SelState*>(ws);
  uint32_t* gcount = reinterpret_cast<uint32_t*>(static_cast<char*>(ws) + select_ws_bytes(n_rows));
  int32_t* buf = reinterpret_cast<int32_t*>(gcount + n_rows);
  fill_u32(gcount, 0, n_rows, s);
  uint32_t parts = 2048 / n_rows ? 2048 / n_rows : 1u;
  const uint32_t max_parts = (max_n + 4095) / 4096 ? (max_n + 4095) / 4096 : 1u;
  if (parts > max_parts) parts = max_parts;
  hipLaunchKernelGGL(k_sel_gather, dim3(parts, n_rows), dim3(kSelBlock), 0, s, rows, st, K, gcount, buf);
  uint32_t Kpad = kSelBlock;
  while (Kpad < K) Kpad <<= 1;
  hipLaunchKernelGGL(k_sel_prefix, dim3(n_rows), dim3(kSelBlock), 0, s, st, static_cast<const uint32_t*>(gcount),
                     static_cast<const int32_t*>(buf), K, Kpad, out);
}

// Launch-only steps of the AMCERA for callers that own their buffers.
void rade_words_launch(uint64_t seed, uint32_t instance, uint64_t s0, uint64_t s1, uint32_t t, uint64_t* words,
                       hipStream_t s) {
  const uint32_t Wt = (t + 63) / 64;
  if (s1 > s0)
    hipLaunchKernelGGL(k_rade_words, dim3(grid_for((s1 - s0) * ((Wt + 3) / 4), 256)), dim3(256), 0, s, seed, instance,
                       s0, s1, Wt, words);
}

void rade_count_launch(const uint32_t* inc, const uint32_t* inc_node, const uint64_t* he_off, uint64_t m0, uint64_t m1,
                       uint64_t span_cap, uint64_t limit, const uint64_t* words, uint32_t t, int32_t* P, hipStream_t s) {
  const uint32_t Wt = (t + 63) / 64;
  if (m1 > m0 && span_cap) {
    const uint64_t waves = (span_cap + kSpan - 1) / kSpan;
    const uint64_t blocks = (waves * kWave + kCountBlock - 1) / kCountBlock;
    hipLaunchKernelGGL(k_rade_count, dim3(static_cast<unsigned>(blocks), Wt), dim3(kCountBlock), 0, s, inc, inc_node,
                       he_off, m0, m1, limit, words, Wt, t, P);
  }
}

void rade_finish_launch(const int32_t* P, const uint32_t* deg, uint32_t n, uint32_t t, int32_t* Rtm, hipStream_t s) {
  hipLaunchKernelGGL(k_rade_finish, dim3((n + 63) / 64, (t + 63) / 64), dim3(256), 0, s, P, deg, n, t, Rtm,
                     static_cast<int32_t*>(nullptr));
}

void bmax_launch(const uint64_t* he_off, uint64_t m0, uint64_t m1, uint32_t* b_max, hipStream_t s) {
  if (m1 > m0)
    hipLaunchKernelGGL(k_bmax, dim3(grid_for(m1 - m0, kBmaxBlock, 512)), dim3(kBmaxBlock), 0, s, he_off + m0, m1 - m0,
                       b_max);
}

int mcera_reserve(centra_ctx* ctx, uint32_t n, uint64_t m, uint32_t t, hipStream_t s) {
  const uint32_t Wt = (t + 63) / 64;
  int rc;
  if ((rc = ensure(ctx, ctx->words, size_t(m) * Wt * 8, true, s))) return rc;
  if ((rc = ensure(ctx, ctx->P, size_t(n) * t * 4, true, s))) return rc;
  if ((rc = ensure(ctx, ctx->Rtm, size_t(n) * t * 4, false, s))) return rc;
  if ((rc = ensure(ctx, ctx->topk_tmp, select_ws_bytes(t + 1), false, s))) return rc;
  if ((rc = ensure(ctx, ctx->sel_rows, size_t(t + 1) * sizeof(SelRow), false, s))) return rc;
  return ensure(ctx, ctx->ext_bmax, 256, true, s);
}

// The selection rows of the AMCERA: trial j's row of Rtm, then the degree
// row (built on the device, so that no host buffer has to outlive the call).
__global__ void k_mcera_rows(SelRow* rows, const int32_t* Rtm, const int32_t* deg, uint32_t n, uint32_t t, uint32_t k,
                             int64_t* topk_sum, int64_t* deg_topk) {
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j > t) return;
  rows[j] = j < t ? SelRow{Rtm + size_t(j) * n, n, k, topk_sum + j} : SelRow{deg, n, k, deg_topk};
}

int mcera_on_incidence(centra_ctx* ctx, uint32_t n, uint64_t m, uint64_t m0, const uint64_t* he_off, uint32_t t,
                       uint32_t k, int64_t* topk_sum, uint64_t* deg_topk, uint32_t* b_max, int32_t* R_out,
                       hipStream_t s) {
  // samples [m0, m) are counted: entries [he_off[m0], he_off[m]) of the
  // incidence, at most the newest segment's span when that is where m0 is
  const uint64_t span_cap = m0 == ctx->inc_m0 ? ctx->inc_span_cap : ctx->inc_limit;
  int rc;
  if ((rc = ensure(ctx, ctx->P, size_t(n) * t * 4, m0 > 0, s))) return rc;
  if ((rc = ensure(ctx, ctx->Rtm, size_t(n) * t * 4, false, s))) return rc;
  const uint32_t rows = t + 1;
  if ((rc = ensure(ctx, ctx->topk_tmp, select_ws_bytes(rows), false, s))) return rc;
  if ((rc = ensure(ctx, ctx->sel_rows, size_t(rows) * sizeof(SelRow), false, s))) return rc;
  int32_t* P = static_cast<int32_t*>(ctx->P.ptr);
  int32_t* Rtm = static_cast<int32_t*>(ctx->Rtm.ptr);
  if (m0 == 0) fill_u32(reinterpret_cast<uint32_t*>(P), 0, size_t(n) * t, s);
  rade_count_launch(static_cast<const uint32_t*>(ctx->inc.ptr), static_cast<const uint32_t*>(ctx->inc_node.ptr), he_off,
                    m0, m, span_cap, ctx->inc_limit, static_cast<const uint64_t*>(ctx->words.ptr), t, P, s);
  hipLaunchKernelGGL(k_rade_finish, dim3((n + 63) / 64, (t + 63) / 64), dim3(256), 0, s, P,
                     static_cast<const uint32_t*>(ctx->deg.ptr), n, t, Rtm, R_out);
  // selection over the t trial rows and the degree row
  SelRow* drows = static_cast<SelRow*>(ctx->sel_rows.ptr);
  hipLaunchKernelGGL(k_mcera_rows, dim3((rows + 255) / 256), dim3(256), 0, s, drows, Rtm,
                     static_cast<const int32_t*>(ctx->deg.ptr), n, t, k, topk_sum, reinterpret_cast<int64_t*>(deg_topk));
  select_topk_rows(drows, rows, n, ctx->topk_tmp.ptr, s);
  if (m0 == 0) fill_u32(b_max, 0, 1, s);
  if (m > m0)
    hipLaunchKernelGGL(k_bmax, dim3(grid_for(m - m0, kBmaxBlock, 512)), dim3(kBmaxBlock), 0, s, he_off + m0, m - m0,
                       b_max);
  CENTRA_HIP(ctx, hipGetLastError());
  return CENTRA_OK;
}

}  // namespace centra
