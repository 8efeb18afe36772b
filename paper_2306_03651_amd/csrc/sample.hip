// sampleHEs for set betweenness on gfx950.
//
// Each workgroup of a persistent grid owns one BFS slot and takes sample
// indices from an atomic work counter until the batch is exhausted.  One
// sample = pair draw, level-synchronous BFS from s with normalised path
// counts, backtrack of a uniform shortest path from t.  Every quantity the
// output depends on (levels, integer count sums, level maxima, the ordered
// scan of in-neighbours) is independent of thread timing, so the result is
// bit-identical to a sequential implementation.
//
// State of a slot, in HBM: one 16-byte record per node {sigma' u64, tag
// u64} (a node's claim, level, count reads and writes touch a single cache
// line), the visit queue (u32, nodes in level order) and the stored
// per-pair counts of the last 3-hop test.  The tag is stamp << 32 |
// (kUnseen - level), where the stamp numbers the BFSs of the context in
// launch and work order: a slot's records carry only stamps older than its
// current BFS's unless that BFS claimed them, so nothing is ever reset
// between samples (records start at stamp 0; the stamps restart after a
// full clear when 32 bits run out).  The visited set of the completed
// levels is an exact bitmap in LDS (the 1024-thread variant, n up to about
// 1.1M; cleared per visited node) or a Bloom filter in LDS backed by the
// tags (the default variants).
//
// Level expansion (push): the frontier is processed in chunks of BLOCK
// nodes; their out-degrees are prefix-summed in LDS and each thread takes
// UNROLL arcs per round (tid, tid + BLOCK, ...), locating their sources by
// binary search in LDS (load balance over skewed degrees; consecutive
// threads read consecutive col_idx entries; UNROLL independent chains keep
// more memory requests in flight).  An arc w -> v whose target is not in a
// completed level raises v's tag to (stamp, L+1) with a returning 64-bit
// atomic max: the one that sees an older stamp is the first arrival, claims
// v (appended to the queue with one LDS atomic per wave, ballot +
// popcount) and starts its count with its own contribution; after a
// barrier the other arrivals add theirs with returning 64-bit atomics
// (the inverted level keeps the max from touching nodes of lower levels).
// The returned partial sums also give the level's largest raw count, so
// the normalisation shift needs no extra pass; only when the shift is
// nonzero are the level's counts rewritten.
//
// Early stop.  After levels 0..L are complete, every visited in-neighbour
// of an unvisited node is at level L (a lower one would have put the node
// in a completed level).  Before expanding level L the workgroup tests, on
// rings of in-neighbours around t:
//   (1) t has a visited in-neighbour: d(s,t) = L+1;
//   (2) some pair (w in in(t), u in in(w)) has u visited: w is at L+1 and
//       d = L+2; the raw count of each such w is the sum of its visited
//       in-neighbours' counts;
//   (3) some u of those pairs (unvisited) has visited in-neighbours: u is
//       at L+1, its w at L+2 and d = L+3; the raw counts of u and w follow
//       the same way, and the per-pair counts of u are kept for the
//       backtrack.
// Levels L+1 (and L+2) are then never produced.  Their normalisation
// would be a no-op when every count of theirs is below 2^C: level L+1
// counts are at most S_L (the sum of the level-L counts) and level L+2
// counts at most S_L times the largest out-degree, so (2) is taken only if
// S_L < 2^C and (3) only if also S_L * max out-degree < 2^C; otherwise the
// levels are produced and normalised as usual.  Test (3) scans the in-rows
// of the ring's nodes (the cone), so it runs only when the cone is at most
// kConeRatio times the CSR entries that expanding level L would scan, and
// (2) only when its pairs are at most kPairRatio times those entries.  All
// routes give the same counts, hence the same hyperedge.
//
// Unreachable targets.  A t without in-neighbours skips the BFS; when the
// rings show that every ancestor of t is within backward distance 1 or 2,
// the BFS stops once the tests have ruled out those distances.
//
// Node ids.  The kernel traverses the graph's locality-relabelled copy
// (grouped so that nodes reached from one hub have nearby ids); the pair
// is drawn in caller ids and mapped in, and hyperedge nodes are mapped back.
// Rows keep the caller's order, so every scan order is the caller's.
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <type_traits>
#include <vector>

#include "common.hpp"
#include "internal.hpp"
#include "sample.hpp"

namespace centra {

// Ring limits: t with at most Ring<BLOCK>::kCache in-neighbours gets the
// 2-hop test on the pairs (w in in(t), u in in(w)); the 3-hop test also
// needs at most kPairMax pairs.  Cost rules (kConeRatio, kPairRatio) decide
// at which levels they run.
// Bloom filter of the visited set for the HBM variant (see BitsRec).
constexpr uint32_t kBloomLog = 14;
constexpr uint32_t kBloomWords = (1u << kBloomLog) / 32;

template <int BLOCK>
struct Ring {
  static constexpr uint32_t kCache = BLOCK >= 512 ? 512u : 256u;
};
constexpr uint64_t kConeRatio = 3;
// The 2-hop test runs at a level only when its pairs are at most kPairRatio
// times the out-arcs expanding that level would scan (a pair costs a
// sequential read and an LDS probe, an expanded arc a random atomic).
constexpr uint64_t kPairRatio = 4;

// Record accessors: word 0 = sigma', word 1 = tag.  With base = stamp << 32
// the tag of a node at level l of the current BFS is base + (kUnseen - l):
// "claimed by this BFS" is tag >= base, "at level <= L" is
// tag >= base + (kUnseen - L).
__device__ __forceinline__ uint64_t* sig_of(uint64_t* rec, uint32_t v) { return rec + 2 * size_t(v); }
__device__ __forceinline__ uint64_t* tag_of(uint64_t* rec, uint32_t v) { return rec + 2 * size_t(v) + 1; }
__device__ __forceinline__ uint64_t level_tag(uint64_t base, uint32_t level) { return base + (kUnseen - level); }

template <int BLOCK>
struct SampleShared {
  uint32_t off[BLOCK];
  uint32_t rs[BLOCK];
  uint64_t sg[BLOCK];
  uint32_t scan[BLOCK / kWave + 1];
  uint64_t red[BLOCK / kWave];
  uint32_t poff[Ring<BLOCK>::kCache];   // pair offsets of t's in-neighbours
  uint32_t rw[Ring<BLOCK>::kCache];     // t's in-neighbours w
  uint32_t rrs[Ring<BLOCK>::kCache];    // in_ptr[w]
  uint64_t ring_a[Ring<BLOCK>::kCache];  // per in-neighbour w of t: level-(L+1) count
  uint64_t ring_b[Ring<BLOCK>::kCache];  // per in-neighbour w of t: level-(L+2) count
  uint32_t bloom[BLOCK >= 1024 ? 1 : kBloomWords];   // HBM variant (<= 512 threads): visited filter
  uint64_t base;
  uint64_t hub_pairs;
  uint32_t hpos;
  uint32_t pick;
  uint32_t qlen;
  uint32_t next;
};

// Saturating u64 addition (only "below 2^C" is ever asked of these sums).
__device__ __forceinline__ uint64_t sat_add(uint64_t a, uint64_t b) {
  const uint64_t c = a + b;
  return c < a ? ~0ull : c;
}

template <int BLOCK>
__device__ __forceinline__ uint64_t block_sat_sum(uint64_t v, uint64_t* scratch) {
  constexpr int NW = BLOCK / kWave;
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v = sat_add(v, shfl_xor_u64(v, m));
  if (lane_id() == 0) scratch[threadIdx.x / kWave] = v;
  __syncthreads();
  uint64_t r = 0;
#pragma unroll
  for (int i = 0; i < NW; ++i) r = sat_add(r, scratch[i]);
  __syncthreads();
  return uniform_u64(r);
}

// Visited set.  Between levels, "visited" means "in a completed level"
// (levels 0..L), which is also "claimed by this BFS".  done(v, L) is that
// test; maybe(v) may answer true for an unvisited node but never false for
// a visited one; count(v) is sigma'_v for a visited v, else 0; set(v) adds
// v when its level closes.  base is the current BFS's stamp << 32.

// LDS variant: an exact bitmap of n bits in LDS.
struct BitsLds {
  uint32_t* w;
  uint64_t* rec;
  uint64_t base;
  __device__ __forceinline__ bool maybe(uint32_t v) const { return (w[v >> 5] >> (v & 31u)) & 1u; }
  __device__ __forceinline__ bool done(uint32_t v, uint32_t) const { return maybe(v); }
  __device__ __forceinline__ uint64_t count(uint32_t v) const { return maybe(v) ? ld_u64(sig_of(rec, v)) : 0ull; }
  __device__ __forceinline__ void set(uint32_t v) { atomicOr(&w[v >> 5], 1u << (v & 31u)); }
};

// HBM variant: no bitmap.  A one-hash Bloom filter of kBloomBits bits in
// LDS holds the nodes of the completed levels: a clear filter bit proves
// "not visited" without touching HBM (most tests: the visited set is small
// next to n); a set one defers to the node's tag.

__device__ __forceinline__ uint32_t bloom_bit(uint32_t v) { return (v * 0x9E3779B1u) >> (32 - kBloomLog); }

struct BitsRec {
  uint64_t* rec;
  uint32_t* bloom;   // LDS, kBloomWords
  uint64_t base;
  __device__ __forceinline__ bool maybe(uint32_t v) const {
    const uint32_t b = bloom_bit(v);
    return (bloom[b >> 5] >> (b & 31u)) & 1u;
  }
  __device__ __forceinline__ bool done(uint32_t v, uint32_t L) const {
    return maybe(v) && ld_u64(tag_of(rec, v)) >= level_tag(base, L);
  }
  __device__ __forceinline__ uint64_t count(uint32_t v) const {
    if (!maybe(v)) return 0;
    const uint64_t tg = ld_u64(tag_of(rec, v));   // both loads in flight together
    const uint64_t c = ld_u64(sig_of(rec, v));
    return tg >= base ? c : 0ull;
  }
  __device__ __forceinline__ void set(uint32_t v) {
    const uint32_t b = bloom_bit(v);
    atomicOr(&bloom[b >> 5], 1u << (b & 31u));
  }
};

template <bool LDS_BITS>
__device__ __forceinline__ typename std::conditional<LDS_BITS, BitsLds, BitsRec>::type make_bits(uint32_t* lds_bits,
                                                                                              uint64_t* rec,
                                                                                              uint32_t* bloom) {
  if constexpr (LDS_BITS) {
    (void)bloom;
    return BitsLds{lds_bits, rec, 0};
  } else {
    (void)lds_bits;
    return BitsRec{rec, bloom, 0};
  }
}

// Raw counts of one chunk of nodes, one node u per thread (kUnseen for
// none) with its in-row (start rs_u, length deg_u): sh.sg[tid] = sum of
// sigma' over u's visited in-neighbours, 0 for a visited u.  For an unvisited u every visited in-neighbour is at the last
// produced level (a lower one would have put u in a produced level), so
// this is u's raw count one level below.  Load balanced like the
// expansion: in-degrees prefix-summed in LDS, UNROLL entries per thread
// per round, sources found by binary search.  Adds the entries scanned to
// n_arcs.  Contains barriers; sh.sg is valid on return until the next call.
template <int BLOCK, int UNROLL, typename Bits>
__device__ void raw_counts_chunk(const SampleArgs& a, const Bits& bits, uint64_t* rec, uint32_t u, uint32_t rs_u,
                                 uint32_t deg_u, uint32_t L, SampleShared<BLOCK>& sh, uint64_t& n_arcs) {
  const int tid = threadIdx.x;
  uint32_t deg = 0, rs = 0;
  if (u != kUnseen && !bits.done(u, L)) {
    rs = rs_u;
    deg = deg_u;
  }
  uint32_t total;
  const uint32_t off = block_excl_scan_u32<BLOCK>(deg, &total, sh.scan);
  n_arcs += total;
  sh.off[tid] = off;
  sh.rs[tid] = rs;
  sh.sg[tid] = 0;
  __syncthreads();
  for (uint32_t base = 0; base < total; base += BLOCK * UNROLL) {
    uint32_t x[UNROLL], j[UNROLL];
#pragma unroll
    for (int k = 0; k < UNROLL; ++k) {
      const uint32_t e = base + k * BLOCK + tid;
      x[k] = kUnseen;
      j[k] = 0;
      if (e < total) {
        int lo = 0, hi = BLOCK - 1;
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (sh.off[mid] <= e)
            lo = mid;
          else
            hi = mid - 1;
        }
        j[k] = lo;
        x[k] = a.in_idx[sh.rs[lo] + (e - sh.off[lo])];
      }
    }
#pragma unroll
    for (int k = 0; k < UNROLL; ++k) {
      const uint64_t c = x[k] != kUnseen ? bits.count(x[k]) : 0ull;   // 0: unvisited
      if (c) atomicAdd(reinterpret_cast<unsigned long long*>(&sh.sg[j[k]]), static_cast<unsigned long long>(c));
    }
  }
  __syncthreads();
}

// Exclusive scan of one u64 per thread in thread order, with the total.
template <int BLOCK>
__device__ __forceinline__ uint64_t block_excl_scan_u64(uint64_t v, uint64_t* total, uint64_t* scratch) {
  constexpr int NW = BLOCK / kWave;
  const int wid = threadIdx.x / kWave;
  const uint64_t incl = wave_incl_scan_u64(v);
  if (lane_id() == kWave - 1) scratch[wid] = incl;
  __syncthreads();
  uint64_t before = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < NW; ++i) {
    const uint64_t x = scratch[i];
    before += i < wid ? x : 0ull;
    tot += x;
  }
  __syncthreads();
  *total = uniform_u64(tot);
  return before + incl - v;
}

// Weighted pick over entries j = 0 .. len-1 in ascending order, workgroup
// wide: W = sum of weight(j) (or W_known when nonzero, the caller's exact
// sum), r = bounded(st, W), and the result is the smallest j whose
// inclusive prefix sum exceeds r; kUnseen when W = 0.  Each thread holds
// kPickPer consecutive entries per round, so a round covers BLOCK *
// kPickPer entries with that many loads in flight; rows of at most one
// round are summed and searched from the same registers.  Uniform control
// flow; every thread draws the same words.
constexpr uint32_t kPickPer = 4;

template <int BLOCK, typename F>
__device__ uint32_t block_pick(uint32_t len, const F& weight, uint64_t W_known, WordStream& st,
                               SampleShared<BLOCK>& sh) {
  constexpr uint32_t kRound = BLOCK * kPickPer;
  const uint32_t first = threadIdx.x * kPickPer;
  uint64_t x[kPickPer];
  uint64_t W = W_known, run = 0, r = 0;
  if (len > kRound && !W) {
    for (uint32_t c = 0; c < len; c += kRound) {
      uint64_t ts = 0;
#pragma unroll
      for (uint32_t k = 0; k < kPickPer; ++k) ts += c + first + k < len ? weight(c + first + k) : 0ull;
      W += block_sum_u64<BLOCK>(ts, sh.red);
    }
    if (!W) return kUnseen;
  }
  if (W) r = bounded(st, W);
  for (uint32_t c = 0; c < len; c += kRound) {
    uint64_t ts = 0;
#pragma unroll
    for (uint32_t k = 0; k < kPickPer; ++k) {
      x[k] = c + first + k < len ? weight(c + first + k) : 0ull;
      ts += x[k];
    }
    uint64_t tot;
    uint64_t incl = run + block_excl_scan_u64<BLOCK>(ts, &tot, sh.red);
    if (!W) {   // single round, sum not known before: draw now
      W = tot;
      if (!W) return kUnseen;
      r = bounded(st, W);
    }
    if (run + tot > r) {
      uint32_t cand = kUnseen;
#pragma unroll
      for (uint32_t k = 0; k < kPickPer; ++k) {
        incl += x[k];
        if (cand == kUnseen && incl > r) cand = c + first + k;
      }
      return ~static_cast<uint32_t>(block_max_u64<BLOCK>(uint64_t(~cand), sh.red));   // uniform
    }
    run += tot;
  }
  return kUnseen;
}

// Backtrack weight of in-neighbour w of a node at level want + 1: sigma'_w
// if w is at level want of this BFS, else 0 (both loads issued together).
template <typename Bits>
__device__ __forceinline__ uint64_t pred_weight(const Bits& bits, uint64_t* rec, uint32_t w, uint32_t want) {
  if (!bits.maybe(w)) return 0;
  const uint64_t tg = ld_u64(tag_of(rec, w));
  const uint64_t c = ld_u64(sig_of(rec, w));
  return tg == level_tag(bits.base, want) ? c : 0ull;
}

__device__ __forceinline__ uint32_t caller_id(const SampleArgs& a, uint32_t v) { return a.orig_of ? a.orig_of[v] : v; }

// A BFS past its scan budget is handed over only on a level of at least
// this many nodes: the device-wide BFS pays a host round trip per level, so
// deep, narrow searches (long grids) stay on their workgroups.
constexpr uint32_t kWideMinWidth = 4096;

// Appends work item idx to the deferred list (workgroup uniform); true if
// it fit, the sample then being left to the device-wide BFS.
template <int BLOCK>
__device__ __forceinline__ bool defer_sample(const SampleArgs& a, uint32_t idx, SampleShared<BLOCK>& sh) {
  if (threadIdx.x == 0) {
    const uint32_t at = atomicAdd(a.defer_count, 1u);
    if (at < a.defer_cap) a.defer_list[at] = idx;
    sh.pick = at;
  }
  __syncthreads();
  const uint32_t at = uniform_u32(sh.pick);
  __syncthreads();
  return at < a.defer_cap;
}

// Cost rule of the hub 2-hop test at a level (queue entries [lb, le)):
// true when the in-rows of t's dt in-neighbours (starting at in_idx[tb])
// hold at most kPairRatio times the out-arcs of the level.  Both sums grow
// chunk by chunk only until the comparison is decided; the in-row sum and
// its position persist in sh across levels.  Uniform; contains barriers.
template <int BLOCK>
__device__ __forceinline__ bool hub_rule(const SampleArgs& g, const uint32_t* q, uint32_t tb, uint32_t dt, uint32_t lb,
                                      uint32_t le, SampleShared<BLOCK>& sh, uint64_t& n_arcs) {
  const uint32_t tid = threadIdx.x;
  uint32_t hpos = uniform_u32(sh.hpos);
  uint64_t hub = uniform_u64(sh.hub_pairs);
  uint32_t fpos = lb;
  uint64_t fpart = 0;
  bool run;
  for (;;) {
    const bool hdone = hpos >= dt, fdone = fpos >= le;
    if (hdone && hub <= kPairRatio * fpart) {
      run = true;
      break;
    }
    if (fdone && hub > kPairRatio * fpart) {
      run = false;
      break;
    }
    if (!hdone && (fdone || hub <= kPairRatio * fpart)) {
      const uint32_t e = hpos + tid;
      uint64_t c = 0;
      if (e < dt) {
        const uint32_t w = g.in_idx[tb + e];
        c = g.in_ptr[w + 1] - g.in_ptr[w];
      }
      hub += block_sum_u64<BLOCK>(c, sh.red);
      n_arcs += dt - hpos < uint32_t(BLOCK) ? dt - hpos : uint32_t(BLOCK);
      hpos += BLOCK;
    } else {
      const uint32_t i = fpos + tid;
      uint64_t c = 0;
      if (i < le) {
        const uint32_t w = ld_u32(&q[i]);
        c = g.row_ptr[w + 1] - g.row_ptr[w];
      }
      fpart += block_sum_u64<BLOCK>(c, sh.red);
      fpos += BLOCK;
    }
  }
  __syncthreads();
  if (tid == 0) {
    sh.hpos = hpos;
    sh.hub_pairs = hub;
  }
  __syncthreads();
  return run;
}

// Ring index of pair p: largest i with poff[i] <= p.
__device__ __forceinline__ int ring_of(const uint32_t* poff, uint32_t dt, uint32_t p) {
  int lo = 0, hi = static_cast<int>(dt) - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (poff[mid] <= p)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// Up to 512 threads the kernel is held to 6 waves per SIMD (at most 80
// VGPRs, some spill; with the 16 Kbit filter 12 workgroups of 128 threads
// fit a CU's LDS): more resident BFSs hide more of the latency of their
// dependent random accesses than the spill costs.
//
// MULTI: a fused launch over several graphs (sample pools).  Each work
// item's graph is looked up in the instance table and its arguments are
// placed in LDS, from where the BFS reads them; every other step is the
// same, so each hyperedge equals that of a launch on its graph alone.
template <int BLOCK, int UNROLL, bool LDS_BITS, bool MULTI = false>
__global__ __launch_bounds__(BLOCK, BLOCK <= 512 ? 6 : 1) void k_sample_paths(SampleArgs a) {
  __shared__ SampleShared<BLOCK> sh;
  __shared__ typename std::conditional<MULTI, SampleArgs, char>::type item_args;
  extern __shared__ uint32_t dyn_bits[];
  const int tid = threadIdx.x;
  const int lane = lane_id();
  const int wid = tid / kWave;
  const size_t slot = blockIdx.x;
  uint64_t* rec = a.rec + 2 * slot * a.slot_stride;
  uint32_t* q = a.q + slot * a.slot_stride;
  uint64_t* praw = a.praw + slot * kPairMax;
  uint32_t* pu = a.pinfo + slot * 3 * kPairMax;   // per pair: u, in_ptr[u], in-degree of u
  uint32_t* prs = pu + kPairMax;
  uint32_t* pdg = prs + kPairMax;
  using Bits = typename std::conditional<LDS_BITS, BitsLds, BitsRec>::type;
  Bits bits = make_bits<LDS_BITS>(dyn_bits, rec, sh.bloom);
  const uint64_t lane_lt = (1ull << lane) - 1ull;

  if (LDS_BITS)
    for (uint32_t i = tid; i < a.bit_words; i += BLOCK) dyn_bits[i] = 0;
  // work counters (uniform across the workgroup): arcs scanned, nodes visited
  uint64_t n_arcs = 0, n_nodes = 0;

  for (;;) {
    if (tid == 0) sh.next = atomicAdd(a.work, 1u);
    __syncthreads();
    const uint32_t idx = uniform_u32(sh.next);
    __syncthreads();
    if (idx >= a.count) break;
    if constexpr (MULTI) {
      if (tid == 0) {
        // the pool of work item idx: the last j with item_off[j] <= idx
        uint32_t lo = 0, hi = a.n_inst - 1;
        while (lo < hi) {
          const uint32_t mid = (lo + hi + 1) >> 1;
          if (a.item_off[mid] <= idx)
            lo = mid;
          else
            hi = mid - 1;
        }
        const SampleInst ins = a.inst[lo];
        SampleArgs v = a;
        v.n = ins.n;
        v.c_bits = ins.c_bits;
        v.max_out_deg = ins.max_out_deg;
        v.row_ptr = ins.row_ptr;
        v.col_idx = ins.col_idx;
        v.in_ptr = ins.in_ptr;
        v.in_idx = ins.in_idx;
        v.new_of = ins.new_of;
        v.orig_of = ins.orig_of;
        v.seed = ins.seed;
        v.instance = ins.instance;
        v.first = ins.first - a.item_off[lo];   // sample = first + idx (mod 2^64)
        item_args = v;
      }
      __syncthreads();
    }
    const SampleArgs& g = [&]() -> const SampleArgs& {
      if constexpr (MULTI) return item_args; else return a;
    }();
    const uint64_t cap = g.c_bits >= 64 ? ~0ull : (1ull << g.c_bits);
    const uint64_t sample = g.first + idx;
    bits.base = uint64_t(a.stamp0 + idx) << 32;

    // pair draw: every thread draws the same words (uniform, no broadcast)
    WordStream st(g.seed, sample, g.instance, 0);
    const uint32_t s0 = static_cast<uint32_t>(bounded(st, g.n));
    const uint32_t tp = static_cast<uint32_t>(bounded(st, g.n - 1));
    const uint32_t t0 = tp + (tp >= s0 ? 1u : 0u);
    const uint32_t s = g.new_of ? g.new_of[s0] : s0;   // traversal ids
    const uint32_t t = g.new_of ? g.new_of[t0] : t0;

    if (!LDS_BITS) {
      for (uint32_t i = tid; i < kBloomWords; i += BLOCK) sh.bloom[i] = 0;
      __syncthreads();
    }
    if (tid == 0) {
      st_u64(tag_of(rec, s), level_tag(bits.base, 0));
      st_u64(sig_of(rec, s), 1);
      st_u32(&q[0], s);
      bits.set(s);
      sh.qlen = 1;
    }

    // Rings around t: R1 = in(t), the pairs (w in R1, u in in(w)) and, if
    // the cone is small enough, in(u) for those u.  poff[i] = number of
    // pairs before R1's i-th entry.  The cone's size (CSR entries a 3-hop
    // test scans) is summed lazily: pairs [0, cpos) so far.
    const uint32_t tb = g.in_ptr[t], te = g.in_ptr[t + 1];
    const uint32_t dt = te - tb;
    const bool rings = dt <= Ring<BLOCK>::kCache;
    uint32_t pairs = 0, cpos = 0;
    uint64_t cone_part = 0;
    if (rings) {
      for (uint32_t cb = 0; cb < dt; cb += BLOCK) {
        const uint32_t i = cb + tid;
        uint32_t dw = 0;
        if (i < dt) {
          const uint32_t w = g.in_idx[tb + i];
          const uint32_t r0 = g.in_ptr[w];
          dw = g.in_ptr[w + 1] - r0;
          sh.rw[i] = w;
          sh.rrs[i] = r0;
        }
        uint32_t tot;
        const uint32_t o = block_excl_scan_u32<BLOCK>(dw, &tot, sh.scan);
        if (i < dt) sh.poff[i] = pairs + o;
        pairs += tot;
      }
      n_arcs += dt;
    }
    __syncthreads();
    // sizes the cone over the next BLOCK pairs, keeping each pair's u and
    // in-row for the 3-hop test
    auto cone_step = [&]() {
      const uint32_t p = cpos + tid;
      uint32_t dg = 0;
      if (p < pairs) {
        const int i = ring_of(sh.poff, dt, p);
        const uint32_t u = g.in_idx[sh.rrs[i] + (p - sh.poff[i])];
        const uint32_t r0 = g.in_ptr[u];
        dg = g.in_ptr[u + 1] - r0;
        st_u32(&pu[p], u);
        st_u32(&prs[p], r0);
        st_u32(&pdg[p], dg);
      }
      cone_part += block_sum_u64<BLOCK>(dg, sh.red);
      n_arcs += pairs - cpos < BLOCK ? pairs - cpos : BLOCK;
      cpos += BLOCK;
    };
    // Depth of t's ancestors when the rings show it: every ancestor of t is
    // within backward distance `depth`, so a reachable t has d <= depth and
    // the BFS can stop once the tests have ruled out d <= depth.  Pairs = 0
    // (t's in-neighbours have no in-neighbours) gives 1; a cone of size 0
    // gives 2 (sized here only when the pairs fit one chunk).
    uint32_t depth = kUnseen;
    if (rings && dt) {
      if (pairs == 0) {
        depth = 1;
      } else if (pairs <= BLOCK) {
        cone_step();
        if (cone_part == 0) depth = 2;
      }
    }

    // The 2-hop test of a t with more in-neighbours than the ring cache
    // scans the in-rows of all of them (sh.hub_pairs entries, sized lazily
    // over in(t) entries [0, sh.hpos); kept in LDS, as they are read once
    // per level); like test (2) it runs at a level only when those entries
    // are at most kPairRatio times the out-arcs expanding the level would
    // scan.
    if (tid == 0) {
      sh.hpos = 0;
      sh.hub_pairs = 0;
    }
    uint32_t lb = 0, le = 1, L = 0, d = kUnseen;
    uint64_t sumL = 1;        // S_L: sum of the level-L counts (saturating)
    uint32_t shortcut = 0;    // 2 or 3: levels L+1 (and L+2) were not produced
    uint64_t w_short = 0;     // W of the first backtrack step when shortcut
    uint64_t shifted = 0;     // bit l: the counts of produced level l < 64 were shifted
    // t without in-neighbours is unreachable: no BFS at all (on skewed
    // directed graphs such targets are common, and s may reach millions)
    bool deferred = false;
    const uint64_t arcs0 = n_arcs;   // this BFS's scans are n_arcs - arcs0
    for (; dt != 0;) {
      // (1) a visited in-neighbour of t: it is at level L (an earlier check
      //     would have fired otherwise), so d = L + 1
      int found = 0;
      n_arcs += dt;
      for (uint32_t e = tb + tid; e < te; e += BLOCK)
        if (bits.done(g.in_idx[e], L)) found = 1;
      if (__syncthreads_or(found)) {
        d = L + 1;
        break;
      }
      if (L + 1 >= depth) break;   // every d <= depth ruled out: unreachable
      if (rings) {
        // out-arcs of level L (the cost of expanding it), summed in
        // workgroup chunks only as far as a cost rule below needs: most
        // produced levels are never expanded
        uint32_t fpos = lb;
        uint64_t fpart = 0;
        auto fcost_step = [&]() {
          const uint32_t i = fpos + tid;
          uint64_t c = 0;
          if (i < le) {
            const uint32_t w = ld_u32(&q[i]);
            c = g.row_ptr[w + 1] - g.row_ptr[w];
          }
          fpart += block_sum_u64<BLOCK>(c, sh.red);
          fpos += BLOCK;
        };
        const uint64_t need2 = (pairs + kPairRatio - 1) / kPairRatio;
        while (fpos < le && fpart < need2) fcost_step();
        if (fpart >= need2) {
          // (2) pairs (w, u): a visited u is at level L (w is unvisited, so a
          //     lower level would have put w in a produced level), hence w at
          //     L+1 and d = L+2; ring_a[i] = sum of sigma'_u over visited u,
          //     the raw count of w_i
          for (uint32_t i = tid; i < dt; i += BLOCK) {
            sh.ring_a[i] = 0;
            sh.ring_b[i] = 0;
          }
          __syncthreads();
          int hit2 = 0;
          for (uint32_t p = tid; p < pairs; p += BLOCK) {
            const int i = ring_of(sh.poff, dt, p);
            const uint32_t u = g.in_idx[sh.rrs[i] + (p - sh.poff[i])];
            const uint64_t c = bits.count(u);   // 0: unvisited
            if (c) {
              hit2 = 1;
              atomicAdd(reinterpret_cast<unsigned long long*>(&sh.ring_a[i]), static_cast<unsigned long long>(c));
            }
          }
          n_arcs += pairs;
          if (__syncthreads_or(hit2)) {
            if (sumL < cap) {
              // no count of level L+1 can need a shift (each <= S_L < 2^C)
              d = L + 2;
              shortcut = 2;
              break;
            }
          } else if (L + 2 >= depth) {
            break;   // every d <= depth ruled out: unreachable
          } else if (pairs <= kPairMax) {
            // (3) cone: an unvisited u with visited in-neighbours is at L+1
            //     (they are all at L), its w at L+2 and d = L+3.  Only when
            //     the counts of levels L+1 and L+2 cannot need a shift (level
            //     L+1 counts <= S_L, level L+2 counts <= S_{L+1} <= S_L * max
            //     out-degree) and when the cone is at most kConeRatio times
            //     the out-arcs of level L.  That comparison grows both sums
            //     chunk by chunk until it is decided; sizing the cone also
            //     keeps each pair's u and in-row for the test.
            const uint64_t bound =
                (g.max_out_deg && sumL > ~0ull / g.max_out_deg) ? ~0ull : sumL * g.max_out_deg;
            bool cheap = false;
            if (sumL < cap && bound < cap) {
              for (;;) {
                const bool cdone = cpos >= pairs, fdone = fpos >= le;
                if (cdone && cone_part <= kConeRatio * fpart) {
                  cheap = true;
                  break;
                }
                if (fdone && cone_part > kConeRatio * fpart) break;
                if (!cdone && (fdone || cone_part <= kConeRatio * fpart))
                  cone_step();
                else
                  fcost_step();
              }
            }
            if (cheap) {
              int hit3 = 0;
              for (uint32_t cb = 0; cb < pairs; cb += BLOCK) {
                const uint32_t p = cb + tid;
                uint32_t u = kUnseen, r0 = 0, dg = 0;
                int i = 0;
                if (p < pairs) {
                  i = ring_of(sh.poff, dt, p);
                  u = ld_u32(&pu[p]);
                  r0 = ld_u32(&prs[p]);
                  dg = ld_u32(&pdg[p]);
                }
                raw_counts_chunk<BLOCK, UNROLL>(g, bits, rec, u, r0, dg, L, sh, n_arcs);
                const uint64_t raw = sh.sg[tid];
                if (p < pairs) st_u64(&praw[p], raw);
                if (raw) {
                  hit3 = 1;
                  atomicAdd(reinterpret_cast<unsigned long long*>(&sh.ring_b[i]), static_cast<unsigned long long>(raw));
                }
                __syncthreads();
              }
              if (__syncthreads_or(hit3)) {
                d = L + 3;
                shortcut = 3;
                break;
              }
            }
          }
        }
      } else if (sumL < cap && hub_rule<BLOCK>(g, q, tb, dt, lb, le, sh, n_arcs)) {
        // t with more in-neighbours than the ring cache: in-neighbours w of t
        // at level L+1, raw_w = sum of sigma' over w's in-neighbours at level L
        uint64_t wsum = 0, wscan = 0;
        for (uint32_t e = tb + wid; e < te; e += BLOCK / kWave) {
          const uint32_t w = g.in_idx[e];
          const uint32_t ub = g.in_ptr[w], ue = g.in_ptr[w + 1];
          uint64_t x = 0;
          for (uint32_t f = ub + lane; f < ue; f += kWave) {
            const uint32_t u = g.in_idx[f];
            // w is unvisited (check (1) failed), so a visited u is at level L
            x += bits.count(u);
          }
          wsum += wave_sum_u64(x);
          wscan += ue - ub;
        }
        if (lane != 0) {
          wsum = 0;
          wscan = 0;
        }
        wsum = block_sum_u64<BLOCK>(wsum, sh.red);
        n_arcs += block_sum_u64<BLOCK>(wscan, sh.red);
        if (wsum) {
          d = L + 2;
          shortcut = 2;
          w_short = wsum;
          break;
        }
      }
      if constexpr (!LDS_BITS && !MULTI) {
        // a level too wide for one workgroup, or a wide level of a BFS that
        // has already scanned millions of entries: the sample goes to the
        // device-wide BFS (if the list has room), which redraws it in full
        if (a.defer_nodes &&
            (le - lb > a.defer_nodes || (n_arcs - arcs0 > a.defer_arcs && le - lb >= kWideMinWidth)) &&
            defer_sample<BLOCK>(a, idx, sh)) {
          deferred = true;
          break;
        }
      }
      // expand level L (queue entries [lb, le)) into level L+1
      const uint32_t nl = L + 1;
      uint64_t mx = 0, added = 0;
      for (uint32_t cb = lb; cb < le; cb += BLOCK) {
        const uint32_t i = cb + tid;
        uint32_t deg = 0, rs = 0;
        uint64_t sw = 0;
        if (i < le) {
          const uint32_t w = ld_u32(&q[i]);
          rs = g.row_ptr[w];
          deg = g.row_ptr[w + 1] - rs;
          sw = ld_u64(sig_of(rec, w));
        }
        uint32_t total;
        const uint32_t off = block_excl_scan_u32<BLOCK>(deg, &total, sh.scan);
        n_arcs += total;
        if constexpr (!LDS_BITS && !MULTI) {
          // a level whose arcs run past the scan budget (hub frontiers): the
          // device-wide BFS redraws the sample (uniform; the partial level
          // is abandoned with the BFS's stamp)
          if (a.defer_nodes && n_arcs - arcs0 > a.defer_arcs && le - lb >= kWideMinWidth &&
              defer_sample<BLOCK>(a, idx, sh)) {
            deferred = true;
            break;
          }
        }
        sh.off[tid] = off;
        sh.rs[tid] = rs;
        sh.sg[tid] = sw;
        __syncthreads();
        for (uint32_t base = 0; base < total; base += BLOCK * UNROLL) {
          uint32_t v[UNROLL];
          uint64_t add[UNROLL];
          bool act[UNROLL], claimed[UNROLL];
#pragma unroll
          for (int k = 0; k < UNROLL; ++k) {
            const uint32_t e = base + k * BLOCK + tid;
            act[k] = e < total;
            v[k] = 0;
            add[k] = 0;
            if (act[k]) {
              // largest j with off[j] <= e (zero-degree entries share the
              // offset of the next entry, so the largest match has arcs)
              int lo = 0, hi = BLOCK - 1;
              while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (sh.off[mid] <= e)
                  lo = mid;
                else
                  hi = mid - 1;
              }
              v[k] = g.col_idx[sh.rs[lo] + (e - sh.off[lo])];
              add[k] = sh.sg[lo];
            }
          }
#pragma unroll
          for (int k = 0; k < UNROLL; ++k)
            if (act[k] && bits.done(v[k], L)) act[k] = false;
          const uint64_t tag_new = level_tag(bits.base, nl);
#pragma unroll
          for (int k = 0; k < UNROLL; ++k) {
            claimed[k] = false;
            if (act[k])
              claimed[k] = atomicMax(reinterpret_cast<unsigned long long*>(tag_of(rec, v[k])),
                                     static_cast<unsigned long long>(tag_new)) < bits.base;
          }
#pragma unroll
          for (int k = 0; k < UNROLL; ++k)
            if (claimed[k]) st_u64(sig_of(rec, v[k]), add[k]);
          __syncthreads();   // every claimed count is started before the other arrivals add
#pragma unroll
          for (int k = 0; k < UNROLL; ++k) {
            if (act[k]) {
              uint64_t x = add[k];
              if (!claimed[k])
                x += atomicAdd(reinterpret_cast<unsigned long long*>(sig_of(rec, v[k])),
                               static_cast<unsigned long long>(add[k]));
              mx = x > mx ? x : mx;
              added = sat_add(added, add[k]);
            }
            // wave-aggregated append of newly claimed nodes
            const uint64_t m = __ballot(claimed[k]);
            if (m) {
              uint32_t wbase = 0;
              const int leader = __ffsll(static_cast<unsigned long long>(m)) - 1;
              if (lane == leader) wbase = atomicAdd(&sh.qlen, static_cast<uint32_t>(__popcll(m)));
              wbase = __shfl(wbase, leader, kWave);
              if (claimed[k]) st_u32(&q[wbase + __popcll(m & lane_lt)], v[k]);
            }
          }
        }
        __syncthreads();
      }
      if (deferred) break;   // uniform
      const uint32_t ne = uniform_u32(sh.qlen);
      if (ne == le) break;   // nothing new: t unreachable
      // level L+1 is complete: its largest raw count decides the shift;
      // S_{L+1} is the sum of the added contributions, or of the shifted
      // counts when a shift applies
      mx = block_max_u64<BLOCK>(mx, sh.red);
      const uint32_t bl = bitlen64(mx);
      const uint32_t shift = bl > g.c_bits ? bl - g.c_bits : 0u;
      uint64_t ssum = 0;
      for (uint32_t i = le + tid; i < ne; i += BLOCK) {
        const uint32_t v = ld_u32(&q[i]);
        bits.set(v);
        if (shift) {
          uint64_t x = ld_u64(sig_of(rec, v)) >> shift;
          x = x ? x : 1ull;
          st_u64(sig_of(rec, v), x);
          ssum = sat_add(ssum, x);
        }
      }
      if (!shift) ssum = added;
      if (shift && nl < 64) shifted |= 1ull << nl;
      sumL = block_sat_sum<BLOCK>(ssum, sh.red);   // contains the barrier closing the level
      lb = le;
      le = ne;
      L = nl;
    }

    if (deferred) {   // uniform: nothing is staged for this sample here
      n_nodes += uniform_u32(sh.qlen);
      __syncthreads();
      continue;
    }

    // backtrack: from v = t, pick a predecessor w at level(v) - 1 with
    // probability sigma'_w / W, scanning in-neighbours in ascending order,
    // until level 1.  Workgroup wide (block_pick); steps through unproduced
    // levels (shortcut 2 or 3) take their weights from the ring sums and the
    // stored pair counts.
    const uint32_t len = (d != kUnseen && d >= 2) ? d - 1 : 0u;
    if (tid == 0) {
      sh.base = len ? atomicAdd(reinterpret_cast<unsigned long long*>(g.stage_used),
                                static_cast<unsigned long long>(len))
                    : 0ull;
    }
    uint32_t v = t, dv = len ? d : 0u, written = 0;   // no backtrack when t is unreachable or adjacent
    // W of the next step when known without a summing pass: the raw count
    // of v, i.e. the sum of its predecessors' counts (a ring sum or stored
    // pair count after a shortcut step; sigma'_v itself when v was claimed
    // at a level whose counts were not shifted)
    uint64_t w_next = 0;
    bool claimed_v = false;
    __syncthreads();   // sh.base, ring sums and stored pair counts are visible
    const uint64_t hbase = uniform_u64(sh.base);
    bool ok = true;
    if (dv && shortcut && rings) {
      // step from t through level d-1: weights ring_a (shortcut 2) or
      // ring_b (shortcut 3) of t's in-neighbours, in ascending order
      const uint64_t* wts = shortcut == 2 ? sh.ring_a : sh.ring_b;
      const uint32_t pi = block_pick<BLOCK>(dt, [&](uint32_t j) { return wts[j]; }, 0, st, sh);
      if (pi == kUnseen) {
        ok = false;
      } else {
        v = sh.rw[pi];
        if (tid == 0 && hbase < g.stage_cap) g.stage[hbase] = caller_id(g, v);
        written = 1;
        dv = d - 1;
        w_next = shortcut == 2 ? uniform_u64(sh.ring_a[pi]) : 0ull;
        if (shortcut == 3) {
          // step from w (level L+2) through level L+1: weights raw_u of the
          // pairs (w, u), stored by the cone test in in(w) order; their sum
          // is ring_b of w, i.e. sigma'_w
          const uint32_t p0 = sh.poff[pi];
          const uint32_t pn = (pi + 1 < dt ? sh.poff[pi + 1] : pairs) - p0;
          const uint32_t j =
              block_pick<BLOCK>(pn, [&](uint32_t jj) { return ld_u64(&praw[p0 + jj]); }, sh.ring_b[pi], st, sh);
          if (j == kUnseen) {
            ok = false;
          } else {
            w_next = uniform_u64(ld_u64(&praw[p0 + j]));
            v = g.in_idx[sh.rrs[pi] + j];
            if (tid == 0 && hbase + 1 < g.stage_cap) g.stage[hbase + 1] = caller_id(g, v);
            written = 2;
            dv = d - 2;
          }
        }
      }
    } else if (dv && shortcut) {
      // shortcut without the ring cache (t has many in-neighbours): the
      // first step recomputes raw_w, on wave 0 (every thread draws, so the
      // streams stay identical for the next steps)
      const uint64_t r = bounded(st, w_short);
      if (wid == 0) {
        uint64_t acc = 0;
        uint32_t pick = kUnseen;
        for (uint32_t e = tb; e < te; ++e) {
          const uint32_t w = g.in_idx[e];
          const uint32_t ub = g.in_ptr[w], ue = g.in_ptr[w + 1];
          uint64_t x = 0;
          for (uint32_t f = ub + lane; f < ue; f += kWave) x += bits.count(g.in_idx[f]);
          acc += wave_sum_u64(x);
          if (acc > r) {
            pick = w;
            break;
          }
        }
        if (lane == 0) sh.pick = pick;
      }
      __syncthreads();
      const uint32_t pick = uniform_u32(sh.pick);
      if (pick == kUnseen) {
        ok = false;
      } else {
        v = pick;
        if (tid == 0 && hbase < g.stage_cap) g.stage[hbase] = caller_id(g, v);
        written = 1;
        dv = d - 1;
      }
    }
    while (ok && dv >= 2) {
      const uint32_t want = dv - 1;
      const uint32_t vb = g.in_ptr[v], ve = g.in_ptr[v + 1];
      // a known W spares rows longer than one pick round their summing pass
      uint64_t wk = w_next;
      if (!wk && claimed_v && dv < 64 && !((shifted >> dv) & 1ull)) wk = ld_u64(sig_of(rec, v));
      wk = ve - vb > uint32_t(BLOCK) * kPickPer ? uniform_u64(wk) : 0ull;
      const uint32_t j = block_pick<BLOCK>(
          ve - vb, [&](uint32_t jj) { return pred_weight(bits, rec, g.in_idx[vb + jj], want); }, wk, st, sh);
      if (j == kUnseen) {
        ok = false;
        break;
      }
      w_next = 0;
      claimed_v = true;   // predecessors lie on produced levels
      v = g.in_idx[vb + j];
      if (tid == 0 && hbase + written < g.stage_cap) g.stage[hbase + written] = caller_id(g, v);
      ++written;
      --dv;
    }
    if (tid == 0) {
      if (!ok) atomicOr(g.flags, kErrBacktrack);
      g.stage_pos[idx] = hbase;
      g.he_len[idx] = len;
      if (g.st_out) {
        g.st_out[2 * size_t(idx)] = s0;
        g.st_out[2 * size_t(idx) + 1] = t0;
      }
      if (g.dist_out) g.dist_out[idx] = d;
    }
    __syncthreads();
    // the records keep this BFS's stamp (older than any later one); only
    // the LDS bitmap is cleared
    const uint32_t nv = uniform_u32(sh.qlen);
    n_nodes += nv;
    if (LDS_BITS) {
      for (uint32_t i = tid; i < nv; i += BLOCK) dyn_bits[ld_u32(&q[i]) >> 5] = 0;
      __syncthreads();
    }
  }
  // (a workgroup whose targets all lacked in-neighbours scanned no arc but
  // still gave every source a level)
  if (tid == 0 && a.stats && (n_arcs || n_nodes)) {
    atomicAdd(reinterpret_cast<unsigned long long*>(&a.stats[0]), static_cast<unsigned long long>(n_arcs));
    atomicAdd(reinterpret_cast<unsigned long long*>(&a.stats[1]), static_cast<unsigned long long>(n_nodes));
  }
}

// Lays the staged hyperedges out in sample order.
__global__ void k_stage_gather(uint32_t count, const uint64_t* stage_pos, const uint32_t* he_len,
                               const uint64_t* rel_off, uint64_t base, const uint32_t* stage, uint64_t* he_off,
                               uint32_t* he_nodes) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i > count) return;
  const uint64_t o = rel_off[i];
  if (he_off) he_off[i] = base + o;
  if (i == count) return;
  if (!he_nodes) return;
  const uint64_t p = stage_pos[i];
  const uint32_t len = he_len[i];
  for (uint32_t x = 0; x < len; ++x) he_nodes[o + x] = stage[p + x];
}

// Launch wrappers for the host side of the sampler (sample_launch.hip).
hipError_t sample_kernel_occupancy(int block, bool lds_bits, bool multi, size_t dyn_lds, int* per_cu) {
  if (lds_bits) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_sample_paths<kLdsBlock, kUnroll, true>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(dyn_lds));
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k_sample_paths<kLdsBlock, kUnroll, true>, kLdsBlock,
                                                        dyn_lds);
  }
#define CENTRA_OCC(B, M) hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k_sample_paths<B, kUnroll, false, M>, B, 0)
  switch (block) {
    case 512: return multi ? CENTRA_OCC(512, true) : CENTRA_OCC(512, false);
    case 256: return multi ? CENTRA_OCC(256, true) : CENTRA_OCC(256, false);
    case 64: return multi ? CENTRA_OCC(64, true) : CENTRA_OCC(64, false);
    default: return multi ? CENTRA_OCC(128, true) : CENTRA_OCC(128, false);
  }
#undef CENTRA_OCC
}

size_t sample_lds_variant_bytes() { return sizeof(SampleShared<kLdsBlock>); }

void sample_kernel_launch(const SampleArgs& a, int block, bool lds_bits, bool multi, uint32_t grid, size_t dyn_lds,
                          hipStream_t s) {
  if (lds_bits) {
    hipLaunchKernelGGL((k_sample_paths<kLdsBlock, kUnroll, true>), dim3(grid), dim3(kLdsBlock), dyn_lds, s, a);
    return;
  }
#define CENTRA_LAUNCH(B, M) hipLaunchKernelGGL((k_sample_paths<B, kUnroll, false, M>), dim3(grid), dim3(B), 0, s, a)
  switch (block) {
    case 512:
      if (multi)
        CENTRA_LAUNCH(512, true);
      else
        CENTRA_LAUNCH(512, false);
      break;
    case 256:
      if (multi)
        CENTRA_LAUNCH(256, true);
      else
        CENTRA_LAUNCH(256, false);
      break;
    case 64:
      if (multi)
        CENTRA_LAUNCH(64, true);
      else
        CENTRA_LAUNCH(64, false);
      break;
    default:
      if (multi)
        CENTRA_LAUNCH(128, true);
      else
        CENTRA_LAUNCH(128, false);
      break;
  }
#undef CENTRA_LAUNCH
}

// ---------------------------------------------------------------------------
// Device-wide BFS of a deferred sample.  A few samples of skewed graphs
// flood millions of nodes (R-MAT scale 22: one in about 300k floods the 2M
// nodes its source reaches, 63M arcs), which takes one 128-thread workgroup
// about a second and holds its launch that long.  Such a sample is redrawn
// here with each level expanded by the whole GPU: full levels (no ring
// tests), which give the same levels, normalised counts and predecessor
// weights as the shortcuts do, then the same backtrack over the same word
// stream, so the hyperedge is the one the workgroup kernel would stage.
// The state is slot 0's records and queue (the launch that deferred the
// sample has finished) under a stamp of its own.
constexpr int kWideBlock = 256;
constexpr unsigned kWideGrid = 2048;
// a level is pulled when the unvisited nodes' in-arcs (plus a quarter of n
// for reading every tag) are fewer than kPullRatio times the frontier's
// out-arcs: a push scans them twice and claims with returning atomics
constexpr uint64_t kPullRatio = 8;

// ctl: [0] queue length, [1] largest raw count of the new level, [2] 1 if
// t is on the new level, [3] out-arcs of the last level (the cost of
// pushing it), [4] t (traversal id), [5] in-arcs of the visited nodes
// (the graph's in-arcs less the cost of pulling), [6] arcs scanned, [7]
// nodes given a level
__global__ void k_wide_start(SampleArgs a, uint32_t idx, uint64_t base, uint64_t* ctl) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  WordStream st(a.seed, a.first + idx, a.instance, 0);
  const uint32_t s0 = static_cast<uint32_t>(bounded(st, a.n));
  const uint32_t tp = static_cast<uint32_t>(bounded(st, a.n - 1));
  const uint32_t t0 = tp + (tp >= s0 ? 1u : 0u);
  const uint32_t s = a.new_of ? a.new_of[s0] : s0;
  const uint32_t t = a.new_of ? a.new_of[t0] : t0;
  st_u64(tag_of(a.rec, s), level_tag(base, 0));
  st_u64(sig_of(a.rec, s), 1);
  st_u32(&a.q[0], s);
  ctl[0] = 1;
  ctl[1] = 0;
  ctl[2] = 0;
  ctl[3] = a.row_ptr[s + 1] - a.row_ptr[s];
  ctl[4] = t;
  ctl[5] = a.in_ptr[s + 1] - a.in_ptr[s];
  ctl[6] = 0;
  ctl[7] = 1;
}

// Level nl - 1 = queue entries [lb, le) expanded by every workgroup, a
// chunk of kWideBlock frontier nodes at a time: pass 0 claims the new
// level's nodes (returning atomic max on the tag; the claimer zeroes the
// count and appends the node, one queue atomic per wave), pass 1 adds each
// frontier node's count to its new-level out-neighbours.
template <int PASS>
__global__ __launch_bounds__(kWideBlock) void k_wide_level(SampleArgs a, uint32_t lb, uint32_t le, uint64_t base,
                                                           uint32_t nl, uint64_t* ctl) {
  __shared__ uint32_t off[kWideBlock], rs[kWideBlock], scan[kWideBlock / kWave + 1];
  __shared__ uint64_t sg[kWideBlock];
  const int tid = threadIdx.x, lane = lane_id();
  const uint64_t tag_new = level_tag(base, nl);
  const uint64_t lane_lt = (1ull << lane) - 1ull;
  uint64_t arcs = 0;
  for (uint64_t cb = lb + uint64_t(blockIdx.x) * kWideBlock; cb < le; cb += uint64_t(gridDim.x) * kWideBlock) {
    const uint64_t i = cb + tid;
    uint32_t deg = 0, r0 = 0;
    uint64_t sw = 0;
    if (i < le) {
      const uint32_t w = ld_u32(&a.q[i]);
      r0 = a.row_ptr[w];
      deg = a.row_ptr[w + 1] - r0;
      if (PASS == 1) sw = ld_u64(sig_of(a.rec, w));
    }
    uint32_t total;
    const uint32_t o = block_excl_scan_u32<kWideBlock>(deg, &total, scan);
    off[tid] = o;
    rs[tid] = r0;
    sg[tid] = sw;
    arcs += total;
    __syncthreads();
    for (uint32_t e0 = 0; e0 < total; e0 += kWideBlock) {   // uniform trip count
      const uint32_t e = e0 + tid;
      bool claimed = false;
      uint32_t v = 0;
      if (e < total) {
        int lo = 0, hi = kWideBlock - 1;   // the last j with off[j] <= e (it has arcs)
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (off[mid] <= e)
            lo = mid;
          else
            hi = mid - 1;
        }
        v = a.col_idx[rs[lo] + (e - off[lo])];
        if (PASS == 0) {
          // most arcs of a flood reach visited nodes: a plain look at the
          // tag spares them the returning atomic
          if (ld_u64(tag_of(a.rec, v)) < base)
            claimed = atomicMax(reinterpret_cast<unsigned long long*>(tag_of(a.rec, v)),
                                static_cast<unsigned long long>(tag_new)) < base;
          if (claimed) st_u64(sig_of(a.rec, v), 0);
        } else if (ld_u64(tag_of(a.rec, v)) == tag_new) {
          atomicAdd(reinterpret_cast<unsigned long long*>(sig_of(a.rec, v)), static_cast<unsigned long long>(sg[lo]));
        }
      }
      if (PASS == 0) {
        const uint64_t m = __ballot(claimed);
        if (m) {
          const int leader = __ffsll(static_cast<unsigned long long>(m)) - 1;
          uint64_t wb = 0;
          if (lane == leader)
            wb = atomicAdd(reinterpret_cast<unsigned long long*>(&ctl[0]), static_cast<unsigned long long>(__popcll(m)));
          wb = __shfl(wb, leader, kWave);
          if (claimed) st_u32(&a.q[wb + __popcll(m & lane_lt)], v);
        }
      }
    }
    __syncthreads();   // off, rs and sg are reused by the next chunk
  }
  // arcs is uniform over the workgroup (each chunk's total): one add
  if (PASS == 0 && a.stats && tid == 0 && arcs)
    atomicAdd(reinterpret_cast<unsigned long long*>(&a.stats[0]), static_cast<unsigned long long>(arcs));
}

// Level nl pulled instead of pushed (late levels of a flood, when the
// unvisited nodes' in-arcs are fewer than the frontier's out-arcs): every
// unvisited node sums the counts of its in-neighbours on level nl - 1; a
// positive sum puts it on level nl with that raw count.  Each node is
// written by its own thread only, so no atomics on the records.
__global__ __launch_bounds__(kWideBlock) void k_wide_pull(SampleArgs a, uint64_t base, uint32_t nl, uint64_t* ctl) {
  __shared__ uint64_t red[kWideBlock / kWave];
  const int lane = lane_id();
  const uint64_t tag_new = level_tag(base, nl), tag_prev = level_tag(base, nl - 1);
  const uint64_t lane_lt = (1ull << lane) - 1ull;
  uint64_t arcs = 0;
  const uint64_t n_pad = (uint64_t(a.n) + kWideBlock - 1) / kWideBlock * kWideBlock;   // uniform trip count
  for (uint64_t v0 = uint64_t(blockIdx.x) * kWideBlock; v0 < n_pad; v0 += uint64_t(gridDim.x) * kWideBlock) {
    const uint64_t v = v0 + threadIdx.x;
    bool claimed = false;
    if (v < a.n && ld_u64(tag_of(a.rec, static_cast<uint32_t>(v))) < base) {
      const uint32_t ib = a.in_ptr[v], ie = a.in_ptr[v + 1];
      uint64_t raw = 0;
      for (uint32_t e = ib; e < ie; ++e) {
        const uint32_t w = a.in_idx[e];
        if (ld_u64(tag_of(a.rec, w)) == tag_prev) raw += ld_u64(sig_of(a.rec, w));
      }
      arcs += ie - ib;
      if (raw) {
        st_u64(sig_of(a.rec, static_cast<uint32_t>(v)), raw);
        st_u64(tag_of(a.rec, static_cast<uint32_t>(v)), tag_new);
        claimed = true;
      }
    }
    const uint64_t m = __ballot(claimed);
    if (m) {
      const int leader = __ffsll(static_cast<unsigned long long>(m)) - 1;
      uint64_t wb = 0;
      if (lane == leader)
        wb = atomicAdd(reinterpret_cast<unsigned long long*>(&ctl[0]), static_cast<unsigned long long>(__popcll(m)));
      wb = __shfl(wb, leader, kWave);
      if (claimed) st_u32(&a.q[wb + __popcll(m & lane_lt)], static_cast<uint32_t>(v));
    }
  }
  arcs = block_sum_u64<kWideBlock>(arcs, red);
  if (threadIdx.x == 0 && a.stats && arcs)
    atomicAdd(reinterpret_cast<unsigned long long*>(&a.stats[0]), static_cast<unsigned long long>(arcs));
}

// The new level [le, ne = ctl[0]): its largest raw count into ctl[1]
// (zeroed by the caller), whether t is on it into ctl[2], its size into
// the node statistics.
__global__ __launch_bounds__(kWideBlock) void k_wide_close(SampleArgs a, uint32_t le, uint64_t base, uint32_t nl,
                                                           uint32_t t, uint64_t* ctl) {
  __shared__ uint64_t red[kWideBlock / kWave];
  const uint32_t ne = static_cast<uint32_t>(ctl[0]);
  uint64_t mx = 0, out_arcs = 0, in_arcs = 0;
  for (uint64_t i = le + uint64_t(blockIdx.x) * kWideBlock + threadIdx.x; i < ne; i += uint64_t(gridDim.x) * kWideBlock) {
    const uint32_t v = ld_u32(&a.q[i]);
    const uint64_t x = ld_u64(sig_of(a.rec, v));
    mx = x > mx ? x : mx;
    out_arcs += a.row_ptr[v + 1] - a.row_ptr[v];
    in_arcs += a.in_ptr[v + 1] - a.in_ptr[v];
  }
  mx = block_max_u64<kWideBlock>(mx, red);
  out_arcs = block_sum_u64<kWideBlock>(out_arcs, red);
  in_arcs = block_sum_u64<kWideBlock>(in_arcs, red);
  if (threadIdx.x == 0) {
    if (mx) atomicMax(reinterpret_cast<unsigned long long*>(&ctl[1]), static_cast<unsigned long long>(mx));
    if (out_arcs) atomicAdd(reinterpret_cast<unsigned long long*>(&ctl[3]), static_cast<unsigned long long>(out_arcs));
    if (in_arcs) atomicAdd(reinterpret_cast<unsigned long long*>(&ctl[5]), static_cast<unsigned long long>(in_arcs));
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ctl[2] = ld_u64(tag_of(a.rec, t)) == level_tag(base, nl) ? 1u : 0u;
    if (a.stats) atomicAdd(reinterpret_cast<unsigned long long*>(&a.stats[1]), static_cast<unsigned long long>(ne - le));
  }
}

// Normalisation of the new level: sigma' = max(1, raw >> shift).
__global__ void k_wide_shift(SampleArgs a, uint32_t le, uint32_t ne, uint32_t shift) {
  for (uint64_t i = le + uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < ne; i += uint64_t(gridDim.x) * blockDim.x) {
    uint64_t* p = sig_of(a.rec, ld_u32(&a.q[i]));
    const uint64_t x = ld_u64(p) >> shift;
    st_u64(p, x ? x : 1ull);
  }
}

// The backtrack of the sample (t at distance d, kUnseen if unreachable) by
// one workgroup over the same word stream as the workgroup kernel (the
// pair's words, then one bounded draw per step), staged the same way.
__global__ __launch_bounds__(kWideBlock) void k_wide_backtrack(SampleArgs a, uint32_t idx, uint64_t base, uint32_t d) {
  __shared__ SampleShared<kWideBlock> sh;
  const int tid = threadIdx.x;
  WordStream st(a.seed, a.first + idx, a.instance, 0);
  const uint32_t s0 = static_cast<uint32_t>(bounded(st, a.n));
  const uint32_t tp = static_cast<uint32_t>(bounded(st, a.n - 1));
  const uint32_t t0 = tp + (tp >= s0 ? 1u : 0u);
  const uint32_t t = a.new_of ? a.new_of[t0] : t0;
  const uint32_t len = (d != kUnseen && d >= 2) ? d - 1 : 0u;
  if (tid == 0)
    sh.base = len ? atomicAdd(reinterpret_cast<unsigned long long*>(a.stage_used), static_cast<unsigned long long>(len))
                  : 0ull;
  __syncthreads();
  const uint64_t hbase = uniform_u64(sh.base);
  uint32_t v = t, dv = len ? d : 0u, written = 0;
  bool ok = true;
  while (dv >= 2) {
    const uint32_t want = dv - 1;
    const uint64_t tag_want = level_tag(base, want);
    const uint32_t vb = a.in_ptr[v], ve = a.in_ptr[v + 1];
    const uint32_t j = block_pick<kWideBlock>(
        ve - vb,
        [&](uint32_t jj) {
          const uint32_t w = a.in_idx[vb + jj];
          const uint64_t tg = ld_u64(tag_of(a.rec, w));
          const uint64_t c = ld_u64(sig_of(a.rec, w));
          return tg == tag_want ? c : 0ull;
        },
        0, st, sh);
    if (j == kUnseen) {
      ok = false;
      break;
    }
    v = a.in_idx[vb + j];
    if (tid == 0 && hbase + written < a.stage_cap) a.stage[hbase + written] = caller_id(a, v);
    ++written;
    --dv;
  }
  if (tid == 0) {
    if (!ok) atomicOr(a.flags, kErrBacktrack);
    a.stage_pos[idx] = hbase;
    a.he_len[idx] = len;
    if (a.st_out) {
      a.st_out[2 * size_t(idx)] = s0;
      a.st_out[2 * size_t(idx) + 1] = t0;
    }
    if (a.dist_out) a.dist_out[idx] = d;
  }
}

int wide_samples(const SampleArgs& a_in, const uint32_t* idx, uint32_t n_items, uint64_t stamp0, uint64_t* ctl,
                 uint64_t* host_ctl, uint64_t* arcs, hipStream_t s) {
  // per sample j: slot j's records and queue, ctl + 8 j, stamp stamp0 + j
  struct Walk {
    SampleArgs a;
    uint64_t base, push_cost, visited_in;
    uint32_t t, lb, le, L, d;
    bool live;
  };
  std::vector<Walk> w(n_items);
  for (uint32_t j = 0; j < n_items; ++j) {
    Walk& x = w[j];
    x.a = a_in;
    x.a.rec = a_in.rec + 2 * size_t(j) * a_in.slot_stride;
    x.a.q = a_in.q + size_t(j) * a_in.slot_stride;
    x.a.stats = ctl + 8 * size_t(j) + 6;   // its arcs and nodes, apart from the workgroup kernel's
    x.base = (stamp0 + j) << 32;
    hipLaunchKernelGGL(k_wide_start, dim3(1), dim3(64), 0, s, x.a, idx[j], x.base, ctl + 8 * size_t(j));
  }
  const size_t ctl_bytes = size_t(n_items) * 8 * 8;
  if (hipMemcpyAsync(host_ctl, ctl, ctl_bytes, hipMemcpyDeviceToHost, s) != hipSuccess) return CENTRA_EHIP;
  if (hipStreamSynchronize(s) != hipSuccess) return CENTRA_EHIP;
  for (uint32_t j = 0; j < n_items; ++j) {
    Walk& x = w[j];
    x.t = static_cast<uint32_t>(host_ctl[8 * j + 4]);
    x.lb = 0;
    x.le = 1;
    x.L = 0;
    x.d = kUnseen;
    x.live = true;
    x.push_cost = host_ctl[8 * j + 3];
    x.visited_in = host_ctl[8 * j + 5];
  }
  // rounds: every live sample expands one level (pushed, or pulled when the
  // unvisited nodes' in-arcs cost less than pushing the frontier twice)
  // and closes it; one synchronisation per round reads every sample's new
  // level size, maximum, costs and whether t is on it
  for (uint32_t live = n_items; live;) {
    for (uint32_t j = 0; j < n_items; ++j) {
      Walk& x = w[j];
      if (!x.live) continue;
      uint64_t* c = ctl + 8 * size_t(j);
      const uint32_t nl = x.L + 1;
      const uint64_t pull_cost = (x.a.n_arcs - x.visited_in) + x.a.n / 4;
      fill_u64(c + 1, 0, 3, s);
      if (pull_cost < kPullRatio * x.push_cost) {
        hipLaunchKernelGGL(k_wide_pull, dim3(kWideGrid), dim3(kWideBlock), 0, s, x.a, x.base, nl, c);
      } else {
        const unsigned grid = std::min<uint64_t>(kWideGrid, (uint64_t(x.le - x.lb) + kWideBlock - 1) / kWideBlock);
        hipLaunchKernelGGL(k_wide_level<0>, dim3(grid), dim3(kWideBlock), 0, s, x.a, x.lb, x.le, x.base, nl, c);
        hipLaunchKernelGGL(k_wide_level<1>, dim3(grid), dim3(kWideBlock), 0, s, x.a, x.lb, x.le, x.base, nl, c);
      }
      hipLaunchKernelGGL(k_wide_close, dim3(kWideGrid), dim3(kWideBlock), 0, s, x.a, x.le, x.base, nl, x.t, c);
    }
    if (hipMemcpyAsync(host_ctl, ctl, ctl_bytes, hipMemcpyDeviceToHost, s) != hipSuccess) return CENTRA_EHIP;
    if (hipStreamSynchronize(s) != hipSuccess) return CENTRA_EHIP;
    for (uint32_t j = 0; j < n_items; ++j) {
      Walk& x = w[j];
      if (!x.live) continue;
      const uint64_t* h = host_ctl + 8 * size_t(j);
      const uint32_t nl = x.L + 1, ne = static_cast<uint32_t>(h[0]);
      if (ne == x.le || h[2]) {   // nothing new (t unreachable), or t on level nl
        x.d = ne == x.le ? kUnseen : nl;
        x.live = false;
        --live;
        continue;
      }
      uint32_t bl = 0;
      for (uint64_t v = h[1]; v; v >>= 1) ++bl;
      const uint32_t shift = bl > x.a.c_bits ? bl - x.a.c_bits : 0u;
      if (shift) {
        const unsigned gc = std::min<uint64_t>(kWideGrid, (uint64_t(ne - x.le) + kWideBlock - 1) / kWideBlock);
        hipLaunchKernelGGL(k_wide_shift, dim3(gc), dim3(kWideBlock), 0, s, x.a, x.le, ne, shift);
      }
      x.push_cost = h[3];
      x.visited_in = h[5];
      x.lb = x.le;
      x.le = ne;
      x.L = nl;
    }
  }
  for (uint32_t j = 0; j < n_items; ++j)
    hipLaunchKernelGGL(k_wide_backtrack, dim3(1), dim3(kWideBlock), 0, s, w[j].a, idx[j], w[j].base, w[j].d);
  if (hipGetLastError() != hipSuccess) return CENTRA_EHIP;
  if (hipMemcpyAsync(host_ctl, ctl, ctl_bytes, hipMemcpyDeviceToHost, s) != hipSuccess) return CENTRA_EHIP;
  if (hipStreamSynchronize(s) != hipSuccess) return CENTRA_EHIP;
  *arcs = 0;
  for (uint32_t j = 0; j < n_items; ++j) *arcs += host_ctl[8 * j + 6];
  return CENTRA_OK;
}

void stage_gather_launch(uint32_t count, const uint64_t* stage_pos, const uint32_t* he_len, const uint64_t* rel_off,
                         uint64_t base, const uint32_t* stage, uint64_t* he_off, uint32_t* he_nodes, hipStream_t s) {
  hipLaunchKernelGGL(k_stage_gather, dim3((count + 1 + 255) / 256), dim3(256), 0, s, count, stage_pos, he_len, rel_off,
                     base, stage, he_off, he_nodes);
}

}  // namespace centra
