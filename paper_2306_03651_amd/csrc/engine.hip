// The batching and serving engine: Algorithm 1 for many (graph, k, eps,
// delta) queries at once, over sample pools kept resident on the device.
//
// A pool is one graph with one sample stream (seed, instance): its samples
// are a prefix of that stream, drawn as queries need them, and its sample
// sizes follow one geometric schedule m_0 = m_init, m_{j+1} =
// min(ceil(m_j g), m_max) (the sampling schedule of Algorithm 1).  For each
// level j the pool keeps what every query at that sample size needs: the
// incidence segment of samples [m_{j-1}, m_j) (so levels 0..j form the
// incidence of the first m_j samples), deg_H over [0, m_j), the
// trial-major Rademacher sums R_j = 2 P_j - deg_j of its t trials, and
// max |h|.  Because samples and signs are functions of (seed, instance,
// sample index, trial) only, a query's iteration i on the pool sees exactly
// the hyperedges, signs and counts that centra_progressive would draw for
// the same parameters alone, whoever drew them and whenever: each result
// is that of a standalone run.
//
// A query holds only its greedy round state and its outputs.  One engine
// tick advances every admitted query by one iteration:
//   1. queries that have arrived are admitted in arrival order while the
//      engine's device memory stays within its budget;
//   2. pools that lack the level some query needs draw the missing samples
//      in one fused sampling launch over all such pools (the multi-pool
//      form of the BFS kernel), then build the level's incidence segment
//      and Rademacher sums;
//   3. the greedy rounds of all active queries run fused: one argmax and
//      one covering launch per round for every query together (blockIdx.y
//      picks the query), the rounds replayed from a captured HIP graph;
//   4. the per-trial top-k sums of all queries run fused (one selection
//      over every query's t trial rows and degree row);
//   5. one copy brings every query's counts to the host, which evaluates
//      the bound of Theorem bound_dev and retires certified queries (and
//      those at the pool's last level).
// Queries arriving while others run join at the next tick: their work
// shares the fused launches with the running ones (continuous batching).
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <map>
#include <string>
#include <thread>
#include <vector>

#include "common.hpp"
#include "internal.hpp"

namespace centra {

namespace {

// Destination of one pool's staged samples in a fused launch.
struct GatherDesc {
  uint64_t* he_off;     // pool offsets at the first new sample
  uint32_t* he_nodes;   // pool nodes at the first new entry
  uint64_t base;        // entries before the first new sample
  uint64_t rel0;        // staged offset of the pool's first item
};

// Lays each pool's staged hyperedges out in its store, sample after
// sample: item i of pool j writes offset he_off[local + 1] and its nodes.
__global__ void k_gather_pools(uint32_t count, const uint32_t* item_off, uint32_t n_pools, const GatherDesc* d,
                               const uint64_t* stage_pos, const uint32_t* he_len, const uint64_t* rel,
                               const uint32_t* stage) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  uint32_t lo = 0, hi = n_pools - 1;
  while (lo < hi) {
    const uint32_t mid = (lo + hi + 1) >> 1;
    if (item_off[mid] <= i)
      lo = mid;
    else
      hi = mid - 1;
  }
  const GatherDesc g = d[lo];
  const uint32_t local = i - item_off[lo];
  const uint64_t o = rel[i] - g.rel0;
  const uint32_t len = he_len[i];
  g.he_off[local + 1] = g.base + o + len;
  const uint64_t p = stage_pos[i];
  for (uint32_t x = 0; x < len; ++x) g.he_nodes[o + x] = stage[p + x];
}

__global__ void k_copy_u32(const uint32_t* src, uint32_t* dst, uint64_t n) {
  for (uint64_t i = blockIdx.x * uint64_t(blockDim.x) + threadIdx.x; i < n; i += uint64_t(gridDim.x) * blockDim.x)
    dst[i] = src[i];
}

unsigned grid_for(uint64_t n, unsigned block, unsigned cap = 16384) {
  uint64_t g = (n + block - 1) / block;
  if (g > cap) g = cap;
  return g ? static_cast<unsigned>(g) : 1u;
}

double now_s() {
  using clk = std::chrono::steady_clock;
  static const clk::time_point t0 = clk::now();
  return std::chrono::duration<double>(clk::now() - t0).count();
}

}  // namespace

// Results of one level of a pool, kept for later queries at that level:
// they depend only on the level's samples (functions of their indices), so
// a query reuses them bit for bit.  Greedy: the picks of a run of gk rounds
// (gnp < gk: it stopped early, so every larger k has the same picks).
// Selection: for each trial row and the degree row, the sum of its i + 1
// largest positive values for every i < sK (ssat: every row has fewer than
// sK positive values, so any k takes them all).
struct LevelCache {
  uint32_t gk = 0, gnp = 0;
  std::vector<uint32_t> picks;
  std::vector<uint64_t> cov;
  uint32_t sK = 0, st = 0;
  bool ssat = false;
  std::vector<int64_t> topk;   // [trial][i], st x sK
  std::vector<int64_t> dk;     // [i], sK
};

struct EnginePool {
  const centra_graph* g = nullptr;
  centra_pool_params p{};
  uint32_t k_hint = 0;                 // the largest k submitted on the pool
  std::vector<LevelCache> cache;       // per level
  std::vector<uint64_t> level_m;   // the schedule m_0 < m_1 < ... <= m_max
  uint32_t levels_built = 0;
  uint64_t m_have = 0, I_have = 0;
  DevBuf off, nodes, inc, inc_node, seg_off, cursor, sdeg, deg_cur, tiles, words, P, bmax;
  std::vector<DevBuf> deg, R;        // per level
  std::vector<uint32_t> bmax_host;   // per level
  uint32_t active = 0;               // admitted queries not yet done
  uint32_t queued = 0;               // submitted queries not yet admitted
  bool released = false;             // some level's R and deg were released
};

struct EngineQuery {
  uint32_t pool = 0;
  uint32_t k = 0, t = 0;
  double eps = 0, delta = 0, arrival = 0, admitted = -1, finished = -1;
  int state = 0;   // 0 queued, 1 active, 2 done
  uint32_t level = 0;
  int rc = 0;
  centra_result res{};
  std::vector<uint32_t> picks;
  size_t bytes = 0;
};

}  // namespace centra

namespace centra {
// The device state of one greedy run of a tick (shared by the queries at
// one level of one pool); reused from tick to tick.
struct GreedyWs {
  DevBuf gain, covered, part, best, cand;   // best: best | newcov; cand: list | state | histogram
};
}  // namespace centra

struct centra_engine {
  centra_ctx* ctx = nullptr;
  std::vector<centra::GreedyWs> ws;
  size_t budget = 0;
  uint32_t flags = 0;
  std::vector<centra::EnginePool> pools;
  std::vector<centra::EngineQuery> queries;
  size_t next_queued = 0;   // queries before this index were admitted (arrival order = submit order)
  centra::DevBuf descs, rows, sel_ws, tick_res, round_base, gather;
  hipStream_t cap_stream = nullptr;
  // captured greedy rounds, keyed by (descriptor capacity, argmax grid, cover grid)
  std::map<std::tuple<uint32_t, uint32_t, uint32_t>, hipGraphExec_t> graphs;
  void* graphs_for = nullptr;   // descriptor buffer the captured graphs read
  int tuned_block = 0;
  centra_engine_stats st{};
  std::string log;
  double run_t0 = 0;
};

namespace centra {

static constexpr uint32_t kRoundChunk = 8;   // greedy rounds per captured graph

static size_t pool_bytes(const EnginePool& p) {
  size_t b = p.off.bytes + p.nodes.bytes + p.inc.bytes + p.inc_node.bytes + p.seg_off.bytes + p.cursor.bytes +
             p.sdeg.bytes + p.deg_cur.bytes + p.tiles.bytes + p.words.bytes + p.P.bytes + p.bmax.bytes;
  for (const DevBuf& d : p.deg) b += d.bytes;
  for (const DevBuf& r : p.R) b += r.bytes;
  return b;
}

static size_t ws_bytes(const GreedyWs& w);

static size_t engine_bytes(const centra_engine* e) {
  size_t b = 0;
  for (const EnginePool& p : e->pools) b += pool_bytes(p);
  for (const GreedyWs& w : e->ws) b += ws_bytes(w);
  return b;
}

static size_t cand_bytes() { return (size_t(greedy_cand_words()) + 4 + greedy_hist_words()) * 4 + 256; }

// Device bytes a pool reaches with every level of its schedule built (none
// released), from the mean hyperedge size of the samples it holds, plus a
// tenth for the estimate.  Admission reserves this for every pool with an
// active query.
static size_t pool_projection(const EnginePool& p) {
  const size_t n = p.g->n, t = p.p.t, M = p.p.m_max, L = p.level_m.size();
  const double mean_h = p.m_have ? double(p.I_have) / double(p.m_have) : 0.0;
  const size_t I = static_cast<size_t>(mean_h * double(M)) + 1;
  const size_t Wt = (t + 63) / 64;
  // per level: R_j and deg_j, and one greedy run's state (gains, covered
  // bitmap, candidate list, round state for k up to 1,024)
  const size_t per_level = n * (t + 1) * 4 + n * 4 + (M / 32 + 1) * 4 + cand_bytes() + greedy_part_words() * 8 +
                           1024 * 16;
  const size_t b = (M + 1) * 8 + I * 12 + M * Wt * 8 + n * t * 4 + L * (n + 1) * 8 + n * 24 +
                   scan_tile_words(n) * 8 + 64 * 4 + L * per_level;
  return b + b / 10;
}

// Memory that admission compares with the budget: each pool with an
// active query at its projection (which includes its greedy runs' state)
// or its present size if larger, idle pools at their present size.
static size_t engine_reserved(const centra_engine* e) {
  size_t b = 0;
  for (const EnginePool& p : e->pools) b += p.active ? std::max(pool_bytes(p), pool_projection(p)) : pool_bytes(p);
  return b;
}



static size_t ws_bytes(const GreedyWs& w) {
  return w.gain.bytes + w.covered.bytes + w.part.bytes + w.best.bytes + w.cand.bytes;
}

// Draws the samples of every pool up to its target level in one fused
// launch and lays them out in the pools' stores.
static int sample_pools(centra_engine* e, const std::vector<uint32_t>& want_level, hipStream_t s) {
  centra_ctx* ctx = e->ctx;
  std::vector<MultiSampleItem> items;
  std::vector<uint32_t> which;
  for (uint32_t pi = 0; pi < e->pools.size(); ++pi) {
    EnginePool& p = e->pools[pi];
    if (want_level[pi] == ~0u) continue;
    const uint64_t target = p.level_m[want_level[pi]];
    if (target <= p.m_have) continue;
    items.push_back(MultiSampleItem{p.g, p.p.seed, p.p.instance, p.m_have, static_cast<uint32_t>(target - p.m_have)});
    which.push_back(pi);
  }
  if (items.empty()) return CENTRA_OK;
  hipEvent_t* ev = ctx->ev;
  CENTRA_HIP(ctx, hipEventRecord(ev[0], s));
  uint64_t total = 0;
  const int block = e->tuned_block ? e->tuned_block : 128;
  int rc = sample_multi_to_stage(ctx, items.data(), static_cast<uint32_t>(items.size()), block, &total, s);
  if (rc) return rc;
  uint64_t count = 0;
  std::vector<uint32_t> item_off;
  for (const MultiSampleItem& it : items) {
    item_off.push_back(static_cast<uint32_t>(count));
    count += it.count;
  }
  item_off.push_back(static_cast<uint32_t>(count));
  // relative offsets of every staged item, then each pool's entry count
  uint32_t* len = static_cast<uint32_t*>(ctx->stage_len.ptr);
  uint64_t* rel = reinterpret_cast<uint64_t*>(static_cast<char*>(ctx->stage_len.ptr) + ((count * 4 + 7) & ~uint64_t(7)));
  if ((rc = excl_scan_u32_to_u64(ctx, len, rel, count, s))) return rc;
  std::vector<uint64_t> rel_at(items.size() + 1);
  for (size_t i = 0; i <= items.size(); ++i)
    CENTRA_HIP(ctx, hipMemcpyAsync(&rel_at[i], rel + item_off[i], 8, hipMemcpyDeviceToHost, s));
  CENTRA_HIP(ctx, hipStreamSynchronize(s));
  std::vector<GatherDesc> gd(items.size());
  for (size_t i = 0; i < items.size(); ++i) {
    EnginePool& p = e->pools[which[i]];
    const uint64_t add = rel_at[i + 1] - rel_at[i];
    if ((rc = ensure(ctx, p.nodes, (p.I_have + add + 1) * 4, true, s))) return rc;
    uint64_t* off = static_cast<uint64_t*>(p.off.ptr);
    gd[i] = GatherDesc{off + p.m_have, static_cast<uint32_t*>(p.nodes.ptr) + p.I_have, p.I_have, rel_at[i]};
  }
  const size_t gbytes = gd.size() * sizeof(GatherDesc) + item_off.size() * 4 + 256;
  if ((rc = ensure(ctx, e->gather, gbytes, false, s))) return rc;
  char* gb = static_cast<char*>(e->gather.ptr);
  const size_t io_at = (gd.size() * sizeof(GatherDesc) + 255) & ~size_t(255);
  CENTRA_HIP(ctx, hipMemcpyAsync(gb, gd.data(), gd.size() * sizeof(GatherDesc), hipMemcpyHostToDevice, s));
  CENTRA_HIP(ctx, hipMemcpyAsync(gb + io_at, item_off.data(), item_off.size() * 4, hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(k_gather_pools, dim3(grid_for(count, 256, 1u << 30)), dim3(256), 0, s, static_cast<uint32_t>(count),
                     reinterpret_cast<const uint32_t*>(gb + io_at), static_cast<uint32_t>(gd.size()),
                     reinterpret_cast<const GatherDesc*>(gb), static_cast<const uint64_t*>(ctx->stage_pos.ptr), len,
                     rel, static_cast<const uint32_t*>(ctx->stage_nodes.ptr));
  CENTRA_HIP(ctx, hipGetLastError());
  CENTRA_HIP(ctx, hipEventRecord(ev[1], s));
  CENTRA_HIP(ctx, hipStreamSynchronize(s));   // gd and item_off are read by the copies above
  float ms = 0.f;
  (void)hipEventElapsedTime(&ms, ev[0], ev[1]);
  e->st.ms_sample += ms;
  e->st.sampler_launches += 1;
  e->st.samples += count;
  for (size_t i = 0; i < items.size(); ++i) {
    EnginePool& p = e->pools[which[i]];
    p.m_have += items[i].count;
    p.I_have += rel_at[i + 1] - rel_at[i];
  }
  return CENTRA_OK;
}

// Builds level j of a pool whose samples reach m_j: the incidence segment
// of [m_{j-1}, m_j), deg_j, the Rademacher sums R_j and max |h|.
static int build_level(centra_engine* e, EnginePool& p, uint32_t j, hipStream_t s) {
  centra_ctx* ctx = e->ctx;
  const uint32_t n = p.g->n, t = p.p.t;
  const uint64_t m0 = j ? p.level_m[j - 1] : 0, m1 = p.level_m[j];
  const uint32_t Wt = (t + 63) / 64;
  uint64_t ends[2] = {0, 0};
  const uint64_t* off = static_cast<const uint64_t*>(p.off.ptr);
  CENTRA_HIP(ctx, hipMemcpyAsync(&ends[0], off + m0, 8, hipMemcpyDeviceToHost, s));
  CENTRA_HIP(ctx, hipMemcpyAsync(&ends[1], off + m1, 8, hipMemcpyDeviceToHost, s));
  CENTRA_HIP(ctx, hipStreamSynchronize(s));
  const uint64_t I0 = ends[0], I1 = ends[1];
  int rc;
  if ((rc = ensure(ctx, p.inc, (I1 ? I1 : 1) * 4, true, s))) return rc;
  if ((rc = ensure(ctx, p.inc_node, (I1 ? I1 : 1) * 4, true, s))) return rc;
  if ((rc = ensure(ctx, p.seg_off, (size_t(j) + 1) * (size_t(n) + 1) * 8, true, s))) return rc;
  if ((rc = ensure(ctx, p.cursor, size_t(n) * 8, false, s))) return rc;
  if ((rc = ensure(ctx, p.sdeg, size_t(n) * 4, false, s))) return rc;
  if ((rc = ensure(ctx, p.deg_cur, size_t(n) * 4, true, s))) return rc;
  if ((rc = ensure(ctx, p.tiles, scan_tile_words(n) * 8, false, s))) return rc;
  if ((rc = ensure(ctx, p.words, size_t(m1) * Wt * 8, true, s))) return rc;
  if ((rc = ensure(ctx, p.P, size_t(n) * t * 4, true, s))) return rc;
  if ((rc = ensure(ctx, p.bmax, 64 * 4, true, s))) return rc;
  if (p.deg.size() <= j) p.deg.resize(j + 1);
  if (p.R.size() <= j) p.R.resize(j + 1);
  if ((rc = ensure(ctx, p.deg[j], size_t(n) * 4, false, s))) return rc;
  if ((rc = ensure(ctx, p.R[j], size_t(n) * t * 4, false, s))) return rc;
  uint32_t* deg_cur = static_cast<uint32_t*>(p.deg_cur.ptr);
  if (n <= kIncBucketMaxNodes) {
    if ((rc = ensure(ctx, ctx->inc_ws, incidence_ws_bytes(n, I1 - I0), false, s))) return rc;
    incidence_segment_bucketed(n, m0, m1, I1 - I0, I1, off, static_cast<const uint32_t*>(p.nodes.ptr), j == 0, deg_cur,
                               static_cast<uint32_t*>(p.sdeg.ptr), static_cast<uint64_t*>(p.seg_off.ptr) + size_t(j) * (n + 1),
                               static_cast<uint64_t*>(p.cursor.ptr), static_cast<uint32_t*>(p.inc.ptr),
                               static_cast<uint32_t*>(p.inc_node.ptr), ctx->inc_ws.ptr, ctx->d_flags, s);
  } else {
    incidence_segment(n, m0, m1, I1 - I0, I1, off, static_cast<const uint32_t*>(p.nodes.ptr), j == 0, deg_cur,
                      static_cast<uint32_t*>(p.sdeg.ptr), static_cast<uint64_t*>(p.seg_off.ptr) + size_t(j) * (n + 1),
                      static_cast<uint64_t*>(p.cursor.ptr), static_cast<uint32_t*>(p.inc.ptr),
                      static_cast<uint32_t*>(p.inc_node.ptr), static_cast<uint64_t*>(p.tiles.ptr), ctx->d_flags, s);
  }
  uint32_t* degj = static_cast<uint32_t*>(p.deg[j].ptr);
  hipLaunchKernelGGL(k_copy_u32, dim3(grid_for(n, 256)), dim3(256), 0, s, deg_cur, degj, uint64_t(n));
  uint64_t* words = static_cast<uint64_t*>(p.words.ptr);
  rade_words_launch(p.p.seed, p.p.instance, m0, m1, t, words, s);
  int32_t* P = static_cast<int32_t*>(p.P.ptr);
  if (j == 0) fill_u32(reinterpret_cast<uint32_t*>(P), 0, size_t(n) * t, s);
  rade_count_launch(static_cast<const uint32_t*>(p.inc.ptr), static_cast<const uint32_t*>(p.inc_node.ptr), off, m0, m1,
                    I1 - I0, I1, words, t, P, s);
  rade_finish_launch(P, degj, n, t, static_cast<int32_t*>(p.R[j].ptr), s);
  uint32_t* bm = static_cast<uint32_t*>(p.bmax.ptr);
  if (j == 0)
    fill_u32(bm, 0, 1, s);
  else
    hipLaunchKernelGGL(k_copy_u32, dim3(1), dim3(64), 0, s, bm + (j - 1), bm + j, uint64_t(1));
  bmax_launch(off, m0, m1, bm + j, s);
  CENTRA_HIP(ctx, hipGetLastError());
  uint32_t host_bm = 0;
  CENTRA_HIP(ctx, hipMemcpyAsync(&host_bm, bm + j, 4, hipMemcpyDeviceToHost, s));
  CENTRA_HIP(ctx, hipStreamSynchronize(s));
  if ((rc = check_flags(ctx, s, "engine level"))) return rc;
  if (p.bmax_host.size() <= j) p.bmax_host.resize(j + 1);
  p.bmax_host[j] = host_bm;
  p.levels_built = j + 1;
  return CENTRA_OK;
}

// Autotuner: times the fused sampling launch of a probe batch (the first
// samples of every pool) with workgroups of 128, 256 and 512 threads, the
// best of two timed launches after one that pays the slot set-up, and keeps
// the fastest unless it beats the default 128 by under 2% (differences
// within the probe's noise did not carry over to full launches).  64-thread
// workgroups are not tried: they won short probes but lost full launches,
// whose twice as many slots carry twice the slot state.  The probe's
// samples are the pools' own, and every variant draws the same hyperedges,
// so the choice changes no result.  CENTRA_TUNE_CACHE names a file of
// "key block" lines that keeps choices across runs.
static int autotune(centra_engine* e, hipStream_t s) {
  centra_ctx* ctx = e->ctx;
  char key[160];
  uint64_t nsum = 0, asum = 0;
  for (const EnginePool& p : e->pools) {
    nsum += p.g->n;
    asum += p.g->n_arcs;
  }
  snprintf(key, sizeof(key), "pools=%zu,nodes=%llu,arcs=%llu", e->pools.size(), (unsigned long long)nsum,
           (unsigned long long)asum);
  const char* cache = getenv("CENTRA_TUNE_CACHE");
  if (cache) {
    if (FILE* f = fopen(cache, "r")) {
      char k[160];
      int b = 0;
      while (fscanf(f, "%159s %d", k, &b) == 2)
        if (!strcmp(k, key) && (b == 64 || b == 128 || b == 256 || b == 512)) e->tuned_block = b;
      fclose(f);
      if (e->tuned_block) {
        e->log += std::string("autotune: ") + key + " -> block " + std::to_string(e->tuned_block) + " (cache)\n";
        return CENTRA_OK;
      }
    }
  }
  std::vector<MultiSampleItem> probe;
  for (const EnginePool& p : e->pools) {
    const uint64_t c = std::min<uint64_t>(p.level_m[0], std::max<uint64_t>(64, 16384 / e->pools.size()));
    probe.push_back(MultiSampleItem{p.g, p.p.seed, p.p.instance, 0, static_cast<uint32_t>(c)});
  }
  const int blocks[] = {128, 256, 512};
  constexpr int kDefaultBlock = 128;
  float best_ms = 0.f, default_ms = 0.f;
  int best = kDefaultBlock;
  std::string line = std::string("autotune: ") + key + ":";
  for (int b : blocks) {
    uint64_t total = 0;
    float ms = 0.f;
    for (int rep = 0; rep < 3; ++rep) {   // the first run pays the slot set-up
      int rc = sample_multi_to_stage(ctx, probe.data(), static_cast<uint32_t>(probe.size()), b, &total, s);
      if (rc) return rc;
      float t = 0.f;
      if (hipEventElapsedTime(&t, ctx->ev[6], ctx->ev[7]) != hipSuccess) t = 0.f;
      if (rep == 1 || (rep > 1 && t < ms)) ms = t;
    }
    line += " " + std::to_string(b) + "=" + std::to_string(ms) + "ms";
    if (b == kDefaultBlock) default_ms = ms;
    if (best_ms == 0.f || ms < best_ms) {
      best_ms = ms;
      best = b;
    }
  }
  if (best != kDefaultBlock && default_ms > 0.f && best_ms > 0.98f * default_ms) best = kDefaultBlock;
  e->tuned_block = best;
  e->log += line + " -> block " + std::to_string(best) + "\n";
  if (cache)
    if (FILE* f = fopen(cache, "a")) {
      fprintf(f, "%s %d\n", key, best);
      fclose(f);
    }
  return CENTRA_OK;
}

// Layout of one active query's outputs in the tick's result block.
struct ResLayout {
  size_t picks, cov, np, topk, dk, end;
};
static ResLayout res_layout(size_t at, uint32_t k, uint32_t t) {
  ResLayout L;
  L.picks = at;
  L.cov = (at + size_t(k) * 4 + 7) & ~size_t(7);
  L.np = L.cov + size_t(k) * 8;
  L.topk = L.np + 8;
  L.dk = L.topk + size_t(t) * 8;
  L.end = L.dk + 8;
  return L;
}

static int greedy_rounds(centra_engine* e, uint32_t cap_q, uint32_t max_n, uint32_t gc, uint32_t kmax, hipStream_t s) {
  centra_ctx* ctx = e->ctx;
  GreedyDesc* d = static_cast<GreedyDesc*>(e->descs.ptr);
  uint32_t* rb = static_cast<uint32_t*>(e->round_base.ptr);
  fill_u32(rb, 0, 1, s);
  const uint32_t chunks = (kmax + kRoundChunk - 1) / kRoundChunk;
  if (e->flags & CENTRA_ENGINE_NO_GRAPHS) {
    for (uint32_t c = 0; c < chunks; ++c) greedy_multi_rounds(d, cap_q, max_n, gc, rb, kRoundChunk, s);
    CENTRA_HIP(ctx, hipGetLastError());
    e->st.greedy_launches += uint64_t(chunks) * (4 * kRoundChunk + 1);
    return CENTRA_OK;
  }
  if (e->graphs_for != e->descs.ptr) {   // the descriptor buffer moved: drop graphs that read the old one
    for (auto& kv : e->graphs) (void)hipGraphExecDestroy(kv.second);
    e->graphs.clear();
    e->graphs_for = e->descs.ptr;
  }
  const auto gkey = std::make_tuple(cap_q, max_n, gc);
  auto it = e->graphs.find(gkey);
  if (it == e->graphs.end()) {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    CENTRA_HIP(ctx, hipStreamBeginCapture(e->cap_stream, hipStreamCaptureModeThreadLocal));
    greedy_multi_rounds(d, cap_q, max_n, gc, rb, kRoundChunk, e->cap_stream);
    hipError_t err = hipStreamEndCapture(e->cap_stream, &graph);
    if (err != hipSuccess) return hip_fail(ctx, err, "engine: greedy capture");
    err = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (err != hipSuccess) return hip_fail(ctx, err, "engine: graph instantiate");
    it = e->graphs.emplace(gkey, exec).first;
    e->st.graphs_captured += 1;
  }
  for (uint32_t c = 0; c < chunks; ++c) CENTRA_HIP(ctx, hipGraphLaunch(it->second, s));
  e->st.graph_replays += chunks;
  return CENTRA_OK;
}

// Drops every level of an idle pool, with its incidence, signs and counts
// (its samples stay): levels are built again, from level 0, as queries
// need them.
static void reset_levels(centra_engine* e, EnginePool& p) {
  for (DevBuf& d : p.deg) release(e->ctx, d);
  for (DevBuf& r : p.R) release(e->ctx, r);
  DevBuf* bufs[] = {&p.inc, &p.inc_node, &p.seg_off, &p.cursor, &p.sdeg, &p.deg_cur, &p.tiles, &p.words, &p.P,
                    &p.bmax};
  for (DevBuf* b : bufs) release(e->ctx, *b);
  p.levels_built = 0;
  p.released = false;
}

// Releases the per-level arrays (R_j, deg_j) of a pool that no queued or
// active query can need again: every active query is past level j and none
// is waiting.  They hold most of a pool's memory when many pools share the
// device (one level of R is n t 4 bytes).
static void release_levels(centra_engine* e, EnginePool& p, uint32_t pool_id) {
  if (p.queued) return;
  if (!p.active) {   // idle with nothing waiting: keep the samples only
    if (p.levels_built || p.P.ptr) reset_levels(e, p);
    return;
  }
  uint32_t lowest = p.levels_built;
  for (const EngineQuery& q : e->queries)
    if (q.state == 1 && q.pool == pool_id) lowest = std::min(lowest, q.level);
  for (uint32_t j = 0; j < lowest && j < p.R.size(); ++j) {
    if (p.R[j].ptr || p.deg[j].ptr) p.released = true;
    release(e->ctx, p.R[j]);
    release(e->ctx, p.deg[j]);
  }
}

// One tick (see the file comment).  *progress is set when any query was
// admitted or advanced.
static int tick(centra_engine* e, double now, bool* progress, hipStream_t s) {
  centra_ctx* ctx = e->ctx;
  *progress = false;
  int rc;
  // 1. admission.  Pools of arrived queries that hold no samples yet draw
  // their first level first (one fused launch), which gives the mean
  // hyperedge size their memory projection needs.
  const double t_adm = now_s() - e->run_t0;
  {
    std::vector<uint32_t> first(e->pools.size(), ~0u);
    bool any = false;
    for (size_t i = e->next_queued; i < e->queries.size() && e->queries[i].arrival <= now; ++i) {
      const uint32_t pi = e->queries[i].pool;
      if (e->pools[pi].m_have == 0) {
        first[pi] = 0;
        any = true;
      }
    }
    if (any && (rc = sample_pools(e, first, s))) return rc;
  }
  while (e->next_queued < e->queries.size()) {
    EngineQuery& q = e->queries[e->next_queued];
    if (q.arrival > now) break;
    EnginePool& p = e->pools[q.pool];
    if (p.released) {
      // levels of this pool were released when no query needed them; a
      // new query rebuilds them once the pool is idle (samples are kept)
      if (p.active) break;
      reset_levels(e, p);
    }
    // if its pool is idle, the pool's projection
    const size_t pool_add = p.active ? 0 : std::max(pool_bytes(p), pool_projection(p)) - pool_bytes(p);
    if (e->budget && engine_reserved(e) + pool_add > e->budget) {
      bool any_active = false;
      for (const EngineQuery& o : e->queries) any_active |= o.state == 1;
      if (any_active) break;   // wait for memory to free up
      q.state = 2;             // alone it cannot fit: refused
      q.rc = CENTRA_ENOMEM;
      q.admitted = q.finished = t_adm;
      p.queued -= 1;
      ++e->next_queued;
      *progress = true;
      continue;
    }
    q.state = 1;
    q.level = 0;
    q.admitted = t_adm;
    p.active += 1;
    p.queued -= 1;
    ++e->next_queued;
    *progress = true;
  }
  std::vector<uint32_t> act;
  for (uint32_t i = 0; i < e->queries.size(); ++i)
    if (e->queries[i].state == 1) act.push_back(i);
  if (act.empty()) return CENTRA_OK;
  *progress = true;
  e->st.ticks += 1;
  if (act.size() > e->st.peak_active) e->st.peak_active = static_cast<uint32_t>(act.size());
  if (!e->tuned_block && !(e->flags & CENTRA_ENGINE_NO_TUNE)) {
    if ((rc = autotune(e, s))) return rc;
  }
  // 2. levels
  std::vector<uint32_t> want(e->pools.size(), ~0u);
  for (uint32_t i : act) {
    const EngineQuery& q = e->queries[i];
    if (want[q.pool] == ~0u || q.level > want[q.pool]) want[q.pool] = q.level;
  }
  for (uint32_t pi = 0; pi < e->pools.size(); ++pi)
    if (want[pi] != ~0u && want[pi] < e->pools[pi].levels_built) want[pi] = ~0u;
  if ((rc = sample_pools(e, want, s))) return rc;
  {
    hipEvent_t* ev = ctx->ev;
    CENTRA_HIP(ctx, hipEventRecord(ev[2], s));
    for (uint32_t pi = 0; pi < e->pools.size(); ++pi) {
      if (want[pi] == ~0u) continue;
      EnginePool& p = e->pools[pi];
      while (p.levels_built <= want[pi])
        if ((rc = build_level(e, p, p.levels_built, s))) return rc;
    }
    CENTRA_HIP(ctx, hipEventRecord(ev[3], s));
    CENTRA_HIP(ctx, hipStreamSynchronize(s));
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, ev[2], ev[3]);
    e->st.ms_levels += ms;
  }
  // 3.-4. fused greedy and selection
  // Greedy is prefix-consistent in k (its first k picks are the picks of
  // any larger k on the same sample, with the same cumulative coverage), so
  // the queries at one level of one pool share a single greedy run with the
  // largest of their k.  With the level caches (the default), a run takes
  // the largest k submitted on the pool, its picks are kept, and so are,
  // for every k up to that size, the per-trial top-k sums of the level
  // (one selection per level, prefix sums of each row's sorted largest
  // values): a later query at the level reuses both.  Without them, queries
  // that share k share their selection rows (the largest of their t, each
  // query summing its first t trials).
  const bool cached = !(e->flags & CENTRA_ENGINE_NO_CACHE);
  struct GGroup {
    uint32_t pool, level, k;
    ResLayout lay;
  };
  struct SGroup {
    uint32_t pool, level, k, t;
    size_t topk, dk;
  };
  std::vector<GGroup> gg;
  std::vector<SGroup> sg;
  std::vector<uint32_t> q_gg(act.size(), ~0u), q_sg(act.size(), ~0u);
  uint32_t K_sel = 0;   // cached selections: the prefix length of this tick
  {
    std::map<std::pair<uint32_t, uint32_t>, uint32_t> gmap;
    std::map<std::tuple<uint32_t, uint32_t, uint32_t>, uint32_t> smap;
    for (size_t a = 0; a < act.size(); ++a) {
      const EngineQuery& q = e->queries[act[a]];
      EnginePool& p = e->pools[q.pool];
      if (p.cache.size() < p.level_m.size()) p.cache.resize(p.level_m.size());
      const LevelCache& C = p.cache[q.level];
      const bool g_hit = cached && C.gk && (C.gk >= q.k || C.gnp < C.gk);
      const bool s_hit = cached && C.sK && C.st >= q.t && (q.k <= C.sK || C.ssat);
      if (!g_hit) {
        auto gk = std::make_pair(q.pool, q.level);
        auto git = gmap.find(gk);
        if (git == gmap.end()) {
          git = gmap.emplace(gk, static_cast<uint32_t>(gg.size())).first;
          gg.push_back(GGroup{q.pool, q.level, 0, {}});
        }
        gg[git->second].k = std::max(gg[git->second].k, cached ? std::max(q.k, p.k_hint) : q.k);
        q_gg[a] = git->second;
      }
      if (!s_hit) {
        const uint32_t kk = cached ? 0u : q.k;
        auto sk = std::make_tuple(q.pool, q.level, kk);
        auto sit = smap.find(sk);
        if (sit == smap.end()) {
          sit = smap.emplace(sk, static_cast<uint32_t>(sg.size())).first;
          sg.push_back(SGroup{q.pool, q.level, kk, 0, 0, 0});
        }
        SGroup& S = sg[sit->second];
        S.t = cached ? p.p.t : std::max(S.t, q.t);
        if (cached) K_sel = std::max(K_sel, std::max(q.k, p.k_hint));
        q_sg[a] = sit->second;
      }
    }
  }
  // a prefix longer than the sort can hold: this tick's selections by
  // exact k (not kept)
  const bool sel_prefix = cached && K_sel <= kSelPrefixMax;
  if (cached && !sel_prefix) {
    std::map<std::tuple<uint32_t, uint32_t, uint32_t>, uint32_t> smap;
    std::vector<SGroup> sg2;
    for (size_t a = 0; a < act.size(); ++a) {
      if (q_sg[a] == ~0u) continue;
      const EngineQuery& q = e->queries[act[a]];
      auto sk = std::make_tuple(q.pool, q.level, q.k);
      auto sit = smap.find(sk);
      if (sit == smap.end()) {
        sit = smap.emplace(sk, static_cast<uint32_t>(sg2.size())).first;
        sg2.push_back(SGroup{q.pool, q.level, q.k, 0, 0, 0});
      }
      sg2[sit->second].t = std::max(sg2[sit->second].t, q.t);
      q_sg[a] = sit->second;
    }
    sg.swap(sg2);
  }
  uint32_t cap_q = 1;
  while (cap_q < gg.size()) cap_q <<= 1;
  std::vector<GreedyDesc> gd(cap_q);
  memset(gd.data(), 0, gd.size() * sizeof(GreedyDesc));
  size_t res_bytes = 0;
  uint32_t max_n = 0, kmax = 0, n_rows = 0, max_n_sel = 0;
  uint64_t max_m = 0;
  for (GGroup& G : gg) {
    G.lay = res_layout(res_bytes, G.k, 0);
    res_bytes = G.lay.end;
    const EnginePool& p = e->pools[G.pool];
    max_n = std::max(max_n, p.g->n);
    kmax = std::max(kmax, G.k);
    max_m = std::max(max_m, p.level_m[G.level]);
  }
  for (SGroup& S : sg) {
    if (sel_prefix) {
      S.k = K_sel;
      S.topk = res_bytes;
      S.dk = res_bytes + size_t(S.t) * K_sel * 8;
      res_bytes = S.dk + size_t(K_sel) * 8;
    } else {
      S.topk = res_bytes;
      S.dk = res_bytes + size_t(S.t) * 8;
      res_bytes = S.dk + 8;
    }
    n_rows += S.t + 1;
    max_n_sel = std::max(max_n_sel, e->pools[S.pool].g->n);
  }
  const size_t sel_bytes = sel_prefix ? select_prefix_ws_bytes(n_rows, K_sel) : select_ws_bytes(n_rows);
  if ((rc = ensure(ctx, e->tick_res, res_bytes + 256, false, s))) return rc;
  if ((rc = ensure(ctx, e->descs, size_t(cap_q) * sizeof(GreedyDesc), false, s))) return rc;
  if ((rc = ensure(ctx, e->rows, size_t(n_rows ? n_rows : 1) * sizeof(SelRow), false, s))) return rc;
  if ((rc = ensure(ctx, e->sel_ws, sel_bytes, false, s))) return rc;
  if ((rc = ensure(ctx, e->round_base, 256, false, s))) return rc;
  if (e->ws.size() < gg.size()) e->ws.resize(gg.size());
  char* res = static_cast<char*>(e->tick_res.ptr);
  for (size_t gi = 0; gi < gg.size(); ++gi) {
    const GGroup& G = gg[gi];
    EnginePool& p = e->pools[G.pool];
    GreedyWs& w = e->ws[gi];
    const uint32_t j = G.level, n = p.g->n;
    if ((rc = ensure(ctx, w.gain, size_t(n) * 4, false, s))) return rc;
    if ((rc = ensure(ctx, w.covered, ((p.level_m[j] + 31) / 32 + 1) * 4, false, s))) return rc;
    if ((rc = ensure(ctx, w.part, size_t(greedy_part_words()) * 8, false, s))) return rc;
    if ((rc = ensure(ctx, w.best, size_t(G.k) * 16, false, s))) return rc;
    if ((rc = ensure(ctx, w.cand, cand_bytes(), false, s))) return rc;
    GreedyDesc& d = gd[gi];
    d.gain = static_cast<int32_t*>(w.gain.ptr);
    d.covered = static_cast<uint32_t*>(w.covered.ptr);
    d.part = static_cast<uint64_t*>(w.part.ptr);
    d.best = static_cast<uint64_t*>(w.best.ptr);
    d.newcov = d.best + G.k;
    d.cand = static_cast<uint32_t*>(w.cand.ptr);
    d.cst = d.cand + greedy_cand_words();
    d.hist = d.cst + 4;
    d.deg = static_cast<const uint32_t*>(p.deg[j].ptr);
    d.seg_off = static_cast<const uint64_t*>(p.seg_off.ptr);
    d.inc = static_cast<const uint32_t*>(p.inc.ptr);
    d.he_off = static_cast<const uint64_t*>(p.off.ptr);
    d.he_nodes = static_cast<const uint32_t*>(p.nodes.ptr);
    d.picks = reinterpret_cast<uint32_t*>(res + G.lay.picks);
    d.cov_cum = reinterpret_cast<uint64_t*>(res + G.lay.cov);
    d.n_picked = reinterpret_cast<uint32_t*>(res + G.lay.np);
    d.m = p.level_m[j];
    d.n = n;
    d.n_seg = j + 1;
    d.k = G.k;
  }
  std::vector<SelRow> rows;
  rows.reserve(n_rows);
  for (const SGroup& S : sg) {
    const EnginePool& p = e->pools[S.pool];
    const uint32_t n = p.g->n;
    const int32_t* R = static_cast<const int32_t*>(p.R[S.level].ptr);
    for (uint32_t r = 0; r < S.t; ++r)
      rows.push_back(SelRow{R + size_t(r) * n, n, S.k, sel_prefix ? nullptr : reinterpret_cast<int64_t*>(res + S.topk) + r});
    rows.push_back(SelRow{static_cast<const int32_t*>(p.deg[S.level].ptr), n, S.k,
                          sel_prefix ? nullptr : reinterpret_cast<int64_t*>(res + S.dk)});
  }
  e->st.greedy_runs += gg.size();
  GreedyDesc* dd = static_cast<GreedyDesc*>(e->descs.ptr);
  SelRow* dr = static_cast<SelRow*>(e->rows.ptr);
  if (!gg.empty()) CENTRA_HIP(ctx, hipMemcpyAsync(dd, gd.data(), gd.size() * sizeof(GreedyDesc), hipMemcpyHostToDevice, s));
  if (n_rows) CENTRA_HIP(ctx, hipMemcpyAsync(dr, rows.data(), rows.size() * sizeof(SelRow), hipMemcpyHostToDevice, s));
  hipEvent_t* ev = ctx->ev;
  CENTRA_HIP(ctx, hipEventRecord(ev[4], s));
  if (!gg.empty()) {
    greedy_multi_init(dd, cap_q, max_n, s);
    // cover parts per run: enough for the longest incidence row a run can
    // meet (at most its sample size) at 256 entries each, at most 256 (a
    // part then walks its share of the row in strides)
    uint32_t gc = static_cast<uint32_t>(std::min<uint64_t>(256, (max_m + 255) / 256));
    gc = std::max<uint32_t>(gc, 16);
    uint32_t gcp = 16;
    while (gcp < gc) gcp <<= 1;   // a few graph shapes only
    // the captured graphs are keyed by the argmax shape: round max_n up
    uint32_t max_n_key = 4096;
    while (max_n_key < max_n) max_n_key <<= 1;
    if ((rc = greedy_rounds(e, cap_q, max_n_key, gcp, kmax, s))) return rc;
    greedy_multi_finish(dd, cap_q, s);
  }
  CENTRA_HIP(ctx, hipEventRecord(ev[5], s));
  if (n_rows) {
    if (sel_prefix)
      select_prefix_rows(dr, n_rows, max_n_sel, K_sel, e->sel_ws.ptr,
                         reinterpret_cast<int64_t*>(res + (sg.empty() ? 0 : sg[0].topk)), s);
    else
      select_topk_rows(dr, n_rows, max_n_sel, e->sel_ws.ptr, s);
  }
  CENTRA_HIP(ctx, hipGetLastError());
  CENTRA_HIP(ctx, hipEventRecord(ev[6], s));
  std::string host(res_bytes, '\0');
  if (res_bytes) CENTRA_HIP(ctx, hipMemcpyAsync(&host[0], res, res_bytes, hipMemcpyDeviceToHost, s));
  CENTRA_HIP(ctx, hipStreamSynchronize(s));
  if ((rc = check_flags(ctx, s, "engine tick"))) return rc;
  float ms_g = 0.f, ms_s = 0.f;
  (void)hipEventElapsedTime(&ms_g, ev[4], ev[5]);
  (void)hipEventElapsedTime(&ms_s, ev[5], ev[6]);
  e->st.ms_greedy += ms_g;
  e->st.ms_select += ms_s;
  const char* hb = host.data();
  // keep this tick's results in the level caches
  if (cached) {
    for (const GGroup& G : gg) {
      LevelCache& C = e->pools[G.pool].cache[G.level];
      uint32_t np = 0;
      memcpy(&np, hb + G.lay.np, 4);
      C.gk = G.k;
      C.gnp = np;
      C.picks.assign(np, 0);
      C.cov.assign(np, 0);
      memcpy(C.picks.data(), hb + G.lay.picks, size_t(np) * 4);
      memcpy(C.cov.data(), hb + G.lay.cov, size_t(np) * 8);
    }
    if (sel_prefix) {
      for (const SGroup& S : sg) {
        LevelCache& C = e->pools[S.pool].cache[S.level];
        C.sK = K_sel;
        C.st = S.t;
        C.topk.assign(size_t(S.t) * K_sel, 0);
        C.dk.assign(K_sel, 0);
        memcpy(C.topk.data(), hb + S.topk, C.topk.size() * 8);
        memcpy(C.dk.data(), hb + S.dk, C.dk.size() * 8);
        bool sat = true;   // every row flat at its end: fewer than K_sel positive values
        for (uint32_t r = 0; r <= S.t && sat; ++r) {
          const int64_t* row = r < S.t ? C.topk.data() + size_t(r) * K_sel : C.dk.data();
          sat = K_sel >= 2 ? row[K_sel - 1] == row[K_sel - 2] : row[0] == 0;
        }
        C.ssat = sat;
      }
    }
  }
  // 5. bounds on the host
  const double t_done = now_s() - e->run_t0;
  for (size_t a = 0; a < act.size(); ++a) {
    EngineQuery& q = e->queries[act[a]];
    EnginePool& p = e->pools[q.pool];
    const uint32_t j = q.level;
    static const LevelCache kNone;
    const LevelCache& C = cached ? p.cache[j] : kNone;
    uint32_t np = 0;
    uint64_t cov = 0;
    const uint32_t* picks_src = nullptr;
    if (cached) {   // greedy from the cache (filled above when it missed)
      np = std::min(C.gnp, q.k);
      if (np) cov = C.cov[np - 1];
      picks_src = C.picks.data();
    } else {
      const GGroup& G = gg[q_gg[a]];
      memcpy(&np, hb + G.lay.np, 4);
      if (np > q.k) np = q.k;   // the first k picks of the shared run
      if (np) memcpy(&cov, hb + G.lay.cov + size_t(np - 1) * 8, 8);
      picks_src = reinterpret_cast<const uint32_t*>(hb + G.lay.picks);
    }
    int64_t sum = 0, dk = 0;
    if (cached && q_sg[a] == ~0u) {   // selection from the cache
      const uint32_t i = std::min(q.k, C.sK) - 1;
      for (uint32_t r = 0; r < q.t; ++r) sum += C.topk[size_t(r) * C.sK + i];
      dk = C.dk[i];
    } else if (sel_prefix) {   // kept above; read from the cache
      const uint32_t i = std::min(q.k, C.sK) - 1;
      for (uint32_t r = 0; r < q.t; ++r) sum += C.topk[size_t(r) * C.sK + i];
      dk = C.dk[i];
    } else {
      const SGroup& S = sg[q_sg[a]];
      for (uint32_t r = 0; r < q.t; ++r) {
        int64_t x;
        memcpy(&x, hb + S.topk + size_t(r) * 8, 8);
        sum += x;
      }
      memcpy(&dk, hb + S.dk, 8);
    }
    const uint64_t m = p.level_m[j];
    const double delta_i = ldexp(q.delta, -static_cast<int>(j + 1));
    centra_bound_out o;
    bound_eval(m, cov, sum, q.t, static_cast<uint64_t>(dk), p.bmax_host[j], q.eps, delta_i, &o);
    q.picks.assign(q.k, 0);
    memcpy(q.picks.data(), picks_src, size_t(np) * 4);
    centra_result& r = q.res;
    r.n_picked = np;
    r.iterations = j + 1;
    r.certified = o.certified;
    r.coverage = cov;
    r.m_final = m;
    r.c_hat = o.c_hat;
    r.amcera = o.amcera;
    r.wimpy = o.wimpy;
    r.xi = o.xi;
    r.nu = o.nu;
    r.rtilde = o.rtilde;
    r.r = o.r;
    r.eta = o.eta;
    const bool last = j + 1 >= p.level_m.size();
    if (o.certified || last) {
      q.state = 2;
      q.rc = o.certified ? CENTRA_OK : CENTRA_NOT_CERTIFIED;
      q.finished = t_done;
      p.active -= 1;
    } else {
      q.level = j + 1;
    }
  }
  const size_t b = engine_bytes(e);
  if (b > e->st.peak_bytes) e->st.peak_bytes = b;
  for (uint32_t pi = 0; pi < e->pools.size(); ++pi) release_levels(e, e->pools[pi], pi);
  return CENTRA_OK;
}

}  // namespace centra

using namespace centra;

extern "C" {

int centra_engine_create(centra_ctx* ctx, size_t hbm_budget_bytes, uint32_t flags, centra_engine** out) {
  if (!ctx) return CENTRA_EINVAL;
  if (!out) return fail(ctx, CENTRA_EINVAL, "engine_create: out is NULL");
  *out = nullptr;
  centra_engine* e = new (std::nothrow) centra_engine();
  if (!e) return fail(ctx, CENTRA_ENOMEM, "engine_create: host allocation");
  e->ctx = ctx;
  e->budget = hbm_budget_bytes;
  e->flags = flags;
  int prev = -1;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(ctx->device);
  hipError_t err = hipStreamCreateWithFlags(&e->cap_stream, hipStreamNonBlocking);
  if (prev >= 0) (void)hipSetDevice(prev);
  if (err != hipSuccess) {
    delete e;
    return hip_fail(ctx, err, "engine_create: stream");
  }
  *out = e;
  return CENTRA_OK;
}

void centra_engine_destroy(centra_engine* e) {
  if (!e) return;
  centra_ctx* ctx = e->ctx;
  (void)hipDeviceSynchronize();
  for (auto& kv : e->graphs) (void)hipGraphExecDestroy(kv.second);
  for (GreedyWs& w : e->ws) {
    DevBuf* wb[] = {&w.gain, &w.covered, &w.part, &w.best, &w.cand};
    for (DevBuf* b : wb) release(ctx, *b);
  }
  for (EnginePool& p : e->pools) {
    DevBuf* bufs[] = {&p.off, &p.nodes, &p.inc, &p.inc_node, &p.seg_off, &p.cursor, &p.sdeg, &p.deg_cur, &p.tiles,
                      &p.words, &p.P, &p.bmax};
    for (DevBuf* b : bufs) release(ctx, *b);
    for (DevBuf& d : p.deg) release(ctx, d);
    for (DevBuf& r : p.R) release(ctx, r);
  }
  DevBuf* bufs[] = {&e->descs, &e->rows, &e->sel_ws, &e->tick_res, &e->round_base, &e->gather};
  for (DevBuf* b : bufs) release(ctx, *b);
  if (e->cap_stream) (void)hipStreamDestroy(e->cap_stream);
  delete e;
}

int centra_engine_add_pool(centra_engine* e, const centra_graph* g, const centra_pool_params* pp, uint32_t* pool_id) {
  if (!e) return CENTRA_EINVAL;
  centra_ctx* ctx = e->ctx;
  if (!g || !pp || !pool_id) return fail(ctx, CENTRA_EINVAL, "engine_add_pool: NULL argument");
  if (pp->t == 0 || pp->t > 1024) return fail(ctx, CENTRA_EINVAL, "engine_add_pool: t outside [1, 1024]");
  if (pp->m_init == 0 || pp->m_max < pp->m_init || pp->m_max >= (1ull << 31))
    return fail(ctx, CENTRA_EINVAL, "engine_add_pool: bad m_init / m_max");
  if (pp->growth_den == 0 || pp->growth_num <= pp->growth_den)
    return fail(ctx, CENTRA_EINVAL, "engine_add_pool: growth must exceed 1");
  EnginePool p;
  p.g = g;
  p.p = *pp;
  for (uint64_t m = pp->m_init;;) {
    p.level_m.push_back(m);
    if (m >= pp->m_max || p.level_m.size() >= kMaxSegments) break;
    const unsigned __int128 geo = (static_cast<unsigned __int128>(m) * pp->growth_num + pp->growth_den - 1) / pp->growth_den;
    m = geo > pp->m_max ? pp->m_max : static_cast<uint64_t>(geo);
  }
  if (p.level_m.back() != pp->m_max)
    return fail(ctx, CENTRA_ENOTSUP, "engine_add_pool: the schedule needs more than 64 levels");
  int prev = -1;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(ctx->device);
  int rc = ensure(ctx, p.off, (pp->m_max + 1) * 8);
  if (!rc) fill_u64(static_cast<uint64_t*>(p.off.ptr), 0, 1, nullptr);
  if (!rc && hipStreamSynchronize(nullptr) != hipSuccess) rc = fail(ctx, CENTRA_EHIP, "engine_add_pool: init");
  if (prev >= 0) (void)hipSetDevice(prev);
  if (rc) {
    release(ctx, p.off);
    return rc;
  }
  e->pools.push_back(std::move(p));
  *pool_id = static_cast<uint32_t>(e->pools.size() - 1);
  return CENTRA_OK;
}

int centra_engine_prefill(centra_engine* e, uint32_t pool_id, uint64_t m, void* stream) {
  if (!e) return CENTRA_EINVAL;
  centra_ctx* ctx = e->ctx;
  if (pool_id >= e->pools.size()) return fail(ctx, CENTRA_EINVAL, "engine_prefill: no such pool");
  EnginePool& p = e->pools[pool_id];
  uint32_t level = 0;
  while (level + 1 < p.level_m.size() && p.level_m[level] < m) ++level;
  int prev = -1;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(ctx->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  int rc = CENTRA_OK;
  if (!e->tuned_block && !(e->flags & CENTRA_ENGINE_NO_TUNE)) rc = autotune(e, s);   // before serving starts
  std::vector<uint32_t> want(e->pools.size(), ~0u);
  want[pool_id] = level;
  if (!rc) rc = sample_pools(e, want, s);
  while (!rc && p.levels_built <= level) rc = build_level(e, p, p.levels_built, s);
  const size_t b = engine_bytes(e);
  if (b > e->st.peak_bytes) e->st.peak_bytes = b;
  if (prev >= 0) (void)hipSetDevice(prev);
  return rc;
}

int centra_engine_submit(centra_engine* e, uint32_t pool_id, uint32_t k, uint32_t t, double eps, double delta,
                         double arrival_s, uint32_t* query_id) {
  if (!e) return CENTRA_EINVAL;
  centra_ctx* ctx = e->ctx;
  const double a = 1.0 - exp(-1.0);
  if (pool_id >= e->pools.size()) return fail(ctx, CENTRA_EINVAL, "engine_submit: no such pool");
  if (k == 0 || t == 0 || t > e->pools[pool_id].p.t) return fail(ctx, CENTRA_EINVAL, "engine_submit: bad k or t");
  if (!(eps > 0.0 && eps < a)) return fail(ctx, CENTRA_EINVAL, "engine_submit: eps outside (0, 1-1/e)");
  if (!(delta > 0.0 && delta < 1.0)) return fail(ctx, CENTRA_EINVAL, "engine_submit: delta outside (0, 1)");
  if (!e->queries.empty() && arrival_s < e->queries.back().arrival)
    return fail(ctx, CENTRA_EINVAL, "engine_submit: arrivals must not decrease");
  if (!query_id) return fail(ctx, CENTRA_EINVAL, "engine_submit: query_id is NULL");
  EngineQuery q;
  q.pool = pool_id;
  q.k = k;
  q.t = t;
  q.eps = eps;
  q.delta = delta;
  q.arrival = arrival_s;
  e->queries.push_back(std::move(q));
  e->pools[pool_id].queued += 1;
  e->pools[pool_id].k_hint = std::max(e->pools[pool_id].k_hint, k);
  *query_id = static_cast<uint32_t>(e->queries.size() - 1);
  return CENTRA_OK;
}

int centra_engine_run(centra_engine* e, int realtime, void* stream) {
  if (!e) return CENTRA_EINVAL;
  centra_ctx* ctx = e->ctx;
  int prev = -1;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(ctx->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  e->run_t0 = now_s();
  int rc = CENTRA_OK;
  for (;;) {
    bool pending = false;
    for (const EngineQuery& q : e->queries) pending |= q.state != 2;
    if (!pending) break;
    const double now = realtime ? now_s() - e->run_t0 : 1e300;
    bool progress = false;
    if ((rc = tick(e, now, &progress, s))) break;
    if (!progress) {
      if (!realtime) {
        rc = fail(ctx, CENTRA_EHIP, "engine_run: no progress");
        break;
      }
      // idle until the next arrival
      double next = 1e300;
      for (const EngineQuery& q : e->queries)
        if (q.state == 0) next = std::min(next, q.arrival);
      const double wait = next - (now_s() - e->run_t0);
      if (wait > 0) std::this_thread::sleep_for(std::chrono::duration<double>(std::min(wait, 0.05)));
    }
  }
  if (prev >= 0) (void)hipSetDevice(prev);
  return rc;
}

int centra_engine_result(centra_engine* e, uint32_t query_id, uint32_t* picks, centra_result* res,
                         centra_query_info* info) {
  if (!e) return CENTRA_EINVAL;
  if (query_id >= e->queries.size()) return fail(e->ctx, CENTRA_EINVAL, "engine_result: no such query");
  const EngineQuery& q = e->queries[query_id];
  if (q.state != 2) return fail(e->ctx, CENTRA_EINVAL, "engine_result: query not finished");
  if (q.rc < 0) return fail(e->ctx, q.rc, "engine_result: the query was refused (its state exceeds the budget)");
  if (picks) memcpy(picks, q.picks.data(), size_t(q.res.n_picked) * 4);
  if (res) *res = q.res;
  if (info) {
    info->arrival_s = q.arrival;
    info->admitted_s = q.admitted;
    info->finished_s = q.finished;
    info->pool = q.pool;
  }
  return q.rc;
}

int centra_engine_stats_get(centra_engine* e, centra_engine_stats* out) {
  if (!e || !out) return CENTRA_EINVAL;
  *out = e->st;
  out->tuned_block = static_cast<uint32_t>(e->tuned_block);
  return CENTRA_OK;
}

const char* centra_engine_log(const centra_engine* e) { return e ? e->log.c_str() : ""; }

}  // extern "C"
