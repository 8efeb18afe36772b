// Host side of the single-source path sampler: launch shape, per-BFS slot
// state, the staging area and its redraw on overflow, the layout of the
// staged hyperedges in sample order.  The kernel is in sample.hip.
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <string>
#include <utility>
#include <vector>

#include "common.hpp"
#include "internal.hpp"
#include "sample.hpp"

namespace centra {

// Launch shapes: the LDS-bitmap variant runs one 1024-thread workgroup per
// CU (the bitmap takes most of the LDS); the other variants (Bloom filter in
// LDS, visited state in the HBM records) run several workgroups of 64 to
// 512 threads per CU.
constexpr uint32_t kMaxSlots = 8192;

struct SamplePlan {
  bool lds_bits;
  int block;         // workgroup size of the Bloom-filter variants
  uint32_t bit_words;
  size_t dyn_lds;
  uint32_t resident;   // workgroups resident at once = BFS slots
};

// Variant choice.  Default: the Bloom-filter kernel with 128-thread
// workgroups (many concurrent BFSs per CU hide the latency of the short,
// dependent steps of each BFS).  CENTRA_SAMPLER_VARIANT selects another:
// "lds" (LDS bitmap, 1024 threads, when the bitmap fits), "hbm512",
// "hbm256", "hbm128", "hbm64" (Bloom filter, that many threads).
static SamplePlan plan_for(centra_ctx* ctx, uint32_t n, int block_override = 0) {
  SamplePlan p{};
  p.bit_words = (n + 31) / 32;
  int max_lds = 0, cus = 0;
  if (hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, ctx->device) != hipSuccess)
    max_lds = 65536;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device) != hipSuccess || cus <= 0)
    cus = 256;
  const size_t dyn = size_t(p.bit_words) * 4;
  const char* env = getenv("CENTRA_SAMPLER_VARIANT");
  const char* v = env ? env : "hbm128";
  p.block = 128;
  if (!strcmp(v, "hbm512")) p.block = 512;
  if (!strcmp(v, "hbm256")) p.block = 256;
  if (!strcmp(v, "hbm64")) p.block = 64;
  p.lds_bits = !strcmp(v, "lds") && sample_lds_variant_bytes() + dyn <= size_t(max_lds);
  if (block_override) {   // fused launches: a Bloom-filter variant chosen by the caller
    p.block = block_override;
    p.lds_bits = false;
  }
  int per_cu = 0;
  p.dyn_lds = p.lds_bits ? dyn : 0;
  hipError_t e = sample_kernel_occupancy(p.block, p.lds_bits, block_override != 0, p.dyn_lds, &per_cu);
  if (e != hipSuccess || per_cu <= 0) per_cu = 1;
  (void)hipGetLastError();
  const uint64_t r = uint64_t(cus) * uint64_t(per_cu);
  p.resident = r > kMaxSlots ? kMaxSlots : static_cast<uint32_t>(r);
  return p;
}

// Slot state takes at most half of the device's memory (96 GiB if the size
// cannot be queried); the context budget, when set, limits it further.
static size_t slot_mem_cap() {
  size_t free_b = 0, total_b = 0;
  if (hipMemGetInfo(&free_b, &total_b) != hipSuccess || total_b == 0) {
    (void)hipGetLastError();
    return size_t(96) << 30;
  }
  return total_b / 2;
}

static int ensure_slots(centra_ctx* ctx, uint32_t gn, uint32_t want, hipStream_t s, bool* fresh) {
  *fresh = false;
  const size_t cap_bytes = slot_mem_cap();
  {
    // never ask for more slots than the cap holds
    const size_t per = size_t(gn) * (16 + 4) + kPairMax * (8 + 12);
    const size_t most = cap_bytes / (per ? per : 1);
    if (want > most) want = most ? static_cast<uint32_t>(most) : 1u;
  }
  if (ctx->slots >= want && ctx->slot_n >= gn) return CENTRA_OK;
  // a new allocation is sized for this launch alone: keeping the largest n
  // ever seen with the largest slot count ever asked for would grow the
  // state (and its zero fill) to the memory cap after one large graph
  uint32_t slots = want;
  const uint32_t n = gn;
  const size_t per_slot = size_t(n) * (16 + 4) + kPairMax * (8 + 12);
  // at most the cap of slot state (or the budget, if smaller)
  if (size_t(slots) * per_slot > cap_bytes) slots = static_cast<uint32_t>(cap_bytes / per_slot);
  if (slots == 0) slots = 1;
  // shrink the slot count if the budget cannot hold all of them
  for (;;) {
    const size_t need = size_t(slots) * per_slot;
    const size_t have = ctx->slot_rec.bytes + ctx->slot_q.bytes + ctx->slot_praw.bytes + ctx->slot_pinfo.bytes;
    if (!ctx->budget || ctx->allocated - have + need <= ctx->budget || slots <= 1) break;
    slots /= 2;
  }
  int rc;
  for (;;) {   // halve the slot count while the device cannot hold the state
    release(ctx, ctx->slot_rec);
    release(ctx, ctx->slot_praw);
    release(ctx, ctx->slot_pinfo);
    release(ctx, ctx->slot_q);
    ctx->slots = 0;
    ctx->slot_n = 0;
    rc = ensure(ctx, ctx->slot_rec, size_t(slots) * n * 16, false, s);
    if (!rc) rc = ensure(ctx, ctx->slot_praw, size_t(slots) * kPairMax * 8, false, s);
    if (!rc) rc = ensure(ctx, ctx->slot_pinfo, size_t(slots) * kPairMax * 12, false, s);
    if (!rc) rc = ensure(ctx, ctx->slot_q, size_t(slots) * n * 4, false, s);
    if (rc != CENTRA_ENOMEM || slots <= 64) break;
    slots /= 2;
  }
  if (rc) return rc;
  fill_u64(static_cast<uint64_t*>(ctx->slot_rec.ptr), 0, size_t(slots) * n * 2, s);   // stamp 0: never claimed
  CENTRA_HIP(ctx, hipGetLastError());
  ctx->slots = slots;
  ctx->slot_n = n;
  *fresh = true;
  return CENTRA_OK;
}

// Placement of the slot records.  How fast the sampler runs depends on
// where the allocator put the pages of the per-BFS records: the same launch
// on BA 10^6 takes anywhere from 51 to 61 ms from one allocation of them to
// the next, the same within one allocation to 0.5%, and unchanged when the
// queues or the graph are allocated again.  A short launch ranks
// allocations as the full one does, so fresh records of at least
// kPlaceMinBytes are chosen among kPlaceCandidates allocations by timing
// the batch's first kPlaceProbe work items on each (second of two launches;
// results discarded, stamps used up as by any launch).  It runs for the
// context's first large slot state only (a context that re-allocates as
// its graphs change size would pay the search each time).  The search holds
// two record arrays at a time and stops early if the budget or the device
// cannot, or once a step takes more than kPlaceStepMs of wall time (slow
// probes, or freed memory the device must clear first);
// CENTRA_SLOT_SEARCH=0 turns it off.  It synchronises the stream,
// so stream-ordered launches skip it.
// Wide samples: a BFS about to expand a level of more than kWideNodes
// nodes, or past kWideArcs scanned entries, is left to the device-wide BFS
// (wide_sample in sample.hip); at most kWideCap per launch (the rest finish
// on their workgroups).
constexpr uint32_t kWideNodes = 65536;
constexpr uint64_t kWideArcs = uint64_t(1) << 21;   // about 30 ms of one workgroup's scanning
constexpr uint32_t kWideCap = 4096;
constexpr uint32_t kWideGroup = 64;   // deferred samples advanced together

static bool wide_enabled() {
  const char* e = getenv("CENTRA_WIDE");
  return !(e && !strcmp(e, "0"));
}

// Turns deferral on in `a` (its list in ctx->wide_ws, its counter the u32
// at byte 32 of work_ctr) and clears the counter.
static int defer_args(centra_ctx* ctx, SampleArgs& a, hipStream_t s) {
  int rc;
  if ((rc = ensure(ctx, ctx->wide_ws, size_t(kWideGroup) * 64 + size_t(kWideCap) * 4, false, s))) return rc;
  a.defer_nodes = kWideNodes;
  a.defer_arcs = kWideArcs;
  if (const char* e = getenv("CENTRA_WIDE_NODES")) {   // tests: a lower threshold
    const long v = atol(e);
    if (v >= 1 && v <= 0x7FFFFFFFl) a.defer_nodes = static_cast<uint32_t>(v);
  }
  a.defer_cap = kWideCap;
  a.defer_list = reinterpret_cast<uint32_t*>(static_cast<char*>(ctx->wide_ws.ptr) + size_t(kWideGroup) * 64);
  a.defer_count = reinterpret_cast<uint32_t*>(static_cast<char*>(ctx->work_ctr.ptr) + 32);
  fill_u64(reinterpret_cast<uint64_t*>(a.defer_count), 0, 1, s);
  return CENTRA_OK;
}

constexpr int kPlaceCandidates = 4;
constexpr double kPlaceStepMs = 60.0;   // wall time of one step (allocation, clear, two probes)
constexpr uint32_t kPlaceProbe = 65536;
constexpr size_t kPlaceMinBytes = size_t(4) << 30;

static bool slot_search_enabled() {
  const char* e = getenv("CENTRA_SLOT_SEARCH");
  return !(e && !strcmp(e, "0"));
}

// Sets the per-launch fields of `a` for `count` work items on the current
// slot state and staging area (stage_cap entries).
static void launch_args(centra_ctx* ctx, SampleArgs& a, const SamplePlan& plan, uint32_t count, uint64_t stage_cap) {
  a.stamp0 = ctx->stamp_next;
  ctx->stamp_next += count;
  a.count = count;
  a.slot_stride = ctx->slot_n;
  a.rec = static_cast<uint64_t*>(ctx->slot_rec.ptr);
  a.q = static_cast<uint32_t*>(ctx->slot_q.ptr);
  a.praw = static_cast<uint64_t*>(ctx->slot_praw.ptr);
  a.pinfo = static_cast<uint32_t*>(ctx->slot_pinfo.ptr);
  a.bit_words = plan.bit_words;
  a.work = static_cast<uint32_t*>(ctx->work_ctr.ptr);
  a.stage = static_cast<uint32_t*>(ctx->stage_nodes.ptr);
  a.stage_cap = stage_cap;
  a.stage_used = reinterpret_cast<uint64_t*>(static_cast<char*>(ctx->work_ctr.ptr) + 8);
  a.stage_pos = static_cast<uint64_t*>(ctx->stage_pos.ptr);
  a.he_len = static_cast<uint32_t*>(ctx->stage_len.ptr);
  a.flags = ctx->d_flags;
  a.stats = reinterpret_cast<uint64_t*>(static_cast<char*>(ctx->work_ctr.ptr) + 16);
  a.defer_nodes = 0;
  a.defer_arcs = 0;
  a.defer_cap = 0;
  a.defer_list = nullptr;
  a.defer_count = nullptr;
}

// Stamps: a launch numbers its work items stamp_next, stamp_next + 1, ...;
// before the first launch, and when 32 bits would run out, every record is
// cleared and numbering restarts at 1 (the bidirectional sampler's records
// carry the same stamps).
static void reserve_stamps(centra_ctx* ctx, uint32_t count, hipStream_t s) {
  if (ctx->stamp_next == 0 || uint64_t(ctx->stamp_next) + count > 0xFFFFFFFFull) {
    fill_u64(static_cast<uint64_t*>(ctx->slot_rec.ptr), 0, size_t(ctx->slots) * ctx->slot_n * 2, s);
    if (ctx->bi_rec_f.ptr) {
      fill_u64(static_cast<uint64_t*>(ctx->bi_rec_f.ptr), 0, size_t(ctx->bi_slots) * ctx->bi_n * 2, s);
      fill_u64(static_cast<uint64_t*>(ctx->bi_rec_b.ptr), 0, size_t(ctx->bi_slots) * ctx->bi_n * 2, s);
    }
    ctx->stamp_next = 1;
  }
}

// Times two launches of the first `count` work items on the current slot
// state and returns the second's milliseconds in *ms.
static int probe_slots(centra_ctx* ctx, SampleArgs a, const SamplePlan& plan, bool multi, uint32_t count,
                       hipStream_t s, float* ms) {
  for (int rep = 0; rep < 2; ++rep) {
    reserve_stamps(ctx, count, s);
    fill_u32(static_cast<uint32_t*>(ctx->work_ctr.ptr), 0, 1, s);
    fill_u64(reinterpret_cast<uint64_t*>(static_cast<char*>(ctx->work_ctr.ptr) + 8), 0, 3, s);
    launch_args(ctx, a, plan, count, ctx->stage_nodes.bytes / 4);
    // a flooding sample would hold every probe as long as itself: it is
    // left out, as the timed launches leave it to the device-wide BFS
    int rc;
    if (!multi && !plan.lds_bits && wide_enabled() && (rc = defer_args(ctx, a, s))) return rc;
    const uint32_t grid = count < ctx->slots ? count : ctx->slots;
    CENTRA_HIP(ctx, hipEventRecord(ctx->ev[6], s));
    sample_kernel_launch(a, plan.block, plan.lds_bits, multi, grid, plan.dyn_lds, s);
    CENTRA_HIP(ctx, hipGetLastError());
    CENTRA_HIP(ctx, hipEventRecord(ctx->ev[7], s));
    CENTRA_HIP(ctx, hipStreamSynchronize(s));
    if ((rc = check_flags(ctx, s, "sample_paths (placement probe)"))) return rc;
    if (hipEventElapsedTime(ms, ctx->ev[6], ctx->ev[7]) != hipSuccess) *ms = 0.f;
  }
  return CENTRA_OK;
}

// Chooses the fastest of kPlaceCandidates allocations of the (fresh) slot
// records, by probe_slots.
static int place_slots(centra_ctx* ctx, const SampleArgs& a, const SamplePlan& plan, bool multi, uint32_t count,
                       hipStream_t s) {
  const size_t rec_b = ctx->slot_rec.bytes;
  if (rec_b < kPlaceMinBytes) return CENTRA_OK;
  ctx->placed = true;   // once per context: a later re-allocation keeps what it gets
  const uint32_t pc = count < kPlaceProbe ? count : kPlaceProbe;
  // every slot state held during the search must stay consistent with the
  // stamps: start numbering if nothing has been drawn yet, and skip the
  // search if its launches would run the stamps out (a restart clears only
  // the slot state in use)
  reserve_stamps(ctx, 0, s);
  if (uint64_t(ctx->stamp_next) + uint64_t(2 * kPlaceCandidates) * pc + count > 0xFFFFFFFFull) return CENTRA_OK;
  const auto t0 = std::chrono::steady_clock::now();
  auto since = [](std::chrono::steady_clock::time_point x) {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - x).count();
  };
  float best = 0.f;
  int rc;
  if ((rc = probe_slots(ctx, a, plan, multi, pc, s, &best))) return rc;
  std::string line = "slot placement: " + std::to_string(best);
  // the search stops where it would cost more than it can win: a probe
  // that is slow (long searches) or a step that is (the device clearing
  // freed memory before handing it out again takes seconds for tens of GB)
  bool go = since(t0) <= kPlaceStepMs;
  for (int c = 1; go && c < kPlaceCandidates && best > 0.f; ++c) {
    const auto tc = std::chrono::steady_clock::now();
    if (ctx->budget && ctx->allocated + rec_b > ctx->budget) break;
    void* r2 = nullptr;
    if (hipMalloc(&r2, rec_b) != hipSuccess) {
      (void)hipGetLastError();
      break;
    }
    fill_u64(static_cast<uint64_t*>(r2), 0, rec_b / 8, s);   // stamp 0: never claimed
    std::swap(ctx->slot_rec.ptr, r2);
    float ms = 0.f;
    rc = probe_slots(ctx, a, plan, multi, pc, s, &ms);
    line += " " + std::to_string(ms);
    if (rc || !(ms > 0.f && ms < best)) std::swap(ctx->slot_rec.ptr, r2);   // keep the previous one
    else best = ms;
    (void)hipStreamSynchronize(s);
    (void)hipFree(r2);
    if (rc) return rc;
    go = since(tc) <= kPlaceStepMs;
  }
  const std::string stop = go ? "" : "; stopped: a step took over " + std::to_string(int(kPlaceStepMs)) + " ms";
  const double took = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  ctx->log += line + " ms -> " + std::to_string(best) + " ms (search " + std::to_string(took) + " ms" + stop + ")\n";
  return CENTRA_OK;
}

// Runs one sampling launch of `count` work items into the staging area
// (redrawn with a larger area if it overflows); `a` holds the graph part of
// the arguments (or the instance table of a fused launch), `max_n` the
// largest n of its graphs.  *total receives the staged node count.
// async_cap != 0: stream-ordered form; the staging area holds async_cap
// entries, the launch is not redrawn, nothing is read back (the caller
// learns the size from the device).
static int launch_sampler(centra_ctx* ctx, SampleArgs a, uint32_t count, uint32_t max_n, bool multi, int block,
                          uint64_t* total, hipStream_t s, uint64_t async_cap = 0) {
  int rc;
  *total = 0;
  const SamplePlan plan = plan_for(ctx, max_n, multi ? block : 0);
  uint32_t want = count < plan.resident ? count : plan.resident;
  bool fresh = false;
  if ((rc = ensure_slots(ctx, max_n, want, s, &fresh))) return rc;
  const uint32_t grid = count < ctx->slots ? count : ctx->slots;
  if ((rc = ensure(ctx, ctx->stage_pos, size_t(count) * 8, false, s))) return rc;
  if ((rc = ensure(ctx, ctx->stage_len, size_t(count) * 4 + 8 + 8 * (size_t(count) + 1), false, s))) return rc;
  if ((rc = ensure(ctx, ctx->work_ctr, 64, false, s))) return rc;
  if (fresh && !ctx->placed && !async_cap && slot_search_enabled() && (rc = place_slots(ctx, a, plan, multi, count, s)))
    return rc;
  const uint64_t base_cap = async_cap ? async_cap : size_t(count) * 8 + 1024;
  uint64_t cap = base_cap;
  if (!async_cap && ctx->staged_samples) {
    // entries per sample staged on this context so far, with half again as
    // a margin: an area too small makes the whole launch run twice
    const double per = 1.5 * double(ctx->staged_entries) / double(ctx->staged_samples);
    const uint64_t est = static_cast<uint64_t>(per * double(count)) + 1024;
    if (est > cap) cap = est;
  }
  if (ctx->stage_nodes.bytes / 4 > cap) cap = ctx->stage_nodes.bytes / 4;
  for (int attempt = 0; attempt < 3; ++attempt) {
    rc = ensure(ctx, ctx->stage_nodes, cap * 4, false, s);
    if (rc == CENTRA_ENOMEM && attempt == 0 && cap > base_cap && ctx->stage_nodes.bytes / 4 < cap) {
      cap = base_cap;   // the estimate does not fit the budget: start from the plain size
      rc = ensure(ctx, ctx->stage_nodes, cap * 4, false, s);
    }
    if (rc) return rc;
    cap = ctx->stage_nodes.bytes / 4;
    uint32_t* work = static_cast<uint32_t*>(ctx->work_ctr.ptr);
    uint64_t* used = reinterpret_cast<uint64_t*>(static_cast<char*>(ctx->work_ctr.ptr) + 8);
    fill_u32(work, 0, 1, s);
    fill_u64(used, 0, 1, s);
    reserve_stamps(ctx, count, s);
    launch_args(ctx, a, plan, count, cap);
    const bool wide = !async_cap && !multi && !plan.lds_bits && wide_enabled();
    if (wide && (rc = defer_args(ctx, a, s))) return rc;
    fill_u64(a.stats, 0, 2, s);
    CENTRA_HIP(ctx, hipEventRecord(ctx->ev[6], s));
    sample_kernel_launch(a, plan.block, plan.lds_bits, multi, grid, plan.dyn_lds, s);
    CENTRA_HIP(ctx, hipGetLastError());
    if (async_cap) return CENTRA_OK;
    CENTRA_HIP(ctx, hipEventRecord(ctx->ev[7], s));
    uint64_t host_ctr[5] = {0, 0, 0, 0, 0};   // work, used, arcs, nodes, deferred
    CENTRA_HIP(ctx, hipMemcpyAsync(host_ctr, ctx->work_ctr.ptr, 40, hipMemcpyDeviceToHost, s));
    CENTRA_HIP(ctx, hipStreamSynchronize(s));
    if ((rc = check_flags(ctx, s, "sample_paths"))) return rc;
    const uint32_t n_wide = wide ? static_cast<uint32_t>(std::min<uint64_t>(host_ctr[4] & 0xFFFFFFFFull, kWideCap)) : 0u;
    if (n_wide) {
      // the deferred samples, one device-wide BFS each, on slot 0's state
      std::vector<uint32_t> list(n_wide);
      CENTRA_HIP(ctx, hipMemcpyAsync(list.data(), a.defer_list, size_t(n_wide) * 4, hipMemcpyDeviceToHost, s));
      CENTRA_HIP(ctx, hipStreamSynchronize(s));
      uint64_t* ctl = static_cast<uint64_t*>(ctx->wide_ws.ptr);
      std::vector<uint64_t> host_ctl(size_t(kWideGroup) * 8);
      const auto w0 = std::chrono::steady_clock::now();
      const uint32_t group = std::min<uint32_t>(kWideGroup, ctx->slots);
      for (uint32_t j0 = 0; j0 < n_wide; j0 += group) {   // a group at a time, one slot each
        const uint32_t nj = std::min<uint32_t>(group, n_wide - j0);
        reserve_stamps(ctx, nj, s);
        const uint64_t stamp0 = ctx->stamp_next;
        ctx->stamp_next += nj;
        uint64_t arcs = 0;
        if (wide_samples(a, list.data() + j0, nj, stamp0, ctl, host_ctl.data(), &arcs, s) != CENTRA_OK)
          return hip_fail(ctx, hipGetLastError(), "sample_paths (device-wide BFS)");
        ctx->st.wide_arcs += arcs;
      }
      ctx->st.wide_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - w0).count();
      CENTRA_HIP(ctx, hipMemcpyAsync(&host_ctr[1], static_cast<char*>(ctx->work_ctr.ptr) + 8, 8,
                                     hipMemcpyDeviceToHost, s));
      CENTRA_HIP(ctx, hipStreamSynchronize(s));
      if ((rc = check_flags(ctx, s, "sample_paths (device-wide BFS)"))) return rc;
      ctx->st.wide += n_wide;
    }
    const uint64_t host_used = host_ctr[1];
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, ctx->ev[6], ctx->ev[7]) != hipSuccess) ms = 0.f;
    ctx->st.launches += 1;
    ctx->st.kernel_ms += ms;
    ctx->st.samples += count;
    ctx->st.arcs += host_ctr[2];
    ctx->st.nodes += host_ctr[3];
    ctx->st.hyperedge_nodes += host_used <= cap ? host_used : 0;
    ctx->st.lds_bitmap = plan.lds_bits ? 1 : 0;
    ctx->st.slots = grid;
    if (host_used <= cap) {
      *total = host_used;
      ctx->staged_entries += host_used;
      ctx->staged_samples += count;
      return CENTRA_OK;
    }
    cap = host_used + 1024;   // staging overflowed: the batch is redrawn identically
  }
  return fail(ctx, CENTRA_EHIP, "sample_paths: staging did not converge");
}

int sample_to_stage(centra_ctx* ctx, const centra_graph* g, uint64_t seed, uint32_t instance, uint64_t first,
                    uint32_t count, uint32_t* st_out, uint32_t* dist_out, uint64_t* total, hipStream_t s) {
  *total = 0;
  if (count == 0) return CENTRA_OK;
  SampleArgs a{};
  a.n = g->n;
  a.n_arcs = g->n_arcs;
  a.c_bits = g->count_bits;
  a.max_out_deg = g->max_out_degree;
  a.row_ptr = g->bfs_row_ptr;
  a.col_idx = g->bfs_col_idx;
  a.in_ptr = g->bfs_in_ptr;
  a.in_idx = g->bfs_in_idx;
  a.new_of = g->new_of;
  a.orig_of = g->orig_of;
  a.seed = seed;
  a.instance = instance;
  a.first = first;
  a.st_out = st_out;
  a.dist_out = dist_out;
  return launch_sampler(ctx, a, count, g->n, false, 0, total, s);
}

int sample_multi_to_stage(centra_ctx* ctx, const MultiSampleItem* items, uint32_t n_items, int block,
                          uint64_t* total, hipStream_t s) {
  *total = 0;
  std::vector<SampleInst> tab;
  std::vector<uint32_t> off;
  uint64_t count = 0;
  uint32_t max_n = 0;
  for (uint32_t i = 0; i < n_items; ++i) {
    const MultiSampleItem& it = items[i];
    if (it.count == 0) continue;
    const centra_graph* g = it.g;
    SampleInst x{};
    x.n = g->n;
    x.c_bits = g->count_bits;
    x.max_out_deg = g->max_out_degree;
    x.instance = it.instance;
    x.row_ptr = g->bfs_row_ptr;
    x.col_idx = g->bfs_col_idx;
    x.in_ptr = g->bfs_in_ptr;
    x.in_idx = g->bfs_in_idx;
    x.new_of = g->new_of;
    x.orig_of = g->orig_of;
    x.seed = it.seed;
    x.first = it.first;
    tab.push_back(x);
    off.push_back(static_cast<uint32_t>(count));
    count += it.count;
    if (g->n > max_n) max_n = g->n;
  }
  if (count == 0) return CENTRA_OK;
  if (count >= (1ull << 32)) return fail(ctx, CENTRA_ENOTSUP, "sample_multi: 2^32 work items or more");
  off.push_back(static_cast<uint32_t>(count));
  int rc;
  const size_t tab_bytes = tab.size() * sizeof(SampleInst);
  if ((rc = ensure(ctx, ctx->multi_tab, tab_bytes + off.size() * 4 + 256, false, s))) return rc;
  char* dtab = static_cast<char*>(ctx->multi_tab.ptr);
  const size_t off_at = (tab_bytes + 255) & ~size_t(255);
  CENTRA_HIP(ctx, hipMemcpyAsync(dtab, tab.data(), tab_bytes, hipMemcpyHostToDevice, s));
  CENTRA_HIP(ctx, hipMemcpyAsync(dtab + off_at, off.data(), off.size() * 4, hipMemcpyHostToDevice, s));
  SampleArgs a{};
  a.inst = reinterpret_cast<const SampleInst*>(dtab);
  a.item_off = reinterpret_cast<const uint32_t*>(dtab + off_at);
  a.n_inst = static_cast<uint32_t>(tab.size());
  rc = launch_sampler(ctx, a, static_cast<uint32_t>(count), max_n, true, block, total, s);
  CENTRA_HIP(ctx, hipStreamSynchronize(s));   // the host tables above go out of scope
  return rc;
}

// Lays staged hyperedges out after the base = he_off[0] entries already in
// the store: he_off[i] = base + rel[i] and the nodes at he_nodes + base +
// rel[i] when end = base + rel[count] fits `cap`; otherwise every new
// hyperedge is stored empty (he_off[i] = base, nothing beyond the store
// is referenced) and kErrCapacity is raised.  *total = end either way.
// he_off[0] (rel[0] = 0) is read by every thread and written by none.
__global__ void k_stage_append(uint32_t count, const uint64_t* stage_pos, const uint32_t* he_len, const uint64_t* rel,
                               const uint32_t* stage, uint64_t* he_off, uint32_t* he_nodes, uint64_t cap,
                               uint64_t* total, uint32_t* flags) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i > count) return;
  const uint64_t base = he_off[0];
  const uint64_t end = base + rel[count];
  const bool fits = end <= cap;
  if (i > 0) he_off[i] = fits ? base + rel[i] : base;
  if (i == count) {
    if (total) *total = end;
    if (!fits) atomicOr(flags, kErrCapacity);
    return;
  }
  if (!fits) return;
  const uint64_t p = stage_pos[i];
  const uint64_t o = base + rel[i];
  const uint32_t len = he_len[i];
  for (uint32_t x = 0; x < len; ++x) he_nodes[o + x] = stage[p + x];
}

int sample_reserve(centra_ctx* ctx, const centra_graph* g, uint32_t count, uint64_t stage_entries, hipStream_t s) {
  const SamplePlan plan = plan_for(ctx, g->n);
  const uint32_t want = count < plan.resident ? count : plan.resident;
  int rc;
  bool fresh = false;   // no placement search here: there is no launch to time
  if ((rc = ensure_slots(ctx, g->n, want ? want : 1, s, &fresh))) return rc;
  if ((rc = ensure(ctx, ctx->stage_pos, size_t(count) * 8, false, s))) return rc;
  if ((rc = ensure(ctx, ctx->stage_len, size_t(count) * 4 + 8 + 8 * (size_t(count) + 1), false, s))) return rc;
  if ((rc = ensure(ctx, ctx->work_ctr, 64, false, s))) return rc;
  if ((rc = ensure(ctx, ctx->stage_nodes, (stage_entries ? stage_entries : 1) * 4, false, s))) return rc;
  return ensure(ctx, ctx->scan_tmp, scan_tile_words(count) * 8, false, s);
}

int sample_append(centra_ctx* ctx, const centra_graph* g, uint64_t seed, uint32_t instance, uint64_t first,
                  uint32_t count, uint64_t* he_off, uint32_t* he_nodes, uint64_t he_cap, uint64_t* he_total,
                  hipStream_t s) {
  if (count == 0) return CENTRA_OK;
  SampleArgs a{};
  a.n = g->n;
  a.n_arcs = g->n_arcs;
  a.c_bits = g->count_bits;
  a.max_out_deg = g->max_out_degree;
  a.row_ptr = g->bfs_row_ptr;
  a.col_idx = g->bfs_col_idx;
  a.in_ptr = g->bfs_in_ptr;
  a.in_idx = g->bfs_in_idx;
  a.new_of = g->new_of;
  a.orig_of = g->orig_of;
  a.seed = seed;
  a.instance = instance;
  a.first = first;
  uint64_t total = 0;
  int rc = launch_sampler(ctx, a, count, g->n, false, 0, &total, s, he_cap ? he_cap : 1);
  if (rc) return rc;
  uint32_t* len = static_cast<uint32_t*>(ctx->stage_len.ptr);
  uint64_t* rel = reinterpret_cast<uint64_t*>(static_cast<char*>(ctx->stage_len.ptr) + ((size_t(count) * 4 + 7) & ~size_t(7)));
  if ((rc = excl_scan_u32_to_u64(ctx, len, rel, count, s))) return rc;
  hipLaunchKernelGGL(k_stage_append, dim3((count + 1 + 255) / 256), dim3(256), 0, s, count,
                     static_cast<const uint64_t*>(ctx->stage_pos.ptr), len, rel,
                     static_cast<const uint32_t*>(ctx->stage_nodes.ptr), he_off, he_nodes, he_cap, he_total,
                     ctx->d_flags);
  CENTRA_HIP(ctx, hipGetLastError());
  return CENTRA_OK;
}

int stage_to_output(centra_ctx* ctx, uint32_t count, uint64_t base, uint64_t* he_off, uint32_t* he_nodes,
                    hipStream_t s) {
  uint32_t* len = static_cast<uint32_t*>(ctx->stage_len.ptr);
  uint64_t* rel = reinterpret_cast<uint64_t*>(static_cast<char*>(ctx->stage_len.ptr) + ((size_t(count) * 4 + 7) & ~size_t(7)));
  int rc = excl_scan_u32_to_u64(ctx, len, rel, count, s);
  if (rc) return rc;
  stage_gather_launch(count, static_cast<const uint64_t*>(ctx->stage_pos.ptr), len, rel, base,
                      static_cast<const uint32_t*>(ctx->stage_nodes.ptr), he_off, he_nodes, s);
  CENTRA_HIP(ctx, hipGetLastError());
  return CENTRA_OK;
}

}  // namespace centra
