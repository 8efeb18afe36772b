// The balanced bidirectional path sampler on gfx950 (the sampling procedure
// of Sec. 5): for sample x, a uniform pair s != t from the Philox stream
// (seed, x, instance, tag 7), a search from s over out-arcs and one from t
// over in-arcs, level by level with normalised counts (forward budget from
// the largest in-degree, backward budget from the largest out-degree; a
// level whose largest raw count needs more bits is shifted right and
// clamped to >= 1).  Each step expands the side whose last level has fewer
// arcs to scan (the forward side on ties).  The first new level that meets
// the other side's last level gives d(s,t) = a + b and the meeting set M
// (every shortest path crosses M once).  One node of M is drawn, in
// ascending caller id, with weight sigma_f * sigma_b (the 128-bit product
// shifted so that the weights of M sum below 2^63, clamped to >= 1); the
// path is then walked from it to t over the backward counts (successors in
// row order) and to s over the forward counts (predecessors in row order),
// one draw per step above level 1.  The hyperedge is the path's internal
// nodes, t's neighbour first; it is empty, with no draw after the pair,
// when t is unreachable or adjacent to s.
//
// One workgroup runs one search at a time over a persistent grid, taking
// work items from an atomic counter.  Each side keeps, per slot, records
// {sigma' u64, tag u64} (tag = stamp << 32 | (kUnseen - level), as in the
// single-source sampler, so nothing is reset between samples) and a queue
// of its nodes in level order.  A level is expanded in two passes over its
// arcs: claims (a returning 64-bit atomic max on the target's tag; the
// arrival that sees an older stamp appends the node and zeroes its count),
// then, after a barrier, the count additions of every arc whose target
// carries the new level's tag.  Integer sums and maxima make every count,
// and so every hyperedge, independent of thread timing.
#include <stdlib.h>
#include <string.h>

#include "common.hpp"
#include "internal.hpp"

namespace centra {

namespace {

constexpr int kBiBlock = 256;

struct BiArgs {
  uint32_t n, c_f, c_b;
  const uint32_t* row_ptr;
  const uint32_t* col_idx;
  const uint32_t* in_ptr;
  const uint32_t* in_idx;
  const uint32_t* new_of;
  const uint32_t* orig_of;
  uint64_t seed;
  uint32_t instance;
  uint64_t first;
  uint32_t count;
  uint32_t stamp0;
  uint64_t slot_stride;
  uint64_t* rec_f;   // slots * stride records {sigma, tag}
  uint64_t* rec_b;
  uint32_t* q_f;     // slots * stride
  uint32_t* q_b;
  uint32_t* work;
  uint32_t* stage;
  uint64_t stage_cap;
  uint64_t* stage_used;
  uint64_t* stage_pos;
  uint32_t* he_len;
  uint32_t* st_out;
  uint32_t* dist_out;
  uint32_t* flags;
  uint64_t* stats;   // [0] arcs scanned, [1] nodes given a level
};

struct BiShared {
  uint32_t off[kBiBlock];
  uint32_t rs[kBiBlock];
  uint64_t sg[kBiBlock];
  uint32_t scan[kBiBlock / kWave + 1];
  uint64_t red[kBiBlock / kWave];
  uint32_t next, qadd;
  uint64_t hbase;
};

__device__ __forceinline__ uint64_t* bsig(uint64_t* rec, uint32_t v) { return rec + 2 * size_t(v); }
__device__ __forceinline__ uint64_t* btag(uint64_t* rec, uint32_t v) { return rec + 2 * size_t(v) + 1; }
__device__ __forceinline__ uint64_t blevel_tag(uint64_t base, uint32_t level) { return base + (kUnseen - level); }

__device__ __forceinline__ uint32_t bi_caller(const BiArgs& a, uint32_t v) { return a.orig_of ? a.orig_of[v] : v; }

// Arcs the side's level q[lo, hi) would scan (rows of ptr).
__device__ uint64_t level_cost(const uint32_t* ptr, const uint32_t* q, uint32_t lo, uint32_t hi, BiShared& sh) {
  uint64_t c = 0;
  for (uint32_t i = lo + threadIdx.x; i < hi; i += kBiBlock) {
    const uint32_t u = ld_u32(&q[i]);
    c += ptr[u + 1] - ptr[u];
  }
  return block_sum_u64<kBiBlock>(c, sh.red);
}

// For each arc of the level q[lo, hi) (rows ptr, idx), in chunks of
// kBiBlock sources, calls f(source count slot j, target v) with the chunk's
// sources in sh.rs / sh.off and their counts in sh.sg.  Uniform control
// flow; contains barriers.
template <typename F>
__device__ void for_level_arcs(const uint32_t* ptr, const uint32_t* idx, uint64_t* rec, const uint32_t* q, uint32_t lo,
                               uint32_t hi, bool counts, BiShared& sh, uint64_t& n_arcs, const F& f) {
  for (uint32_t c = lo; c < hi; c += kBiBlock) {
    const uint32_t i = c + threadIdx.x;
    uint32_t deg = 0, rs = 0;
    uint64_t sg = 0;
    if (i < hi) {
      const uint32_t u = ld_u32(&q[i]);
      rs = ptr[u];
      deg = ptr[u + 1] - rs;
      if (counts) sg = ld_u64(bsig(rec, u));
    }
    uint32_t total;
    const uint32_t off = block_excl_scan_u32<kBiBlock>(deg, &total, sh.scan);
    sh.off[threadIdx.x] = off;
    sh.rs[threadIdx.x] = rs;
    sh.sg[threadIdx.x] = sg;
    __syncthreads();
    n_arcs += total;
    for (uint32_t e = threadIdx.x; e < total; e += kBiBlock) {
      // the source of arc e: the last j with off[j] <= e (sources without
      // arcs repeat the next offset)
      int l = 0, h = kBiBlock - 1;
      while (l < h) {
        const int mid = (l + h + 1) >> 1;
        if (sh.off[mid] <= e)
          l = mid;
        else
          h = mid - 1;
      }
      f(l, idx[sh.rs[l] + (e - sh.off[l])]);
    }
    __syncthreads();
  }
}

// Expands the level q[lo, hi) = level L of one side (rows ptr, idx; its
// records rec): level L + 1 is appended at q[hi, new_hi), its counts
// normalised with budget c_bits.  Returns new_hi.
__device__ uint32_t expand_level(const uint32_t* ptr, const uint32_t* idx, uint64_t* rec, uint32_t* q, uint32_t lo,
                                 uint32_t hi, uint64_t base, uint32_t L, uint32_t c_bits, BiShared& sh,
                                 uint64_t& n_arcs) {
  const uint64_t newtag = blevel_tag(base, L + 1);
  if (threadIdx.x == 0) sh.qadd = hi;
  __syncthreads();
  // claims
  for_level_arcs(ptr, idx, rec, q, lo, hi, false, sh, n_arcs, [&](int, uint32_t v) {
    const uint64_t old = atomicMax(reinterpret_cast<unsigned long long*>(btag(rec, v)),
                                   static_cast<unsigned long long>(newtag));
    if (old < base) {   // first arrival of this search
      st_u64(bsig(rec, v), 0);
      st_u32(&q[atomicAdd(&sh.qadd, 1u)], v);
    }
  });
  const uint32_t new_hi = uniform_u32(sh.qadd);
  __syncthreads();
  // counts (the scan pass above is not counted twice)
  uint64_t dummy = 0;
  for_level_arcs(ptr, idx, rec, q, lo, hi, true, sh, dummy, [&](int j, uint32_t v) {
    if (ld_u64(btag(rec, v)) == newtag)
      atomicAdd(reinterpret_cast<unsigned long long*>(bsig(rec, v)), static_cast<unsigned long long>(sh.sg[j]));
  });
  // normalisation of the new level
  uint64_t mx = 0;
  for (uint32_t i = hi + threadIdx.x; i < new_hi; i += kBiBlock) {
    const uint64_t x = ld_u64(bsig(rec, ld_u32(&q[i])));
    mx = x > mx ? x : mx;
  }
  mx = block_max_u64<kBiBlock>(mx, sh.red);
  const uint32_t bl = bitlen64(mx);
  const uint32_t shift = bl > c_bits ? bl - c_bits : 0u;
  if (shift) {
    for (uint32_t i = hi + threadIdx.x; i < new_hi; i += kBiBlock) {
      uint64_t* p = bsig(rec, ld_u32(&q[i]));
      const uint64_t x = ld_u64(p) >> shift;
      st_u64(p, x ? x : 1ull);
    }
    __syncthreads();
  }
  return new_hi;
}

// 128-bit product's bit length, and the scaled weight.
__device__ __forceinline__ uint32_t bitlen128(unsigned __int128 x) {
  const uint64_t hi = static_cast<uint64_t>(x >> 64);
  return hi ? 64u + bitlen64(hi) : bitlen64(static_cast<uint64_t>(x));
}

// The weight of row entry u (0 if u is not on level `want` of the side
// whose records are rec): its count.
__device__ __forceinline__ uint64_t step_weight(uint64_t* rec, uint32_t u, uint64_t want_tag) {
  const uint64_t tg = ld_u64(btag(rec, u));
  const uint64_t c = ld_u64(bsig(rec, u));
  return tg == want_tag ? c : 0ull;
}

// One walk step: among the entries of row [rb, re) of idx on level `want`
// of the side (records rec), the one drawn with weight sigma (in row
// order).  Draws one word (or more, by rejection).
__device__ uint32_t walk_pick(const uint32_t* idx, uint32_t rb, uint32_t re, uint64_t* rec, uint64_t want_tag,
                              WordStream& st, BiShared& sh) {
  uint64_t W = 0;
  for (uint32_t c = rb; c < re; c += kBiBlock) {
    const uint32_t e = c + threadIdx.x;
    W += e < re ? step_weight(rec, idx[e], want_tag) : 0ull;
  }
  W = block_sum_u64<kBiBlock>(W, sh.red);
  if (W == 0) return kUnseen;
  const uint64_t r = bounded(st, W);
  uint64_t run = 0;
  for (uint32_t c = rb; c < re; c += kBiBlock) {
    const uint32_t e = c + threadIdx.x;
    const uint64_t w = e < re ? step_weight(rec, idx[e], want_tag) : 0ull;
    uint64_t tot;
    // inclusive prefix over the chunk (exclusive scan plus own weight)
    uint64_t before = 0;
    {
      const int lane = lane_id(), wid = threadIdx.x / kWave;
      const uint64_t incl = wave_incl_scan_u64(w);
      if (lane == kWave - 1) sh.red[wid] = incl;
      __syncthreads();
      uint64_t off = 0;
      tot = 0;
      for (int i = 0; i < kBiBlock / kWave; ++i) {
        if (i < wid) off += sh.red[i];
        tot += sh.red[i];
      }
      __syncthreads();
      before = off + incl - w;
    }
    tot = uniform_u64(tot);
    if (run + tot > r) {
      const uint64_t lo = run + before;
      const uint32_t cand = (w && lo <= r && r < lo + w) ? e : kUnseen;
      const uint64_t m = block_max_u64<kBiBlock>(cand == kUnseen ? 0ull : uint64_t(cand) + 1, sh.red);
      return m ? idx[static_cast<uint32_t>(m - 1)] : kUnseen;
    }
    run += tot;
  }
  return kUnseen;
}

__global__ __launch_bounds__(kBiBlock) void k_sample_bidir(BiArgs a) {
  __shared__ BiShared sh;
  const int tid = threadIdx.x;
  const size_t slot = blockIdx.x;
  uint64_t* rf = a.rec_f + 2 * slot * a.slot_stride;
  uint64_t* rb = a.rec_b + 2 * slot * a.slot_stride;
  uint32_t* qf = a.q_f + slot * a.slot_stride;
  uint32_t* qb = a.q_b + slot * a.slot_stride;
  uint64_t n_arcs = 0, n_nodes = 0;
  for (;;) {
    if (tid == 0) sh.next = atomicAdd(a.work, 1u);
    __syncthreads();
    const uint32_t idx = uniform_u32(sh.next);
    __syncthreads();
    if (idx >= a.count) break;
    const uint64_t base = uint64_t(a.stamp0 + idx) << 32;
    WordStream st(a.seed, a.first + idx, a.instance, 7);
    const uint32_t s0 = static_cast<uint32_t>(bounded(st, a.n));
    const uint32_t tp = static_cast<uint32_t>(bounded(st, a.n - 1));
    const uint32_t t0 = tp + (tp >= s0 ? 1u : 0u);
    const uint32_t s = a.new_of ? a.new_of[s0] : s0;
    const uint32_t t = a.new_of ? a.new_of[t0] : t0;
    if (tid == 0) {
      st_u64(btag(rf, s), blevel_tag(base, 0));
      st_u64(bsig(rf, s), 1);
      st_u32(&qf[0], s);
      st_u64(btag(rb, t), blevel_tag(base, 0));
      st_u64(bsig(rb, t), 1);
      st_u32(&qb[0], t);
    }
    __syncthreads();
    uint32_t flo = 0, fhi = 1, blo = 0, bhi = 1, da = 0, db = 0, d = kUnseen;
    bool fwd_last = true;
    while (flo < fhi && blo < bhi) {
      const uint64_t cf = level_cost(a.row_ptr, qf, flo, fhi, sh);
      const uint64_t cb = level_cost(a.in_ptr, qb, blo, bhi, sh);
      fwd_last = cf <= cb;
      uint32_t meet = 0;
      if (fwd_last) {
        const uint32_t nh = expand_level(a.row_ptr, a.col_idx, rf, qf, flo, fhi, base, da, a.c_f, sh, n_arcs);
        flo = fhi;
        fhi = nh;
        ++da;
        const uint64_t want = blevel_tag(base, db);
        for (uint32_t i = flo + tid; i < fhi; i += kBiBlock) meet += ld_u64(btag(rb, ld_u32(&qf[i]))) == want;
      } else {
        const uint32_t nh = expand_level(a.in_ptr, a.in_idx, rb, qb, blo, bhi, base, db, a.c_b, sh, n_arcs);
        blo = bhi;
        bhi = nh;
        ++db;
        const uint64_t want = blevel_tag(base, da);
        for (uint32_t i = blo + tid; i < bhi; i += kBiBlock) meet += ld_u64(btag(rf, ld_u32(&qb[i]))) == want;
      }
      if (block_sum_u64<kBiBlock>(meet, sh.red)) {
        d = da + db;
        break;
      }
    }
    n_nodes += fhi + bhi;
    const uint32_t len = (d != kUnseen && d >= 2) ? d - 1 : 0u;
    if (tid == 0)
      sh.hbase = len ? atomicAdd(reinterpret_cast<unsigned long long*>(a.stage_used), static_cast<unsigned long long>(len))
                     : 0ull;
    __syncthreads();
    const uint64_t hbase = uniform_u64(sh.hbase);
    bool ok = true;
    if (len) {
      // the meeting level: the new level of the side expanded last; the
      // other side's records say which of its nodes are in M
      uint32_t* mq = fwd_last ? qf : qb;
      const uint32_t mlo = fwd_last ? flo : blo, mhi = fwd_last ? fhi : bhi;
      uint64_t* mine = fwd_last ? rf : rb;
      uint64_t* other = fwd_last ? rb : rf;
      const uint64_t other_tag = blevel_tag(base, fwd_last ? db : da);
      // |M| and the largest product's bit length
      uint64_t cnt = 0, pb = 0;
      for (uint32_t i = mlo + tid; i < mhi; i += kBiBlock) {
        const uint32_t v = ld_u32(&mq[i]);
        if (ld_u64(btag(other, v)) != other_tag) continue;
        ++cnt;
        const unsigned __int128 p =
            static_cast<unsigned __int128>(ld_u64(bsig(mine, v))) * ld_u64(bsig(other, v));
        const uint64_t b = bitlen128(p);
        pb = b > pb ? b : pb;
      }
      cnt = block_sum_u64<kBiBlock>(cnt, sh.red);
      pb = block_max_u64<kBiBlock>(pb, sh.red);
      const uint32_t room = 63u - bitlen64(cnt);
      const uint32_t shift = pb > room ? static_cast<uint32_t>(pb) - room : 0u;
      auto weight = [&](uint32_t v) -> uint64_t {
        const unsigned __int128 p =
            static_cast<unsigned __int128>(ld_u64(bsig(mine, v))) * ld_u64(bsig(other, v));
        const uint64_t w = static_cast<uint64_t>(p >> shift);
        return w ? w : 1ull;
      };
      uint64_t W = 0;
      for (uint32_t i = mlo + tid; i < mhi; i += kBiBlock) {
        const uint32_t v = ld_u32(&mq[i]);
        if (ld_u64(btag(other, v)) == other_tag) W += weight(v);
      }
      W = block_sum_u64<kBiBlock>(W, sh.red);
      const uint64_t r = bounded(st, W);
      // the first meeting node in ascending caller id whose weight prefix
      // exceeds r: a search over the caller ids, each step one pass over M
      uint32_t lo = 0, hi = a.n - 1;
      while (lo < hi) {
        const uint32_t mid = lo + (hi - lo) / 2;
        uint64_t sum = 0;
        for (uint32_t i = mlo + tid; i < mhi; i += kBiBlock) {
          const uint32_t v = ld_u32(&mq[i]);
          if (ld_u64(btag(other, v)) == other_tag && bi_caller(a, v) <= mid) sum += weight(v);
        }
        sum = block_sum_u64<kBiBlock>(sum, sh.red);
        if (sum > r)
          hi = mid;
        else
          lo = mid + 1;
      }
      const uint32_t vm = a.new_of ? a.new_of[lo] : lo;
      // toward t over the backward counts: successors on out-rows; the node
      // at backward level j goes to position j - 1
      uint32_t cur = vm;
      for (uint32_t j = db; j >= 2; --j) {
        cur = walk_pick(a.col_idx, a.row_ptr[cur], a.row_ptr[cur + 1], rb, blevel_tag(base, j - 1), st, sh);
        if (cur == kUnseen) {
          ok = false;
          break;
        }
        if (tid == 0 && hbase + (j - 2) < a.stage_cap) a.stage[hbase + (j - 2)] = bi_caller(a, cur);
      }
      if (ok && da >= 1 && db >= 1 && tid == 0 && hbase + (db - 1) < a.stage_cap)
        a.stage[hbase + (db - 1)] = lo;
      // toward s over the forward counts: predecessors on in-rows; the node
      // at forward level i goes to position d - 1 - i
      cur = vm;
      for (uint32_t i = da; ok && i >= 2; --i) {
        cur = walk_pick(a.in_idx, a.in_ptr[cur], a.in_ptr[cur + 1], rf, blevel_tag(base, i - 1), st, sh);
        if (cur == kUnseen) {
          ok = false;
          break;
        }
        if (tid == 0 && hbase + (d - i) < a.stage_cap) a.stage[hbase + (d - i)] = bi_caller(a, cur);
      }
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
    __syncthreads();
  }
  if (tid == 0 && a.stats && n_arcs) {
    atomicAdd(reinterpret_cast<unsigned long long*>(&a.stats[0]), static_cast<unsigned long long>(n_arcs));
    atomicAdd(reinterpret_cast<unsigned long long*>(&a.stats[1]), static_cast<unsigned long long>(n_nodes));
  }
}

unsigned grid_cap(uint64_t want, uint32_t cap) { return static_cast<unsigned>(want < cap ? want : cap); }

}  // namespace

// Slot arrays of the bidirectional sampler: forward and backward records
// and queues, 40 bytes per node per slot, at most half of the device's
// memory (the context budget can lower that).
static int ensure_bidir_slots(centra_ctx* ctx, uint32_t n, uint32_t want, hipStream_t s) {
  size_t free_b = 0, total_b = 0;
  if (hipMemGetInfo(&free_b, &total_b) != hipSuccess || total_b == 0) {
    (void)hipGetLastError();
    total_b = size_t(192) << 30;
  }
  const size_t per = size_t(n) * 40;
  size_t most = (total_b / 2) / (per ? per : 1);
  if (most == 0) most = 1;
  if (want > most) want = static_cast<uint32_t>(most);
  if (ctx->bi_slots >= want && ctx->bi_n >= n) return CENTRA_OK;
  uint32_t slots = want;   // sized for this launch alone (see ensure_slots)
  const uint32_t nn = n;
  for (;;) {
    const size_t need = size_t(slots) * nn * 40;
    const size_t have = ctx->bi_rec_f.bytes + ctx->bi_rec_b.bytes + ctx->bi_q_f.bytes + ctx->bi_q_b.bytes;
    if (!ctx->budget || ctx->allocated - have + need <= ctx->budget || slots <= 1) break;
    slots /= 2;
  }
  release(ctx, ctx->bi_rec_f);
  release(ctx, ctx->bi_rec_b);
  release(ctx, ctx->bi_q_f);
  release(ctx, ctx->bi_q_b);
  ctx->bi_slots = 0;
  ctx->bi_n = 0;
  int rc;
  if ((rc = ensure(ctx, ctx->bi_rec_f, size_t(slots) * nn * 16, false, s))) return rc;
  if ((rc = ensure(ctx, ctx->bi_rec_b, size_t(slots) * nn * 16, false, s))) return rc;
  if ((rc = ensure(ctx, ctx->bi_q_f, size_t(slots) * nn * 4, false, s))) return rc;
  if ((rc = ensure(ctx, ctx->bi_q_b, size_t(slots) * nn * 4, false, s))) return rc;
  fill_u64(static_cast<uint64_t*>(ctx->bi_rec_f.ptr), 0, size_t(slots) * nn * 2, s);   // stamp 0: never claimed
  fill_u64(static_cast<uint64_t*>(ctx->bi_rec_b.ptr), 0, size_t(slots) * nn * 2, s);
  CENTRA_HIP(ctx, hipGetLastError());
  ctx->bi_slots = slots;
  ctx->bi_n = nn;
  return CENTRA_OK;
}

int sample_bidir_to_stage(centra_ctx* ctx, const centra_graph* g, uint64_t seed, uint32_t instance, uint64_t first,
                          uint32_t count, uint32_t* st_out, uint32_t* dist_out, uint64_t* total, hipStream_t s) {
  int rc;
  *total = 0;
  if (count == 0) return CENTRA_OK;
  int per_cu = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_sample_bidir, kBiBlock, 0) != hipSuccess || per_cu <= 0)
    per_cu = 1;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device) != hipSuccess || cus <= 0)
    cus = 256;
  (void)hipGetLastError();
  const uint64_t resident = uint64_t(cus) * per_cu;
  if ((rc = ensure_bidir_slots(ctx, g->n, grid_cap(count < resident ? count : resident, 8192), s))) return rc;
  const uint32_t grid = count < ctx->bi_slots ? count : ctx->bi_slots;
  if ((rc = ensure(ctx, ctx->stage_pos, size_t(count) * 8, false, s))) return rc;
  if ((rc = ensure(ctx, ctx->stage_len, size_t(count) * 4 + 8 + 8 * (size_t(count) + 1), false, s))) return rc;
  if ((rc = ensure(ctx, ctx->work_ctr, 64, false, s))) return rc;
  uint64_t cap = size_t(count) * 8 + 1024;
  if (ctx->stage_nodes.bytes / 4 > cap) cap = ctx->stage_nodes.bytes / 4;
  // the count budgets: forward sums run over in-neighbours, backward sums
  // over out-neighbours (a test override lowers both)
  const uint32_t c_f = g->count_bits;
  uint32_t c_b = 63u - (g->max_out_degree ? 32u - static_cast<uint32_t>(__builtin_clz(g->max_out_degree)) : 0u);
  if (g->count_bits_override && g->count_bits_override < c_b) c_b = g->count_bits_override;
  for (int attempt = 0; attempt < 3; ++attempt) {
    if ((rc = ensure(ctx, ctx->stage_nodes, cap * 4, false, s))) return rc;
    cap = ctx->stage_nodes.bytes / 4;
    uint32_t* work = static_cast<uint32_t*>(ctx->work_ctr.ptr);
    uint64_t* used = reinterpret_cast<uint64_t*>(static_cast<char*>(ctx->work_ctr.ptr) + 8);
    fill_u32(work, 0, 1, s);
    fill_u64(used, 0, 1, s);
    if (ctx->stamp_next == 0 || uint64_t(ctx->stamp_next) + count > 0xFFFFFFFFull) {
      // 32-bit stamps would run out: clear every record of both samplers
      fill_u64(static_cast<uint64_t*>(ctx->bi_rec_f.ptr), 0, size_t(ctx->bi_slots) * ctx->bi_n * 2, s);
      fill_u64(static_cast<uint64_t*>(ctx->bi_rec_b.ptr), 0, size_t(ctx->bi_slots) * ctx->bi_n * 2, s);
      if (ctx->slot_rec.ptr)
        fill_u64(static_cast<uint64_t*>(ctx->slot_rec.ptr), 0, size_t(ctx->slots) * ctx->slot_n * 2, s);
      ctx->stamp_next = 1;
    }
    BiArgs a{};
    a.n = g->n;
    a.c_f = c_f;
    a.c_b = c_b;
    a.row_ptr = g->bfs_row_ptr;
    a.col_idx = g->bfs_col_idx;
    a.in_ptr = g->bfs_in_ptr;
    a.in_idx = g->bfs_in_idx;
    a.new_of = g->new_of;
    a.orig_of = g->orig_of;
    a.seed = seed;
    a.instance = instance;
    a.first = first;
    a.count = count;
    a.stamp0 = ctx->stamp_next;
    ctx->stamp_next += count;
    a.slot_stride = ctx->bi_n;
    a.rec_f = static_cast<uint64_t*>(ctx->bi_rec_f.ptr);
    a.rec_b = static_cast<uint64_t*>(ctx->bi_rec_b.ptr);
    a.q_f = static_cast<uint32_t*>(ctx->bi_q_f.ptr);
    a.q_b = static_cast<uint32_t*>(ctx->bi_q_b.ptr);
    a.work = work;
    a.stage = static_cast<uint32_t*>(ctx->stage_nodes.ptr);
    a.stage_cap = cap;
    a.stage_used = used;
    a.stage_pos = static_cast<uint64_t*>(ctx->stage_pos.ptr);
    a.he_len = static_cast<uint32_t*>(ctx->stage_len.ptr);
    a.st_out = st_out;
    a.dist_out = dist_out;
    a.flags = ctx->d_flags;
    a.stats = reinterpret_cast<uint64_t*>(static_cast<char*>(ctx->work_ctr.ptr) + 16);
    fill_u64(a.stats, 0, 2, s);
    CENTRA_HIP(ctx, hipEventRecord(ctx->ev[6], s));
    hipLaunchKernelGGL(k_sample_bidir, dim3(grid), dim3(kBiBlock), 0, s, a);
    CENTRA_HIP(ctx, hipGetLastError());
    CENTRA_HIP(ctx, hipEventRecord(ctx->ev[7], s));
    uint64_t host_ctr[4] = {0, 0, 0, 0};
    CENTRA_HIP(ctx, hipMemcpyAsync(host_ctr, ctx->work_ctr.ptr, 32, hipMemcpyDeviceToHost, s));
    CENTRA_HIP(ctx, hipStreamSynchronize(s));
    if ((rc = check_flags(ctx, s, "sample_paths_bidir"))) return rc;
    const uint64_t host_used = host_ctr[1];
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, ctx->ev[6], ctx->ev[7]) != hipSuccess) ms = 0.f;
    ctx->st.launches += 1;
    ctx->st.kernel_ms += ms;
    ctx->st.samples += count;
    ctx->st.arcs += host_ctr[2];
    ctx->st.nodes += host_ctr[3];
    ctx->st.hyperedge_nodes += host_used <= cap ? host_used : 0;
    ctx->st.lds_bitmap = 0;
    ctx->st.slots = grid;
    if (host_used <= cap) {
      *total = host_used;
      return CENTRA_OK;
    }
    cap = host_used + 1024;   // staging overflowed: the batch is redrawn identically
  }
  return fail(ctx, CENTRA_EHIP, "sample_paths_bidir: staging did not converge");
}

}  // namespace centra
