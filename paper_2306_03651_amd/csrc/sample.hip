// sampleHEs for set betweenness on gfx950.
//
// Each workgroup of a persistent grid owns one BFS slot (level, normalised
// count and visit-queue arrays of n entries in HBM) and takes sample
// indices from an atomic work counter until the batch is exhausted.  One
// sample = pair draw, level-synchronous BFS from s with normalised path
// counts, backtrack of a uniform shortest path from t.  Every quantity the
// output depends on (levels, integer count sums, level maxima, the ordered
// scan of in-neighbours) is independent of thread timing, so the result is
// bit-identical to a sequential implementation.
//
// Level expansion (push): the frontier is processed in chunks of BLOCK
// nodes; their out-degrees are prefix-summed in LDS and every thread takes
// arcs e = tid, tid + BLOCK, ... of the chunk, locating its source by
// binary search in LDS (load balance over skewed degrees; consecutive
// threads read consecutive col_idx entries).  A node is claimed for the next
// level by compare-and-swap on its level word; claimed nodes are appended to
// the visit queue with one LDS atomic per wave (ballot + popcount).  Count
// contributions are 64-bit atomic adds, so their sum is order independent.
//
// Before expanding level L the workgroup checks whether t has an
// in-neighbour at level L; if so d(s,t) = L + 1 and the BFS stops: the
// largest level is never expanded, and the backtrack only needs levels
// <= d - 1, which are complete.
//
// After a sample the workgroup resets exactly the entries it visited, so
// the slot arrays are clean for the next sample without an O(n) clear.
#include "common.hpp"
#include "internal.hpp"

namespace centra {

struct SampleArgs {
  uint32_t n;
  uint32_t c_bits;
  const uint32_t* row_ptr;
  const uint32_t* col_idx;
  const uint32_t* in_ptr;
  const uint32_t* in_idx;
  uint64_t seed;
  uint32_t instance;
  uint64_t first;
  uint32_t count;
  uint32_t* lvl;      // slots * n
  uint64_t* sig;      // slots * n
  uint32_t* q;        // slots * n
  uint32_t* work;     // work counter
  uint32_t* stage;    // staging for hyperedge nodes
  uint64_t stage_cap;
  uint64_t* stage_used;
  uint64_t* stage_pos;   // per sample
  uint32_t* he_len;      // per sample
  uint32_t* st_out;      // optional
  uint32_t* dist_out;    // optional
  uint32_t* flags;
};

template <int BLOCK>
struct SampleShared {
  uint32_t off[BLOCK];
  uint32_t rs[BLOCK];
  uint64_t sg[BLOCK];
  uint32_t scan[BLOCK / kWave + 1];
  uint64_t red[BLOCK / kWave];
  uint32_t qlen;
  uint32_t next;
};

template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_sample_paths(SampleArgs a) {
  __shared__ SampleShared<BLOCK> sh;
  const int tid = threadIdx.x;
  const int lane = lane_id();
  const int wid = tid / kWave;
  const size_t slot = blockIdx.x;
  uint32_t* lvl = a.lvl + slot * a.n;
  uint64_t* sig = a.sig + slot * a.n;
  uint32_t* q = a.q + slot * a.n;
  const uint64_t lane_lt = (1ull << lane) - 1ull;

  for (;;) {
    if (tid == 0) sh.next = atomicAdd(a.work, 1u);
    __syncthreads();
    const uint32_t idx = sh.next;
    __syncthreads();
    if (idx >= a.count) break;
    const uint64_t sample = a.first + idx;

    // pair draw: every thread draws the same words (uniform, no broadcast)
    WordStream st(a.seed, sample, a.instance, 0);
    const uint32_t s = static_cast<uint32_t>(bounded(st, a.n));
    const uint32_t tp = static_cast<uint32_t>(bounded(st, a.n - 1));
    const uint32_t t = tp + (tp >= s ? 1u : 0u);

    if (tid == 0) {
      st_u32(&lvl[s], 0);
      st_u64(&sig[s], 1);
      st_u32(&q[0], s);
      sh.qlen = 1;
    }
    __syncthreads();

    uint32_t lb = 0, le = 1, L = 0, d = kUnseen;
    const uint32_t tb = a.in_ptr[t], te = a.in_ptr[t + 1];
    for (;;) {
      // does t have an in-neighbour at level L?
      int found = 0;
      for (uint32_t e = tb + tid; e < te; e += BLOCK)
        if (ld_u32(&lvl[a.in_idx[e]]) == L) found = 1;
      if (__syncthreads_or(found)) {
        d = L + 1;
        break;
      }
      // expand level L (queue entries [lb, le)) into level L+1
      const uint32_t nl = L + 1;
      for (uint32_t cb = lb; cb < le; cb += BLOCK) {
        const uint32_t i = cb + tid;
        uint32_t deg = 0, rs = 0;
        uint64_t sw = 0;
        if (i < le) {
          const uint32_t w = ld_u32(&q[i]);
          rs = a.row_ptr[w];
          deg = a.row_ptr[w + 1] - rs;
          sw = ld_u64(&sig[w]);
        }
        uint32_t total;
        const uint32_t off = block_excl_scan_u32<BLOCK>(deg, &total, sh.scan);
        sh.off[tid] = off;
        sh.rs[tid] = rs;
        sh.sg[tid] = sw;
        __syncthreads();
        for (uint32_t base = 0; base < total; base += BLOCK) {
          const uint32_t e = base + tid;
          bool claimed = false;
          uint32_t v = 0;
          if (e < total) {
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
            v = a.col_idx[sh.rs[lo] + (e - sh.off[lo])];
            uint32_t lv = ld_u32(&lvl[v]);
            if (lv == kUnseen) {
              const uint32_t old = atomicCAS(&lvl[v], kUnseen, nl);
              if (old == kUnseen) {
                claimed = true;
                lv = nl;
              } else {
                lv = old;
              }
            }
            if (lv == nl) atomicAdd(reinterpret_cast<unsigned long long*>(&sig[v]),
                                    static_cast<unsigned long long>(sh.sg[lo]));
          }
          // wave-aggregated append of newly claimed nodes
          const uint64_t m = __ballot(claimed);
          if (m) {
            uint32_t wbase = 0;
            const int leader = __ffsll(static_cast<unsigned long long>(m)) - 1;
            if (lane == leader) wbase = atomicAdd(&sh.qlen, static_cast<uint32_t>(__popcll(m)));
            wbase = __shfl(wbase, leader, kWave);
            if (claimed) st_u32(&q[wbase + __popcll(m & lane_lt)], v);
          }
        }
        __syncthreads();
      }
      const uint32_t ne = sh.qlen;
      if (ne == le) break;   // nothing new: t unreachable
      // normalise level L+1 (queue entries [le, ne))
      uint64_t mx = 0;
      for (uint32_t i = le + tid; i < ne; i += BLOCK) {
        const uint64_t x = ld_u64(&sig[ld_u32(&q[i])]);
        mx = x > mx ? x : mx;
      }
      mx = block_max_u64<BLOCK>(mx, sh.red);
      const uint32_t bl = bitlen64(mx);
      if (bl > a.c_bits) {
        const uint32_t shift = bl - a.c_bits;
        for (uint32_t i = le + tid; i < ne; i += BLOCK) {
          const uint32_t v = ld_u32(&q[i]);
          const uint64_t x = ld_u64(&sig[v]) >> shift;
          st_u64(&sig[v], x ? x : 1ull);
        }
      }
      __syncthreads();
      lb = le;
      le = ne;
      L = nl;
    }

    // backtrack (wave 0): from v = t, pick a predecessor w at level(v) - 1
    // with probability sigma'_w / W by scanning in-neighbours in ascending
    // order, until level 1.
    const uint32_t len = (d != kUnseen && d >= 2) ? d - 1 : 0u;
    if (wid == 0) {
      uint64_t base = 0;
      if (len) {
        if (lane == 0) base = atomicAdd(reinterpret_cast<unsigned long long*>(a.stage_used),
                                        static_cast<unsigned long long>(len));
        base = shfl_u64(base, 0);
        uint32_t v = t, dv = d;
        uint32_t written = 0;
        while (dv >= 2) {
          const uint32_t want = dv - 1;
          const uint32_t vb = a.in_ptr[v], ve = a.in_ptr[v + 1];
          uint64_t W = 0;
          for (uint32_t cb = vb; cb < ve; cb += kWave) {
            const uint32_t e = cb + lane;
            uint64_t x = 0;
            if (e < ve) {
              const uint32_t w = a.in_idx[e];
              if (ld_u32(&lvl[w]) == want) x = ld_u64(&sig[w]);
            }
            W += wave_sum_u64(x);
          }
          uint32_t pick = kUnseen;
          if (W) {
            const uint64_t r = bounded(st, W);
            uint64_t acc = 0;
            for (uint32_t cb = vb; cb < ve; cb += kWave) {
              const uint32_t e = cb + lane;
              uint64_t x = 0;
              uint32_t w = 0;
              if (e < ve) {
                w = a.in_idx[e];
                if (ld_u32(&lvl[w]) == want) x = ld_u64(&sig[w]);
              }
              const uint64_t incl = acc + wave_incl_scan_u64(x);
              const uint64_t hit = __ballot(incl > r);
              if (hit) {
                pick = __shfl(w, __ffsll(static_cast<unsigned long long>(hit)) - 1, kWave);
                break;
              }
              acc = shfl_u64(incl, kWave - 1);
            }
          }
          if (pick == kUnseen) {
            if (lane == 0) atomicOr(a.flags, kErrBacktrack);
            break;
          }
          if (lane == 0 && base + written < a.stage_cap) a.stage[base + written] = pick;
          ++written;
          v = pick;
          --dv;
        }
      }
      if (lane == 0) {
        a.stage_pos[idx] = base;
        a.he_len[idx] = len;
        if (a.st_out) {
          a.st_out[2 * size_t(idx)] = s;
          a.st_out[2 * size_t(idx) + 1] = t;
        }
        if (a.dist_out) a.dist_out[idx] = d;
      }
    }
    __syncthreads();
    // reset the visited entries of this slot
    const uint32_t nv = sh.qlen;
    for (uint32_t i = tid; i < nv; i += BLOCK) {
      const uint32_t v = ld_u32(&q[i]);
      st_u32(&lvl[v], kUnseen);
      st_u64(&sig[v], 0);
    }
    __syncthreads();
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

constexpr int kSampleBlock = 512;
constexpr uint32_t kMaxSlots = 1024;

static int ensure_slots(centra_ctx* ctx, const centra_graph* g, uint32_t want, hipStream_t s) {
  if (ctx->slots >= want && ctx->slot_n >= g->n) return CENTRA_OK;
  uint32_t slots = want > ctx->slots ? want : ctx->slots;
  const uint32_t n = g->n > ctx->slot_n ? g->n : ctx->slot_n;
  // shrink the slot count if the budget cannot hold all of them
  for (;;) {
    const size_t need = size_t(slots) * n * (4 + 8 + 4);
    const size_t have = ctx->slot_lvl.bytes + ctx->slot_sig.bytes + ctx->slot_q.bytes;
    if (!ctx->budget || ctx->allocated - have + need <= ctx->budget || slots <= 1) break;
    slots /= 2;
  }
  release(ctx, ctx->slot_lvl);
  release(ctx, ctx->slot_sig);
  release(ctx, ctx->slot_q);
  ctx->slots = 0;
  ctx->slot_n = 0;
  int rc;
  if ((rc = ensure(ctx, ctx->slot_lvl, size_t(slots) * n * 4, false, s))) return rc;
  if ((rc = ensure(ctx, ctx->slot_sig, size_t(slots) * n * 8, false, s))) return rc;
  if ((rc = ensure(ctx, ctx->slot_q, size_t(slots) * n * 4, false, s))) return rc;
  fill_u32(static_cast<uint32_t*>(ctx->slot_lvl.ptr), kUnseen, size_t(slots) * n, s);
  fill_u64(static_cast<uint64_t*>(ctx->slot_sig.ptr), 0, size_t(slots) * n, s);
  CENTRA_HIP(ctx, hipGetLastError());
  ctx->slots = slots;
  ctx->slot_n = n;
  return CENTRA_OK;
}

// Concurrent BFS slots: as many workgroups as the device keeps resident.
static uint32_t resident_slots(centra_ctx* ctx) {
  int cus = 0, per_cu = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device) != hipSuccess || cus <= 0)
    cus = 256;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_sample_paths<kSampleBlock>, kSampleBlock, 0) !=
          hipSuccess ||
      per_cu <= 0)
    per_cu = 1;
  (void)hipGetLastError();
  const uint64_t r = uint64_t(cus) * uint64_t(per_cu);
  return r > kMaxSlots ? kMaxSlots : static_cast<uint32_t>(r);
}

int sample_to_stage(centra_ctx* ctx, const centra_graph* g, uint64_t seed, uint32_t instance, uint64_t first,
                    uint32_t count, uint32_t* st_out, uint32_t* dist_out, uint64_t* total, hipStream_t s) {
  int rc;
  *total = 0;
  if (count == 0) return CENTRA_OK;
  const uint32_t resident = resident_slots(ctx);
  uint32_t want = count < resident ? count : resident;
  if ((rc = ensure_slots(ctx, g, want, s))) return rc;
  const uint32_t grid = count < ctx->slots ? count : ctx->slots;
  if ((rc = ensure(ctx, ctx->stage_pos, size_t(count) * 8, false, s))) return rc;
  if ((rc = ensure(ctx, ctx->stage_len, size_t(count) * 4 + 8 + 8 * (size_t(count) + 1), false, s))) return rc;
  if ((rc = ensure(ctx, ctx->work_ctr, 64, false, s))) return rc;
  uint64_t cap = size_t(count) * 8 + 1024;
  if (ctx->stage_nodes.bytes / 4 > cap) cap = ctx->stage_nodes.bytes / 4;
  for (int attempt = 0; attempt < 3; ++attempt) {
    if ((rc = ensure(ctx, ctx->stage_nodes, cap * 4, false, s))) return rc;
    cap = ctx->stage_nodes.bytes / 4;
    uint32_t* work = static_cast<uint32_t*>(ctx->work_ctr.ptr);
    uint64_t* used = reinterpret_cast<uint64_t*>(static_cast<char*>(ctx->work_ctr.ptr) + 8);
    fill_u32(work, 0, 1, s);
    fill_u64(used, 0, 1, s);
    SampleArgs a;
    a.n = g->n;
    a.c_bits = g->count_bits;
    a.row_ptr = g->row_ptr;
    a.col_idx = g->col_idx;
    a.in_ptr = g->in_ptr;
    a.in_idx = g->in_idx;
    a.seed = seed;
    a.instance = instance;
    a.first = first;
    a.count = count;
    a.lvl = static_cast<uint32_t*>(ctx->slot_lvl.ptr);
    a.sig = static_cast<uint64_t*>(ctx->slot_sig.ptr);
    a.q = static_cast<uint32_t*>(ctx->slot_q.ptr);
    a.work = work;
    a.stage = static_cast<uint32_t*>(ctx->stage_nodes.ptr);
    a.stage_cap = cap;
    a.stage_used = used;
    a.stage_pos = static_cast<uint64_t*>(ctx->stage_pos.ptr);
    a.he_len = static_cast<uint32_t*>(ctx->stage_len.ptr);
    a.st_out = st_out;
    a.dist_out = dist_out;
    a.flags = ctx->d_flags;
    hipLaunchKernelGGL(k_sample_paths<kSampleBlock>, dim3(grid), dim3(kSampleBlock), 0, s, a);
    CENTRA_HIP(ctx, hipGetLastError());
    uint64_t host_used = 0;
    CENTRA_HIP(ctx, hipMemcpyAsync(&host_used, used, 8, hipMemcpyDeviceToHost, s));
    CENTRA_HIP(ctx, hipStreamSynchronize(s));
    if ((rc = check_flags(ctx, s, "sample_paths"))) return rc;
    if (host_used <= cap) {
      *total = host_used;
      return CENTRA_OK;
    }
    cap = host_used + 1024;   // staging overflowed: the batch is redrawn identically
  }
  return fail(ctx, CENTRA_EHIP, "sample_paths: staging did not converge");
}

int stage_to_output(centra_ctx* ctx, uint32_t count, uint64_t base, uint64_t* he_off, uint32_t* he_nodes,
                    hipStream_t s) {
  uint32_t* len = static_cast<uint32_t*>(ctx->stage_len.ptr);
  uint64_t* rel = reinterpret_cast<uint64_t*>(static_cast<char*>(ctx->stage_len.ptr) + ((size_t(count) * 4 + 7) & ~size_t(7)));
  int rc = excl_scan_u32_to_u64(ctx, len, rel, count, s);
  if (rc) return rc;
  const unsigned blocks = (count + 1 + 255) / 256;
  hipLaunchKernelGGL(k_stage_gather, dim3(blocks), dim3(256), 0, s, count,
                     static_cast<const uint64_t*>(ctx->stage_pos.ptr), len, rel, base,
                     static_cast<const uint32_t*>(ctx->stage_nodes.ptr), he_off, he_nodes);
  CENTRA_HIP(ctx, hipGetLastError());
  return CENTRA_OK;
}

}  // namespace centra
