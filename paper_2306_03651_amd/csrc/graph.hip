// Graph preparation: CSR validation and the count bit budget.
#include "common.hpp"
#include "internal.hpp"

namespace centra {

// The splitmix64 output function (Steele, Lea and Flood, "Fast splittable
// pseudorandom number generators", 2014; constants of Stafford's Mix13).
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// One thread per node: row bounds, ascending ids, range, no self loops;
// records the maximum in-degree.  A bad row raises kErrGraph.  With `hash`,
// the sum of mix64(u << 32 | v) over the row's arcs u -> v is added to it.
__global__ void k_validate_rows(uint32_t n, uint64_t n_arcs, const uint32_t* ptr, const uint32_t* idx,
                                uint32_t* flags, uint32_t* max_deg, unsigned long long* hash) {
  const uint32_t u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u == 0 && (ptr[0] != 0 || ptr[n] != n_arcs)) atomicOr(flags, kErrGraph);
  if (u >= n) return;
  const uint32_t b = ptr[u], e = ptr[u + 1];
  if (e < b || e > n_arcs) {
    atomicOr(flags, kErrGraph);
    return;
  }
  uint32_t prev = 0;
  uint64_t h = 0;
  for (uint32_t a = b; a < e; ++a) {
    const uint32_t v = idx[a];
    if (v >= n || v == u || (a > b && v <= prev)) {
      atomicOr(flags, kErrGraph);
      return;
    }
    prev = v;
    h += mix64((uint64_t(u) << 32) | v);
  }
  atomicMax(max_deg, e - b);
  if (hash && h) atomicAdd(hash, static_cast<unsigned long long>(h));
}

// Directed graphs: every arc u -> v must appear as u in v's in-row.  With
// both row sets sorted, duplicate free and of equal total size, this makes
// the reverse CSR exactly the transpose.
__global__ void k_validate_reverse(uint32_t n, const uint32_t* ptr, const uint32_t* idx, const uint32_t* rptr,
                                   const uint32_t* ridx, uint32_t* flags) {
  const uint32_t u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= n) return;
  for (uint32_t a = ptr[u]; a < ptr[u + 1]; ++a) {
    const uint32_t v = idx[a];
    uint32_t lo = rptr[v], hi = rptr[v + 1];
    while (lo < hi) {
      const uint32_t mid = lo + (hi - lo) / 2;
      if (ridx[mid] < u)
        lo = mid + 1;
      else
        hi = mid;
    }
    if (lo >= rptr[v + 1] || ridx[lo] != u) {
      atomicOr(flags, kErrGraph);
      return;
    }
  }
}

// Host side of the graph hash: the arc sum plus mix64 of n | directed << 32.
uint64_t graph_hash_finish(uint32_t n, uint32_t directed, uint64_t arc_sum) {
  uint64_t z = uint64_t(n) | (uint64_t(directed) << 32);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return arc_sum + (z ^ (z >> 31));
}

int validate_graph(centra_ctx* ctx, centra_graph* g, hipStream_t s) {
  uint32_t* flags = ctx->d_flags;
  uint32_t* maxd = ctx->d_flags + 1;
  uint32_t* maxd_in = ctx->d_flags + 2;
  unsigned long long* hash = reinterpret_cast<unsigned long long*>(ctx->d_flags + 4);
  fill_u32(flags, 0, 6, s);
  const unsigned blocks = (g->n + 255) / 256;
  hipLaunchKernelGGL(k_validate_rows, dim3(blocks), dim3(256), 0, s, g->n, g->n_arcs, g->row_ptr, g->col_idx,
                     flags, maxd, hash);
  CENTRA_HIP(ctx, hipGetLastError());
  uint32_t host[3] = {0, 0, 0};
  uint64_t arc_hash = 0;
  CENTRA_HIP(ctx, hipMemcpyAsync(host, ctx->d_flags, sizeof(host), hipMemcpyDeviceToHost, s));
  CENTRA_HIP(ctx, hipMemcpyAsync(&arc_hash, hash, 8, hipMemcpyDeviceToHost, s));
  CENTRA_HIP(ctx, hipStreamSynchronize(s));
  g->hash = graph_hash_finish(g->n, g->directed, arc_hash);
  if (host[0]) {
    fill_u32(flags, 0, 3, s);
    return fail(ctx, CENTRA_EINVAL, "graph: malformed out-CSR (row bounds, order, duplicates, self loops or range)");
  }
  g->max_in_degree = host[1];
  g->max_out_degree = host[1];
  if (g->directed) {
    hipLaunchKernelGGL(k_validate_rows, dim3(blocks), dim3(256), 0, s, g->n, g->n_arcs, g->in_ptr, g->in_idx,
                       flags, maxd_in, static_cast<unsigned long long*>(nullptr));
    CENTRA_HIP(ctx, hipGetLastError());
    CENTRA_HIP(ctx, hipMemcpyAsync(host, ctx->d_flags, sizeof(host), hipMemcpyDeviceToHost, s));
    CENTRA_HIP(ctx, hipStreamSynchronize(s));
    if (host[0]) {
      fill_u32(flags, 0, 3, s);
      return fail(ctx, CENTRA_EINVAL, "graph: malformed reverse CSR");
    }
    hipLaunchKernelGGL(k_validate_reverse, dim3(blocks), dim3(256), 0, s, g->n, g->row_ptr, g->col_idx, g->in_ptr,
                       g->in_idx, flags);
    CENTRA_HIP(ctx, hipGetLastError());
    CENTRA_HIP(ctx, hipMemcpyAsync(host, ctx->d_flags, sizeof(host), hipMemcpyDeviceToHost, s));
    CENTRA_HIP(ctx, hipStreamSynchronize(s));
    if (host[0]) {
      fill_u32(flags, 0, 3, s);
      return fail(ctx, CENTRA_EINVAL, "graph: reverse CSR is not the transpose of the CSR");
    }
    g->max_in_degree = host[2];
  }
  fill_u32(flags, 0, 6, s);
  uint32_t bl = 0;
  for (uint32_t d = g->max_in_degree; d; d >>= 1) ++bl;
  g->count_bits = 63u - bl;
  CENTRA_HIP(ctx, hipStreamSynchronize(s));
  return CENTRA_OK;
}

// ---------------------------------------------------------------------------
// Locality relabelling.  Node v joins the group of its parent p(v), the
// in-neighbour with the largest out-degree (the first such in row order; v
// itself if it has no in-neighbour); groups are laid out in parent-id order,
// members in any order.  The nodes a BFS reaches from one hub then get
// nearby ids, so their 16-byte BFS records, CSR row bounds and rows share
// cache lines.  Rows of the relabelled CSR hold new ids in the caller's
// row order (ascending caller id), which is the order every scan of the
// sampler depends on; sampled nodes are mapped back to caller ids.  So no
// result depends on the permutation, which need not be deterministic.

__global__ void k_parent(uint32_t n, const uint32_t* row_ptr, const uint32_t* in_ptr, const uint32_t* in_idx,
                         uint32_t* par, uint32_t* cnt) {
  const uint32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  uint32_t best = v, bd = 0;
  for (uint32_t a = in_ptr[v]; a < in_ptr[v + 1]; ++a) {
    const uint32_t w = in_idx[a];
    const uint32_t d = row_ptr[w + 1] - row_ptr[w];
    if (d > bd) {
      bd = d;
      best = w;
    }
  }
  par[v] = best;
  atomicAdd(&cnt[best], 1u);
}

__global__ void k_place(uint32_t n, const uint32_t* par, const uint64_t* base, uint32_t* cursor, uint32_t* new_of,
                        uint32_t* orig_of) {
  const uint32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const uint32_t p = par[v];
  const uint32_t nv = static_cast<uint32_t>(base[p]) + atomicAdd(&cursor[p], 1u);
  new_of[v] = nv;
  orig_of[nv] = v;
}

__global__ void k_new_degree(uint32_t n, const uint32_t* ptr, const uint32_t* new_of, uint32_t* ndeg) {
  const uint32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n) ndeg[new_of[v]] = ptr[v + 1] - ptr[v];
}

__global__ void k_narrow(const uint64_t* in, uint32_t* out, uint32_t count) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) out[i] = static_cast<uint32_t>(in[i]);
}

// One wave per row: lanes copy the row's entries, mapped, in row order.
__global__ void k_fill_rows(uint32_t n, const uint32_t* ptr, const uint32_t* idx, const uint32_t* new_of,
                            const uint32_t* nptr, uint32_t* nidx) {
  const uint32_t v = (blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  if (v >= n) return;
  const uint32_t b = ptr[v], e = ptr[v + 1], o = nptr[new_of[v]];
  for (uint32_t a = b + lane_id(); a < e; a += kWave) nidx[o + (a - b)] = new_of[idx[a]];
}

// Relabelled copy of one CSR (ptr, idx) under new_of.
static int relabel_rows(centra_ctx* ctx, uint32_t n, uint64_t n_arcs, const uint32_t* ptr, const uint32_t* idx,
                        const uint32_t* new_of, DevBuf& out_ptr, DevBuf& out_idx, DevBuf& tmp_deg, DevBuf& tmp_scan,
                        hipStream_t s) {
  int rc;
  if ((rc = ensure(ctx, out_ptr, (size_t(n) + 1) * 4, false, s))) return rc;
  if ((rc = ensure(ctx, out_idx, (n_arcs ? n_arcs : 1) * 4, false, s))) return rc;
  uint32_t* ndeg = static_cast<uint32_t*>(tmp_deg.ptr);
  uint64_t* nscan = static_cast<uint64_t*>(tmp_scan.ptr);
  const unsigned blocks = (n + 255) / 256;
  hipLaunchKernelGGL(k_new_degree, dim3(blocks), dim3(256), 0, s, n, ptr, new_of, ndeg);
  CENTRA_HIP(ctx, hipGetLastError());
  if ((rc = excl_scan_u32_to_u64(ctx, ndeg, nscan, n, s))) return rc;
  uint32_t* nptr = static_cast<uint32_t*>(out_ptr.ptr);
  hipLaunchKernelGGL(k_narrow, dim3((n + 1 + 255) / 256), dim3(256), 0, s, nscan, nptr, n + 1);
  const uint64_t threads = uint64_t(n) * kWave;
  hipLaunchKernelGGL(k_fill_rows, dim3(static_cast<unsigned>((threads + 255) / 256)), dim3(256), 0, s, n, ptr, idx,
                     new_of, nptr, static_cast<uint32_t*>(out_idx.ptr));
  CENTRA_HIP(ctx, hipGetLastError());
  return CENTRA_OK;
}

int relabel_graph(centra_ctx* ctx, centra_graph* g, hipStream_t s) {
  const uint32_t n = g->n;
  DevBuf par, cnt, scan;
  int rc = CENTRA_OK;
  do {
    if ((rc = ensure(ctx, par, size_t(n) * 4, false, s))) break;
    if ((rc = ensure(ctx, cnt, size_t(n) * 4, false, s))) break;
    if ((rc = ensure(ctx, scan, (size_t(n) + 1) * 8, false, s))) break;
    if ((rc = ensure(ctx, g->r_new_of, size_t(n) * 4, false, s))) break;
    if ((rc = ensure(ctx, g->r_orig_of, size_t(n) * 4, false, s))) break;
    uint32_t* p = static_cast<uint32_t*>(par.ptr);
    uint32_t* c = static_cast<uint32_t*>(cnt.ptr);
    uint64_t* base = static_cast<uint64_t*>(scan.ptr);
    uint32_t* new_of = static_cast<uint32_t*>(g->r_new_of.ptr);
    const unsigned blocks = (n + 255) / 256;
    fill_u32(c, 0, n, s);
    hipLaunchKernelGGL(k_parent, dim3(blocks), dim3(256), 0, s, n, g->row_ptr, g->in_ptr, g->in_idx, p, c);
    if ((rc = excl_scan_u32_to_u64(ctx, c, base, n, s))) break;
    fill_u32(c, 0, n, s);   // reused as the per-group cursor
    hipLaunchKernelGGL(k_place, dim3(blocks), dim3(256), 0, s, n, p, base, c, new_of,
                       static_cast<uint32_t*>(g->r_orig_of.ptr));
    if (hipGetLastError() != hipSuccess) {
      rc = fail(ctx, CENTRA_EHIP, "graph: relabelling launch failed");
      break;
    }
    // par and scan are reused as the degree and scan scratch of the rows
    if ((rc = relabel_rows(ctx, n, g->n_arcs, g->row_ptr, g->col_idx, new_of, g->r_row_ptr, g->r_col_idx, par,
                           scan, s)))
      break;
    if (g->directed &&
        (rc = relabel_rows(ctx, n, g->n_arcs, g->in_ptr, g->in_idx, new_of, g->r_in_ptr, g->r_in_idx, par, scan, s)))
      break;
    if (hipStreamSynchronize(s) != hipSuccess) {
      rc = fail(ctx, CENTRA_EHIP, "graph: relabelling failed");
      break;
    }
  } while (false);
  release(ctx, par);
  release(ctx, cnt);
  release(ctx, scan);
  if (rc) {
    release_graph_buffers(ctx, g);
    return rc;
  }
  g->bfs_row_ptr = static_cast<const uint32_t*>(g->r_row_ptr.ptr);
  g->bfs_col_idx = static_cast<const uint32_t*>(g->r_col_idx.ptr);
  g->bfs_in_ptr = g->directed ? static_cast<const uint32_t*>(g->r_in_ptr.ptr) : g->bfs_row_ptr;
  g->bfs_in_idx = g->directed ? static_cast<const uint32_t*>(g->r_in_idx.ptr) : g->bfs_col_idx;
  g->new_of = static_cast<const uint32_t*>(g->r_new_of.ptr);
  g->orig_of = static_cast<const uint32_t*>(g->r_orig_of.ptr);
  return CENTRA_OK;
}

void release_graph_buffers(centra_ctx* ctx, centra_graph* g) {
  release(ctx, g->r_row_ptr);
  release(ctx, g->r_col_idx);
  release(ctx, g->r_in_ptr);
  release(ctx, g->r_in_idx);
  release(ctx, g->r_new_of);
  release(ctx, g->r_orig_of);
  release(ctx, g->tri_src);
  release(ctx, g->tri_prefix);
  release(ctx, g->tri_c);
  release(ctx, g->tri_cap);
  release(ctx, g->tri_dir);
  g->tri_list_off = nullptr;
  g->tri_dir_w = 0;
}

}  // namespace centra
