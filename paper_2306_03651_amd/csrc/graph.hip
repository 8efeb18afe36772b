// Graph preparation: CSR validation and the count bit budget.
#include "common.hpp"
#include "internal.hpp"

namespace centra {

// One thread per node: row bounds, ascending ids, range, no self loops;
// records the maximum in-degree.  A bad row raises kErrGraph.
__global__ void k_validate_rows(uint32_t n, uint64_t n_arcs, const uint32_t* ptr, const uint32_t* idx,
                                uint32_t* flags, uint32_t* max_deg) {
  const uint32_t u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u == 0 && (ptr[0] != 0 || ptr[n] != n_arcs)) atomicOr(flags, kErrGraph);
  if (u >= n) return;
  const uint32_t b = ptr[u], e = ptr[u + 1];
  if (e < b || e > n_arcs) {
    atomicOr(flags, kErrGraph);
    return;
  }
  uint32_t prev = 0;
  for (uint32_t a = b; a < e; ++a) {
    const uint32_t v = idx[a];
    if (v >= n || v == u || (a > b && v <= prev)) {
      atomicOr(flags, kErrGraph);
      return;
    }
    prev = v;
  }
  atomicMax(max_deg, e - b);
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

int validate_graph(centra_ctx* ctx, centra_graph* g, hipStream_t s) {
  uint32_t* flags = ctx->d_flags;
  uint32_t* maxd = ctx->d_flags + 1;
  uint32_t* maxd_in = ctx->d_flags + 2;
  fill_u32(flags, 0, 3, s);
  const unsigned blocks = (g->n + 255) / 256;
  hipLaunchKernelGGL(k_validate_rows, dim3(blocks), dim3(256), 0, s, g->n, g->n_arcs, g->row_ptr, g->col_idx,
                     flags, maxd);
  CENTRA_HIP(ctx, hipGetLastError());
  uint32_t host[3] = {0, 0, 0};
  CENTRA_HIP(ctx, hipMemcpyAsync(host, ctx->d_flags, sizeof(host), hipMemcpyDeviceToHost, s));
  CENTRA_HIP(ctx, hipStreamSynchronize(s));
  if (host[0]) {
    fill_u32(flags, 0, 3, s);
    return fail(ctx, CENTRA_EINVAL, "graph: malformed out-CSR (row bounds, order, duplicates, self loops or range)");
  }
  g->max_in_degree = host[1];
  g->max_out_degree = host[1];
  if (g->directed) {
    hipLaunchKernelGGL(k_validate_rows, dim3(blocks), dim3(256), 0, s, g->n, g->n_arcs, g->in_ptr, g->in_idx,
                       flags, maxd_in);
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
  fill_u32(flags, 0, 3, s);
  uint32_t bl = 0;
  for (uint32_t d = g->max_in_degree; d; d >>= 1) ++bl;
  g->count_bits = 63u - bl;
  CENTRA_HIP(ctx, hipStreamSynchronize(s));
  return CENTRA_OK;
}

}  // namespace centra
