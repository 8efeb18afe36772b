// Sampler interface shared by the kernel file (sample.hip) and its host
// side (sample_launch.hip): the kernel arguments and launch wrappers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace centra {

constexpr uint32_t kPairMax = 65536;   // pairs of the ring tests per slot
constexpr int kLdsBlock = 1024;        // threads of the LDS-bitmap variant
constexpr int kUnroll = 8;             // arcs per thread per expansion round

// One graph's share of a fused launch over several sample pools: the
// graph's arrays and counts, the stream of its samples, and the global
// sample index of its first work item.
struct SampleInst {
  uint32_t n, c_bits, max_out_deg, instance;
  const uint32_t* row_ptr;
  const uint32_t* col_idx;
  const uint32_t* in_ptr;
  const uint32_t* in_idx;
  const uint32_t* new_of;
  const uint32_t* orig_of;
  uint64_t seed;
  uint64_t first;
};

struct SampleArgs {
  uint32_t n;
  uint64_t n_arcs;
  uint32_t c_bits;
  uint32_t max_out_deg;
  const uint32_t* row_ptr;
  const uint32_t* col_idx;
  const uint32_t* in_ptr;
  const uint32_t* in_idx;
  const uint32_t* new_of;    // caller id -> traversal id (NULL: identity)
  const uint32_t* orig_of;   // traversal id -> caller id (NULL: identity)
  uint64_t seed;
  uint32_t instance;
  uint64_t first;
  uint32_t count;
  uint64_t* rec;      // slots * n records of two words: sigma', tag
  uint32_t* q;        // slots * n
  uint64_t* praw;     // slots * kPairMax: raw count of each pair's u from the last cone test
  uint32_t* pinfo;    // slots * 3 * kPairMax: per pair its u, in_ptr[u] and in-degree of u
  uint32_t stamp0;    // stamp of work item 0; item i has stamp0 + i
  uint32_t bit_words;
  uint32_t* work;     // work counter
  uint32_t* stage;    // staging for hyperedge nodes
  uint64_t stage_cap;
  uint64_t* stage_used;
  uint64_t* stage_pos;   // per sample
  uint32_t* he_len;      // per sample
  uint32_t* st_out;      // optional
  uint32_t* dist_out;    // optional
  uint32_t* flags;
  uint64_t* stats;       // [0] arcs scanned, [1] nodes visited (accumulated)
  uint64_t slot_stride;  // nodes per slot in rec and q (>= every graph's n)
  // fused launches only: work items [item_off[j], item_off[j+1]) belong to
  // inst[j], j < n_inst (the fields above then describe no graph)
  const SampleInst* inst;
  const uint32_t* item_off;
  uint32_t n_inst;
  // deferral (single-graph launches only; defer_nodes = 0: none): a BFS
  // about to expand a level of more than defer_nodes nodes, or after
  // scanning more than defer_arcs CSR entries, appends its work item to
  // defer_list (at most defer_cap, counted in *defer_count) and leaves it
  // to the device-wide BFS (wide_sample)
  uint32_t defer_nodes;
  uint64_t defer_arcs;
  uint32_t defer_cap;
  uint32_t* defer_list;
  uint32_t* defer_count;
};

hipError_t sample_kernel_occupancy(int block, bool lds_bits, bool multi, size_t dyn_lds, int* per_cu);
size_t sample_lds_variant_bytes();
void sample_kernel_launch(const SampleArgs& a, int block, bool lds_bits, bool multi, uint32_t grid, size_t dyn_lds,
                          hipStream_t s);
// Device-wide BFS of the deferred work items idx[0..n_items) of a
// single-graph launch (a.first, a.seed, a.instance and the graph as in that
// launch), advanced together: every round expands one level of each live
// sample with the whole GPU (claims and counts pushed, or the level pulled),
// then one synchronisation reads them all; then each backtrack by one
// workgroup, the hyperedges staged like the workgroup kernel's.  Sample j
// uses slot j's records and queue (n_items <= slots) with stamp stamp0 + j
// and ctl[8 j .. 8 j + 8) of device memory (host_ctl: as many words on
// the host).  *arcs receives the CSR entries they scanned.
int wide_samples(const SampleArgs& a, const uint32_t* idx, uint32_t n_items, uint64_t stamp0, uint64_t* ctl,
                 uint64_t* host_ctl, uint64_t* arcs, hipStream_t s);
void stage_gather_launch(uint32_t count, const uint64_t* stage_pos, const uint32_t* he_len, const uint64_t* rel_off,
                         uint64_t base, const uint32_t* stage, uint64_t* he_off, uint32_t* he_nodes, hipStream_t s);

}  // namespace centra
