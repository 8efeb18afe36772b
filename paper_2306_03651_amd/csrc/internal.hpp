// Host-side internals of the CentRA library: context, prepared graph,
// device workspaces and the kernel launchers shared by the entry points.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/centra.h"

namespace centra {

// A device buffer owned by the context; grows on demand within the budget.
struct DevBuf {
  void* ptr = nullptr;
  size_t bytes = 0;
};

}  // namespace centra

struct centra_ctx {
  int device = 0;
  size_t budget = 0;          // 0 = unbounded
  size_t allocated = 0;
  std::string err;
  uint32_t* d_flags = nullptr;   // kernel error bits (u32) + scratch counters
  // per-BFS slot arrays (node records {count, stamp and level}, visit
  // queue, stored pair counts), one set per concurrent BFS, sized for the
  // largest graph
  centra::DevBuf slot_rec, slot_q, slot_praw, slot_pinfo;
  centra::DevBuf wide_ws;   // device-wide BFS: u64 ctl[8] per sample of a group, then the deferred work items
  std::string log;   // one-time choices of the context (slot placement), one line each
  bool placed = false;   // the slot records' placement was searched
  uint32_t slots = 0;
  uint32_t slot_n = 0;
  uint32_t stamp_next = 1;   // BFS stamp of the next sample (records start at stamp 0)
  // slot arrays of the bidirectional sampler (forward and backward records
  // and queues); stamps are shared with the single-source sampler
  centra::DevBuf bi_rec_f, bi_rec_b, bi_q_f, bi_q_b;
  uint32_t bi_slots = 0;
  uint32_t bi_n = 0;
  // sampling staging area
  centra::DevBuf stage_nodes, stage_pos, stage_len, work_ctr, multi_tab;
  // hyperedge entries and samples staged by the context's synchronous
  // launches so far (the first staging size of the next launch follows them)
  uint64_t staged_entries = 0, staged_samples = 0;
  // scan scratch
  centra::DevBuf scan_tmp;
  // incidence (node -> samples) and greedy / AMCERA workspaces
  centra::DevBuf deg, inc_off, inc_cursor, inc, inc_node, gain, covered, best, newcov, seg_deg;
  centra::DevBuf inc_ws;              // workspace of the bucketed incidence build
  uint32_t inc_nseg = 0;              // incidence segments held in inc_off / inc / inc_node
  uint64_t inc_m0 = 0;                // first sample of the newest segment (0: it holds every sample)
  uint64_t inc_m1 = 0;                // samples the incidence covers
  uint64_t inc_span_cap = 0;          // bound on the newest segment's entries (launch shapes)
  uint64_t inc_limit = 0;             // entries inc / inc_node are sized for
  std::vector<uint64_t> inc_seg_m0;   // first sample of each segment
  // State of centra_extend: the incidence is that of the store (ext_off,
  // ext_nodes, ext_cap) over ext_n nodes while ext_inc; the AMCERA counts P,
  // the words and ext_bmax cover samples [0, mc_m) of (mc_seed,
  // mc_instance) with mc_t trials while mc_ok.  Any other build clears them.
  bool ext_inc = false, mc_ok = false;
  const uint64_t* ext_off = nullptr;
  const uint32_t* ext_nodes = nullptr;
  uint64_t ext_cap = 0;
  uint32_t ext_n = 0;
  uint64_t mc_m = 0, mc_seed = 0;
  uint32_t mc_instance = 0, mc_t = 0;
  centra::DevBuf ext_bmax;
  // Builds of the incidence and of the Rademacher words so far; the state a
  // progressive run leaves (store, incidence, counts, running b_max) is
  // continued by a resume on this context only if no other build came since.
  uint64_t inc_gen = 0, words_gen = 0;
  bool prog_ok = false;
  const centra_graph* prog_g = nullptr;
  uint64_t prog_ghash = 0, prog_phash = 0, prog_m = 0, prog_entries = 0, prog_inc_gen = 0, prog_words_gen = 0;
  uint32_t prog_i = 0;
  centra::DevBuf words, P, Rtm, topk_tmp, misc, sel_rows;
  // sample store of centra_progressive
  centra::DevBuf store_off, store_nodes;
  centra::DevBuf kp_len;     // kappa-path walk lengths
  centra::DevBuf kp_stage;   // kappa-path walk nodes, kappa slots per walk
  hipEvent_t ev[8] = {};
  centra_sampler_stats st = {};
};

struct centra_graph {
  centra_ctx* ctx = nullptr;
  uint32_t n = 0;
  uint32_t directed = 0;
  uint64_t n_arcs = 0;
  const uint32_t* row_ptr = nullptr;
  const uint32_t* col_idx = nullptr;
  const uint32_t* in_ptr = nullptr;
  const uint32_t* in_idx = nullptr;
  uint32_t max_in_degree = 0;
  uint32_t max_out_degree = 0;
  uint32_t count_bits = 0;
  uint32_t count_bits_override = 0;   // test override of both count budgets (0: none)
  uint64_t hash = 0;                  // centra_graph_hash
  // the arrays the sampler traverses: the locality-relabelled copy
  // (relabel_graph) or the caller's CSR; new_of / orig_of map caller ids
  // to traversal ids and back (both NULL without relabelling)
  const uint32_t* bfs_row_ptr = nullptr;
  const uint32_t* bfs_col_idx = nullptr;
  const uint32_t* bfs_in_ptr = nullptr;
  const uint32_t* bfs_in_idx = nullptr;
  const uint32_t* new_of = nullptr;
  const uint32_t* orig_of = nullptr;
  centra::DevBuf r_row_ptr, r_col_idx, r_in_ptr, r_in_idx, r_new_of, r_orig_of;
  // triangle index (triangles.hip), built on first use: each arc's source and
  // the exclusive prefix over arcs of their triangle counts
  centra::DevBuf tri_src, tri_prefix, tri_cap, tri_c, tri_dir;
  uint64_t tri_dir_w = 0;   // rank directory bucket width; 0: no directory
  const uint64_t* tri_list_off = nullptr;   // per-arc offsets into tri_c; null: no list
  uint64_t tri_total = ~0ull;   // number of triangles; ~0: not built
};

namespace centra {

// Error helpers: set ctx->err and return a code.
int fail(centra_ctx* ctx, int code, const std::string& msg);
int hip_fail(centra_ctx* ctx, hipError_t e, const char* what);

#define CENTRA_HIP(ctx, call)                                 \
  do {                                                        \
    hipError_t e_ = (call);                                   \
    if (e_ != hipSuccess) return ::centra::hip_fail(ctx, e_, #call); \
  } while (0)

// Ensures `b` holds at least `bytes`; contents are not preserved unless
// `keep` is set.  Respects the context budget.
int ensure(centra_ctx* ctx, DevBuf& b, size_t bytes, bool keep = false, hipStream_t s = nullptr);
void release(centra_ctx* ctx, DevBuf& b);

// Fill kernels (used instead of hipMemsetAsync so the work stays a plain
// kernel sequence).
void fill_u32(uint32_t* p, uint32_t v, size_t n, hipStream_t s);
void fill_u64(uint64_t* p, uint64_t v, size_t n, hipStream_t s);

// Exclusive scan of `n` u32 values into `out[0..n]` (u64, out[n] = total).
int excl_scan_u32_to_u64(centra_ctx* ctx, const uint32_t* in, uint64_t* out, size_t n, hipStream_t s);
// The same with a caller-provided tile buffer of scan_tile_words(n) u64
// (launches only; allocates nothing).
size_t scan_tile_words(size_t n);
void excl_scan_u32_to_u64_ws(const uint32_t* in, uint64_t* out, size_t n, uint64_t* tile_sums, hipStream_t s);

// Locality relabelling of a validated graph (graph.hip); fills the bfs_*
// arrays and the id maps of g.
int relabel_graph(centra_ctx* ctx, centra_graph* g, hipStream_t s);
void release_graph_buffers(centra_ctx* ctx, centra_graph* g);

// Triangle hyperedges (triangles.hip).
int triangle_index(centra_ctx* ctx, centra_graph* g, uint64_t* T, hipStream_t s);
// kappa-path hyperedges: walk lengths -> exclusive offsets off[count + 1]
// (relative); then the walks' nodes at he_nodes + off[x], and base added to
// off.  timed: events ev[4], ev[5] (count) and ev[6], ev[7] (write).
int kpath_count(centra_ctx* ctx, const centra_graph* g, uint32_t kappa, uint64_t seed, uint32_t instance,
                uint64_t first, uint32_t count, uint64_t* off, hipStream_t s, bool timed = false);
int kpath_write(centra_ctx* ctx, const centra_graph* g, uint32_t kappa, uint64_t seed, uint32_t instance,
                uint64_t first, uint32_t count, uint64_t* off, uint64_t base, uint32_t* he_nodes, hipStream_t s,
                bool timed = false);
int sample_triangles_into(centra_ctx* ctx, centra_graph* g, uint64_t seed, uint32_t instance, uint64_t first,
                          uint32_t count, uint64_t* he_off, uint64_t base, uint32_t* he_nodes, hipStream_t s,
                          bool timed = false);   // timed: events ev[4], ev[5] around the launch

// Graph checks (graph.hip).
int validate_graph(centra_ctx* ctx, centra_graph* g, hipStream_t s);
uint64_t graph_hash_finish(uint32_t n, uint32_t directed, uint64_t arc_sum);

// Workspace growth ahead of the stream-ordered calls (each grows the
// buffers its step would grow; keep-contents buffers keep them).
int sample_reserve(centra_ctx* ctx, const centra_graph* g, uint32_t count, uint64_t stage_entries, hipStream_t s);
int incidence_reserve(centra_ctx* ctx, uint32_t n, uint64_t entries, uint32_t segments, hipStream_t s);
int greedy_reserve(centra_ctx* ctx, uint32_t n, uint64_t m, uint32_t k, hipStream_t s);
int mcera_reserve(centra_ctx* ctx, uint32_t n, uint64_t m, uint32_t t, hipStream_t s);

// Stream-ordered sampling into a growing store (sample_launch.hip): samples
// [first, first+count) are appended after the he_off[0] entries already in
// the store (read on the device); *he_total (device) receives the store's
// new size; nodes are written only if it fits he_cap.  No synchronisation.
int sample_append(centra_ctx* ctx, const centra_graph* g, uint64_t seed, uint32_t instance, uint64_t first,
                  uint32_t count, uint64_t* he_off, uint32_t* he_nodes, uint64_t he_cap, uint64_t* he_total,
                  hipStream_t s);

// Sampling (sample.hip): samples [first, first+count) into the staging
// area, then lays them out at `he_off`/`he_nodes` (offsets relative,
// plus `base` added to every offset).  *total receives the node count.
int sample_to_stage(centra_ctx* ctx, const centra_graph* g, uint64_t seed, uint32_t instance,
                    uint64_t first, uint32_t count, uint32_t* st_out, uint32_t* dist_out,
                    uint64_t* total, hipStream_t s);
int stage_to_output(centra_ctx* ctx, uint32_t count, uint64_t base, uint64_t* he_off,
                    uint32_t* he_nodes, hipStream_t s);
// The balanced bidirectional sampler (bidir.hip): samples [first,
// first+count) into the staging area, as sample_to_stage.
int sample_bidir_to_stage(centra_ctx* ctx, const centra_graph* g, uint64_t seed, uint32_t instance,
                          uint64_t first, uint32_t count, uint32_t* st_out, uint32_t* dist_out,
                          uint64_t* total, hipStream_t s);
// A fused sampling launch over several graphs: item i draws samples
// [first, first + count) of (g, seed, instance); the staging area holds
// them item after item.  block: threads per BFS (64, 128, 256 or 512).
struct MultiSampleItem {
  const centra_graph* g;
  uint64_t seed;
  uint32_t instance;
  uint64_t first;
  uint32_t count;
};
int sample_multi_to_stage(centra_ctx* ctx, const MultiSampleItem* items, uint32_t n_items, int block,
                          uint64_t* total, hipStream_t s);

// Incidence + greedy (cover.hip).  Builds deg/inc_off/inc/inc_node in the
// context for a sample of m hyperedges.
// Appends the incidence segment of samples [m0, m1) (m0 = 0 starts a new
// sample: every earlier segment is dropped; so does reaching kMaxSegments,
// and the new segment then holds samples [0, m1)).
constexpr uint32_t kMaxSegments = 64;
// entry_cap: a bound on the store's entries, which sizes the incidence
// without reading the sample's size from the device (no synchronisation);
// ~0 reads the exact size.
int build_incidence(centra_ctx* ctx, uint32_t n, uint64_t m0, uint64_t m1, const uint64_t* he_off,
                    const uint32_t* he_nodes, hipStream_t s, uint64_t entry_cap = ~0ull);
int greedy_on_incidence(centra_ctx* ctx, uint32_t n, uint64_t m, const uint64_t* he_off,
                        const uint32_t* he_nodes, uint32_t k, uint32_t* picks, uint64_t* cov_cum,
                        uint32_t* n_picked, hipStream_t s);

// Greedy cover whose workspaces are carved from a fixed device array of
// kStaticScratchBytes (cover.hip); allocates nothing.  *err receives the
// message of a failure.
constexpr size_t kStaticScratchBytes = CENTRA_NOALLOC_SCRATCH_BYTES;
size_t static_greedy_bytes(uint32_t n, uint64_t m, uint64_t I, uint32_t k);
int greedy_cover_static(uint32_t n, uint64_t m, const uint64_t* he_off, const uint32_t* he_nodes, uint32_t k,
                        uint32_t* picks, uint64_t* cov_cum, uint32_t* n_picked, hipStream_t s, std::string* err);

// Fused greedy of many queries (cover.hip): one descriptor per query, read
// by blockIdx.y.  A query with k = 0 is inactive.
struct GreedyDesc {
  int32_t* gain;            // u32[n] round state
  uint32_t* covered;        // u32[m/32 + 1]
  uint64_t* part;           // u64[greedy_part_words()]
  uint64_t* best;           // u64[k]
  uint64_t* newcov;         // u64[k]
  const uint32_t* deg;      // deg_H over the query's sample
  const uint64_t* seg_off;  // incidence segments (n_seg of n + 1 offsets)
  const uint32_t* inc;
  const uint64_t* he_off;
  const uint32_t* he_nodes;
  uint32_t* picks;          // outputs: u32[k], u64[k], u32[1]
  uint64_t* cov_cum;
  uint32_t* n_picked;
  uint32_t* cand;           // u32[greedy_cand_words()]: candidate list
  uint32_t* cst;            // u32[4]: mode, threshold, list length
  uint32_t* hist;           // u32[greedy_hist_words()]: gain histogram
  uint64_t m;
  uint32_t n, n_seg, k, pad;
};
uint32_t greedy_part_words();
uint32_t greedy_cand_words();
uint32_t greedy_hist_words();
void greedy_multi_init(const GreedyDesc* d, uint32_t n_q, uint32_t max_n, hipStream_t s);
// Launches `rounds` rounds (round numbers round_base[0] .. + rounds - 1),
// then advances round_base[0] by `rounds` on the device.
void greedy_multi_rounds(const GreedyDesc* d, uint32_t n_q, uint32_t max_n, uint32_t cover_grid, uint32_t* round_base,
                         uint32_t rounds, hipStream_t s);
void greedy_multi_finish(const GreedyDesc* d, uint32_t n_q, hipStream_t s);
// Launch-only incidence build of one segment (cover.hip).
void incidence_segment(uint32_t n, uint64_t m0, uint64_t m1, uint64_t span_cap, uint64_t limit, const uint64_t* he_off,
                       const uint32_t* he_nodes, bool first_segment, uint32_t* deg, uint32_t* sdeg, uint64_t* off,
                       uint64_t* cur, uint32_t* inc, uint32_t* inc_node, uint64_t* scan_tiles, uint32_t* flags,
                       hipStream_t s);

// Bucketed build of one incidence segment (incidence.hip): the arguments
// and results of incidence_segment, with no global atomic per entry; ws
// holds incidence_ws_bytes(n, span_cap) bytes.  For n <= kIncBucketMaxNodes.
constexpr uint32_t kIncBucketMaxNodes = 4096u * 2048u;
size_t incidence_ws_bytes(uint32_t n, uint64_t span_cap);
void incidence_segment_bucketed(uint32_t n, uint64_t m0, uint64_t m1, uint64_t span_cap, uint64_t limit,
                                const uint64_t* he_off, const uint32_t* he_nodes, bool first_segment, uint32_t* deg,
                                uint32_t* sdeg, uint64_t* off, uint64_t* cur, uint32_t* inc, uint32_t* inc_node,
                                void* ws, uint32_t* flags, hipStream_t s);

// Top-k sums of many rows at once (mcera.hip): the sum of the k largest
// positive values of each row, written to *out (as i64).
struct SelRow {
  const int32_t* vals;
  uint32_t n, k;
  int64_t* out;
};
size_t select_ws_bytes(uint32_t n_rows);
void select_topk_rows(const SelRow* rows, uint32_t n_rows, uint32_t max_n, void* ws, hipStream_t s);
// Sums of the k largest positive values of every row for every k <= K
// (rows[r].k must be K, K <= kSelPrefixMax): out[r * K + k - 1].
constexpr uint32_t kSelPrefixMax = 2048;
size_t select_prefix_ws_bytes(uint32_t n_rows, uint32_t K);
void select_prefix_rows(const SelRow* rows, uint32_t n_rows, uint32_t max_n, uint32_t K, void* ws, int64_t* out,
                        hipStream_t s);
// Launch-only AMCERA steps (mcera.hip).
void rade_words_launch(uint64_t seed, uint32_t instance, uint64_t s0, uint64_t s1, uint32_t t, uint64_t* words,
                       hipStream_t s);
void rade_count_launch(const uint32_t* inc, const uint32_t* inc_node, const uint64_t* he_off, uint64_t m0, uint64_t m1,
                       uint64_t span_cap, uint64_t limit, const uint64_t* words, uint32_t t, int32_t* P, hipStream_t s);
void rade_finish_launch(const int32_t* P, const uint32_t* deg, uint32_t n, uint32_t t, int32_t* Rtm, hipStream_t s);
void bmax_launch(const uint64_t* he_off, uint64_t m0, uint64_t m1, uint32_t* b_max, hipStream_t s);

// AMCERA (mcera.hip): Rademacher words for samples [s0, s1) into ctx->words
// (Wt words per sample), then the per-trial top-k sums on the incidence.
int rade_words(centra_ctx* ctx, uint64_t seed, uint32_t instance, uint64_t s0, uint64_t s1,
               uint32_t t, hipStream_t s);
// Counts of samples [m0, m) are added to those of the earlier ones, kept
// from the previous call unless m0 is 0; b_max likewise takes the new
// samples' maximum into its previous value.
// m0 must be a segment start of the incidence (normally the newest one's,
// ctx->inc_m0) with P holding the counts of samples [0, m0).
int mcera_on_incidence(centra_ctx* ctx, uint32_t n, uint64_t m, uint64_t m0, const uint64_t* he_off, uint32_t t,
                       uint32_t k, int64_t* topk_sum, uint64_t* deg_topk, uint32_t* b_max,
                       int32_t* R_out, hipStream_t s);

// Theorem bound_dev and the stopping condition (host FP64, api.cpp).
void bound_eval(uint64_t m, uint64_t cov, int64_t sum_topk, uint32_t t, uint64_t deg_topk, uint32_t b_max,
                double eps, double delta_i, centra_bound_out* o);

// Device flag word: read (after synchronising `s`) and clear.
int check_flags(centra_ctx* ctx, hipStream_t s, const char* where);

}  // namespace centra
