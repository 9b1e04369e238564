// Host-side context of the library (the opaque ksg_ctx of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <string>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "../../include/ksgcmi.h"
#include "internal.h"

namespace ksg {

// A roctx range for the profiler's marker trace (rocprofv3 --marker-trace): pushed on
// construction, popped on destruction.  Without a profiler attached the calls do nothing.
struct TraceRange {
  explicit TraceRange(const char* name) { roctxRangePushA(name); }
  ~TraceRange() { roctxRangePop(); }
  TraceRange(const TraceRange&) = delete;
  TraceRange& operator=(const TraceRange&) = delete;
};

// A grow-only device allocation owned by the context.
struct DevBuf {
  void* ptr = nullptr;
  size_t cap = 0;
};

// One CMI problem in the engine's own form: one pointer per dimension (X..., Y..., Z...),
// an optional row gather per dimension, and whether the column is already a +inf-padded
// device column (then it is used in place unless gathered).
struct Problem {
  int64_t n;
  int dx, dy, dz, k;
  const float* col[kMaxDims];
  const int32_t* perm[kMaxDims];
  bool padded[kMaxDims];
  float* eps_out;
  int32_t* counts_out;
  double* local_out;
  int out_index;
};

// The host plan of one batch (batch.hip): descriptors, work items, pack jobs and the launch
// layout, in the order the upload writes them.
struct BatchPlan {
  struct Segment {
    int D, kp, off, count;
    double cost;  // brute-force operations of its problems (launch scheduling)
  };
  struct Chunk {
    std::array<int, 3> cls;       // m, G, KP
    std::vector<WorkItem> items;  // radius and X count launches (same items)
    size_t item_off = 0;
    size_t ydesc_off = 0, n_ydesc = 0;
    size_t yitem_off = 0, n_yitems = 0;
  };
  int np = 0;
  std::vector<ProbDesc> descs;
  std::vector<GroupDesc> gdescs;
  std::vector<YZDesc> ydescs;
  std::vector<WorkItem> items;   // ungrouped items: brute force (or algorithm-2 segments), windows, wide
  std::vector<WorkItem> yitems;  // Y/Z count items of every chunk
  std::vector<Chunk> chunks;
  std::vector<PackJob> jobs;     // pool columns (destinations resolved)
  std::vector<PackJob> inplace;  // in-place columns, for the finite check
  std::vector<Segment> segments, wsegments;
  Segment wide_seg{0, 5, 0, 0, 0.0};
  std::vector<std::pair<const float*, int64_t>> wsets;  // window sets: (key column, N)
  std::vector<int64_t> wsigma_off;                      // their key orders in the pool
  int n_plain_items = 0;
  double plain_cost = 0.0;
  int common_shape = -2;
  int kp = 5;
  int max_pad = 0;
  int parts = 0;
  int64_t chunk_elems_max = 0;
  size_t n_gitems = 0;
  float* pool_base = nullptr;
  double brute_ops = 0.0;
  int64_t n_groups = 0;
  int tile_q_plain = kTileQ, tile_q_wide = kTileQ;  // brute-force launches' tile heights
  size_t desc_bytes() const;
  size_t item_count() const;
};

// A captured batch: the instantiated graph, the key it was captured for and its private copies
// of the descriptors, work items and pack jobs.
struct GraphEntry {
  std::vector<uint64_t> key;
  uint64_t hash = 0;
  uint64_t gen = 0;  // buffer generation at capture
  uint64_t last_use = 0;
  hipGraphExec_t exec = nullptr;
  DevBuf desc, items, jobs;
  int64_t n_items = 0, n_groups = 0;
};

// Grouped launches run in chunks of at most this many E / T elements (KSG_OPT_GROUP_CHUNK).
constexpr int64_t kGroupChunkElems = int64_t(1) << 27;

}  // namespace ksg

void ksg_build_harmonic(int64_t nmax, double* out);

// Return a ksg_status from the enclosing function when a HIP call fails.
#define KSG_HIP(ctx, expr)                                   \
  do {                                                       \
    hipError_t e_ = (expr);                                  \
    if (e_ != hipSuccess) return (ctx)->hip_fail(e_, #expr); \
  } while (0)


struct ksg_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  int cus = 0;
  char arch[64] = {0};
  std::string err;

  bool check_finite = true;
  int64_t mem_limit = 0;         // KSG_OPT_MEM_LIMIT: bytes of workspace the context may hold (0 = any)
  size_t mem_held = 0;           // bytes of workspace held now
  int group_size = -1;           // -1: tuned per conditioning dimension, 0: no grouping, 8 or 16
  int algorithm = 1;             // KSG algorithm of every estimate: 1 or 2
  bool use_windows = true;       // key-ordered window search for eligible single problems
  bool windows_untuned = false;  // KSG_OPT_WINDOWS = 2: from N = 2048 whatever the tuner found
  int tuned_g[2][15] = {{0}};    // [k <= 4 ? 0 : 1][m]: group size picked by the autotuner (0 = default)
  // autotuned launch shapes (ksg_autotune), used once `tuned` is set:
  int tuned_tq[2] = {0, 0};      // brute-force tile height for launches of few / many work-groups
  int tuned_win_n[ksg::kMaxDimsCompiled + 1] = {0};  // [D]: smallest N searched with windows
  bool tuned = false;
  int tile_q = 0;                // KSG_OPT_TILE_Q: 0 = tuned (256 before tuning), or 64/128/256
  bool use_graph = false;        // KSG_OPT_USE_GRAPH: capture batches into HIP graphs and replay them
  int64_t group_chunk_elems = 0; // KSG_OPT_GROUP_CHUNK: 0 = kGroupChunkElems

  ksg::DevBuf htab, pool, desc, items, partials, jobs, tmp, embed, cmi, aux, feat;
  ksg::DevBuf ebuf, tbuf;  // grouped search: radii E (FP32) and Y/Z count terms T (FP64)
  int64_t htab_n = 0;
  int* d_counter = nullptr;  // [1]: finite / permutation-range flag
  int* d_flag = nullptr;
  ksg::MaxStatOut* d_ms = nullptr;
  ksg::MaxStatOut* h_ms = nullptr;  // pinned

  // Auxiliary streams (default priority) on which the single-problem search launches of one
  // batch run side by side (one launch per column count or shape): forked from and joined
  // back to `stream` through events, created on first use.
  static constexpr int kAuxStreams = 3;
  hipStream_t aux_streams[kAuxStreams] = {};
  hipEvent_t fork_ev = nullptr;
  hipEvent_t join_ev[kAuxStreams] = {};
  int ensure_aux_streams();

  void* staging = nullptr;  // pinned upload block
  size_t staging_cap = 0;
  hipEvent_t staging_done = nullptr;
  bool staging_pending = false;

  int64_t last_items = 0;
  int64_t last_groups = 0;
  // smallest N from which single problems of D columns use the key-ordered window search
  int window_min_n(int D) const {
    if (!tuned || windows_untuned || D < 3 || D > ksg::kMaxDimsCompiled || tuned_win_n[D] <= 0) return ksg::kWindowMinN;
    return std::max(ksg::kWindowMinN, tuned_win_n[D]);
  }
  // tile height of a brute-force launch of tiles256 tiles of 256 queries
  int brute_tile_q(int64_t tiles256) const {
    if (tile_q) return tile_q;
    if (!tuned) return ksg::kTileQ;
    const int t = tuned_tq[tiles256 < 4 * (int64_t)cus ? 0 : 1];
    return t ? t : ksg::kTileQ;
  }
  int tuned_group_size(int m, int k) const {
    if (m > ksg::kGroupMaxM16) return 8;  // only groups of 8 are compiled for m > 14
    const int t = tuned_g[k <= 4 ? 0 : 1][m];
    return t ? t : 8;
  }
  static double algorithmic_ops(const ksg::Problem& p, int ng);
  unsigned long long* d_work = nullptr;  // grouped-kernel work counters (timing mode)

  // KSG_OPT_TIMING: events around each search launch, harvested by ksg_take_timing.
  bool timing = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> timed;
  // per-kernel spans: kind 0 radius, 1 Y/Z count, 2 X count, 3 single-problem search
  struct Span {
    hipEvent_t a, b;
    int kind;
  };
  std::vector<Span> spans;
  std::vector<hipEvent_t> event_pool;
  double timed_ops = 0.0;
  unsigned long long last_work[5] = {0, 0, 0, 0, 0};  // counters read by the last take_timing
  double last_kernel_ms[4] = {0, 0, 0, 0}, last_kernel_ops[4] = {0, 0, 0, 0};
  int64_t last_kernel_launches[4] = {0, 0, 0, 0};
  hipEvent_t get_event();

  int fail(int status, const char* fmt, ...);
  int hip_fail(hipError_t e, const char* what);
  int reserve(ksg::DevBuf& b, size_t bytes, const char* what);
  int reserve_host(size_t bytes);
  int wait_staging();
  int ensure_htab(int64_t n);
  int validate(const ksg::Problem& p, int index);
  int run_batch(const std::vector<ksg::Problem>& probs, double* d_out);
  int plan_batch(const std::vector<ksg::Problem>& probs, ksg::BatchPlan& plan);
  int upload_batch(const ksg::BatchPlan& plan, void* d_desc, void* d_items, void* d_jobs);
  int enqueue_batch(const ksg::BatchPlan& plan, const void* d_desc, const ksg::WorkItem* d_items,
                    const ksg::PackJob* d_jobs, double* d_out);

  // KSG_OPT_USE_GRAPH: captured batches (least recently used evicted beyond kMaxGraphs).  buf_gen
  // counts reallocations of the work buffers a graph writes (pool, E, T, partials, harmonic
  // table); a graph captured at an older generation is not replayed.
  static constexpr size_t kMaxGraphs = 32;
  std::vector<ksg::GraphEntry> graphs;
  uint64_t buf_gen = 0, graph_clock = 0;
  int64_t graph_captures = 0, graph_replays = 0;
  hipStream_t capture_stream = nullptr;
  int run_batch_graph(const std::vector<ksg::Problem>& probs, double* d_out);
  void drop_graph(ksg::GraphEntry& g);
  void clear_graphs();
  int check_columns_finite(const std::vector<ksg::PackJob>& cols, int max_pad);
  int maxstat_async(const double* d_cmi, int cands, int P, double alpha, int slot);
};
