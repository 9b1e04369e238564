// Internal data structures shared by the host runtime and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ksg {

constexpr int kMaxDims = 32;        // columns of one problem (X + Y + Z)
constexpr int kMaxDimsCompiled = 16; // column counts with kernels compiled per count (brute force,
                                     // key-ordered windows, algorithm 2)
constexpr int kWideDims = 32;        // 16 < D <= 32: one brute-force kernel compiled for 32 columns,
                                     // the columns beyond D being zero columns in Z
constexpr int kGroupMaxM = kMaxDims - 2;  // conditioning columns of grouped problems
constexpr int kGroupMaxM16 = 14;          // ... with 16 problems per group
constexpr int kTileQ = 256;       // queries per work item (4 waves x 64 lanes, one query per lane)
constexpr int kPad = 64;          // column length is padded to a multiple of this with +inf
constexpr int kMaxK = 16;
constexpr int kWindowMinN = 2048;  // smallest N searched with key-ordered windows (single problems)

// One CMI problem as the search kernel sees it.  Columns are ordered X..., Y..., Z...,
// each padded with +inf rows up to n_pad.  256 + 96 bytes, 16-byte aligned.
struct alignas(16) ProbDesc {
  const float* col[kMaxDims];
  int32_t n;          // points
  int32_t n_pad;      // multiple of kPad
  int32_t dx, dy, dz, k;
  int32_t n_tiles;    // ceil(n / tile height of the problem's launch)
  int32_t part_base;  // first slot of this problem's per-tile partial sums
  float* eps_out;     // optional per-point outputs (nullptr when not wanted)
  int32_t* counts_out;
  double* local_out;
  int32_t variant;    // shape id (see shape_id)
  int32_t out_index;  // slot in the output array
  int32_t swap_xy;    // 1: X and Y were exchanged to reach a fast shape (count rows swap back)
  int32_t alg;        // KSG algorithm: 1 (joint radius, strict counts) or 2 (rectangles)
  int32_t key_col;    // key-ordered window search: the column (a Z column) the rows are sorted by
  int32_t pad_;
  const int32_t* key_order;  // window search: source row of each key-ordered row (n_pad entries)
};
static_assert(sizeof(ProbDesc) % 16 == 0, "ProbDesc is copied as an array of 16-byte aligned records");

// G problems that share Y (1-D), Z (m columns), N and k and differ in a 1-D X column.
// All offsets are in floats from one pool.  x_off / y_off / z_off locate the packed source
// columns; xi_off / yzi_off the interleaved blocks the search kernel reads:
//   X block  [n_pad/4][G][4]   (G = the kernel's group size; unused slots repeat column 0)
//   YZ block [n_pad/4][m+1][4] (Y first), shared by every group with the same Y and Z and
//   written by the group with write_yz = 1.
// Both blocks hold the rows in ascending order of the key column (Z_1, or Y when m = 0):
// block row r is source row sigma[r], sigma at sigma_off (int32, n_pad entries, written once
// per Y/Z set; rows n..n_pad-1 map to themselves).  The estimate is a sum over all rows, so
// the order does not change it; it lets a wave of neighbouring queries bound its search to
// a window of the key column.
// Problem g of the group writes its per-tile partial sums at part_base + g * n_tiles + tile.
constexpr int kGroupMax = 16;
struct alignas(16) GroupDesc {
  uint32_t x_off[kGroupMax];
  uint32_t y_off;
  uint32_t z_off[kMaxDims - 2];
  uint32_t xi_off;
  uint32_t yzi_off;
  int32_t n, n_pad, k, m;
  int32_t ng;         // problems in this group
  int32_t G;          // group size of the kernel that searches it
  int32_t n_tiles;
  int32_t part_base;
  int32_t write_yz;
  uint32_t sigma_off;
  uint32_t e_off;  // element offset of the group's radii E[row][G] and terms T[row][G]
};
static_assert(sizeof(GroupDesc) % 16 == 0, "GroupDesc is copied as an array of 16-byte aligned records");

// Y/Z count work (ksg_yzcount.hip): the problems of one Y/Z set held by a run of consecutive
// groups of one launch, slots [slot0, slot0 + n_slots) of the run (slot = group-in-run * G +
// g, all real problems).  Slot s of the run has its radius and term at element
//   e_off + (s / G) * n_pad * G + row * G + s % G   of E (FP32) and T (FP64).
constexpr int kYZSlots = 2048;
struct YZDesc {
  uint32_t yzi_off;  // key-ordered YZ block of the set
  uint32_t e_off;    // element offset of the run's first group
  int32_t n, n_pad, G;
  int32_t slot0, n_slots;
  int32_t pad_;
};

// Work item: one query tile of one problem (or group); prob < 0 marks an empty slot.
struct WorkItem {
  int32_t prob;
  int32_t tile;
};

// A column copy job for the pack kernel: dst[i] = src[perm ? perm[i] : i] (i < n),
// +inf for n <= i < n_pad.  src == nullptr: dst[i] = 0 for i < n, +inf for n <= i < n_pad
// (the zero columns that fill a wide problem up to kWideDims columns).
struct PackJob {
  const float* src;
  const int32_t* perm;
  float* dst;
  int32_t n;
  int32_t n_pad;
  const int32_t* order;  // nullptr, or: destination row r takes source row perm[order[r]] (order[r])
};

// Fast shapes are (dx, dy) in {(1,1), (1,2), (2,2)} with dz in [0, kFastMaxDz]; every
// other shape uses the generic path.  dx > dy is canonicalised by swapping X and Y
// (the estimator is symmetric in X and Y, bit for bit).
constexpr int kFastMaxDz = 12;
constexpr int kGenericShape = 1000;

inline int shape_id(int dx, int dy, int dz) {
  int pair = -1;
  if (dx == 1 && dy == 1) pair = 0;
  else if (dx == 1 && dy == 2) pair = 1;
  else if (dx == 2 && dy == 2) pair = 2;
  if (pair < 0 || dz > kFastMaxDz || dx + dy + dz > kMaxDimsCompiled) return kGenericShape;
  return pair * (kFastMaxDz + 1) + dz;
}

// Step-level outputs of the max-statistic kernel (mirrors ksg_maxstat_result).
struct MaxStatOut {
  int32_t c_star;
  int32_t count;
  int32_t significant;
  int32_t n_perm;
  double t_obs;
  double pval;
  double tau05;
  double tau01;
};

// ---- launchers implemented in the .hip translation units ----
// Search + count + per-tile digamma partial sums for every work item, then the
// per-problem finalisation.  kp = number of top-k registers (5, 9 or 17); shape = the common
// fast shape id of the launch, kGenericShape + D when every problem is a generic shape of D
// columns, or -1 for a mixed launch.
hipError_t launch_ksg_search(const ProbDesc* d_desc, const WorkItem* d_items, int n_items,
                             const double* d_htab, double* d_partials, int shape, int kp,
                             hipStream_t stream, int tile_q = kTileQ);
// Key order of one column (sigma[rank] = row) and the key-ordered window search over the work
// items of problems that all have D columns (k <= 4), KSG algorithm alg (1 or 2).
hipError_t launch_window_rank(const float* key, int n, int n_pad, int32_t* sigma, hipStream_t stream);
hipError_t launch_ksg_window(const ProbDesc* d_desc, const WorkItem* d_items, int n_items, const double* d_htab,
                             double* d_partials, int D, int alg, unsigned long long* d_work, hipStream_t stream);
// KSG algorithm 2 over the work items of problems that all have D columns.
hipError_t launch_ksg_alg2(const ProbDesc* d_desc, const WorkItem* d_items, int n_items,
                           const double* d_htab, double* d_partials, int D, int kp, hipStream_t stream);
hipError_t launch_ksg_group_radius(const float* base, const GroupDesc* d_gdesc, const WorkItem* d_items,
                                   int n_items, float* E, int m, int G, int kp,
                                   unsigned long long* d_work, hipStream_t stream);
hipError_t launch_ksg_yzcount(const float* base, const YZDesc* d_ydesc, const WorkItem* d_items,
                              int n_items, const float* E, double* T, const double* d_htab, int m,
                              unsigned long long* d_work, hipStream_t stream);
hipError_t launch_ksg_group_xcount(const float* base, const GroupDesc* d_gdesc, const WorkItem* d_items,
                                   int n_items, const float* E, const double* T, const double* d_htab,
                                   double* d_partials, int m, int G, unsigned long long* d_work,
                                   hipStream_t stream);
hipError_t launch_key_order(const GroupDesc* d_gdesc, int n_groups, int max_pad, float* base,
                            hipStream_t stream);
hipError_t launch_interleave(const GroupDesc* d_gdesc, int n_groups, int max_pad, float* base,
                             hipStream_t stream);
hipError_t launch_finalize(const ProbDesc* d_desc, int n_probs, const double* d_partials,
                           const double* d_htab, double* d_out, hipStream_t stream);

hipError_t launch_pack(const PackJob* d_jobs, int n_jobs, int max_pad, int* d_flag, hipStream_t stream);
hipError_t launch_finite_check(const PackJob* d_jobs, int n_jobs, int max_pad, int* d_flag,
                               hipStream_t stream);
hipError_t launch_perm_check(const int32_t* perms, int n_perm, int n, int* d_flag, hipStream_t stream);
hipError_t launch_embed(const float* data, int n_vars, int64_t T, int n_trials, int target,
                        int max_lag, float* cand, float* y, int64_t col_stride,
                        hipStream_t stream);
hipError_t launch_maxstat(const double* cmi, int c, int n_perm, double alpha, MaxStatOut* out,
                          hipStream_t stream);
// Set-up of cmi_ksg_noalloc's static scratch array on the current device (once per device).
hipError_t noalloc_init(int device);

}  // namespace ksg
