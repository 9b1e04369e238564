// Data movement and statistics kernels around the search kernel:
//  - column packing (SoA copy / permutation gather into +inf-padded columns),
//  - the finite-data check,
//  - lagged embedding of [trials][vars][T] series into candidate columns,
//  - per-problem finalisation of the digamma sum,
//  - the max-statistic surrogate test.
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>

#include "internal.h"

namespace ksg {

extern const void* search_kernels_kp5[55];
extern const void* search_kernels_kp9[55];
extern const void* search_kernels_kp17[55];
extern const void* group_radius_kernels_kp5_g8[15];
extern const void* group_radius_kernels_kp5_g16[15];
extern const void* group_radius_kernels_kp9_g8[15];
extern const void* group_radius_kernels_kp9_g16[15];
extern const void* group_xcount_kernels_g8[15];
extern const void* group_xcount_kernels_g16[15];
extern const void* yzcount_kernels[kGroupMaxM + 1];
extern const void* group_radius_kernels_kp5_g8_wide[16];
extern const void* group_radius_kernels_kp9_g8_wide[16];
extern const void* group_xcount_kernels_g8_wide[16];
extern const void* search_kernels_wide[3];

// ------------------------------------------------------------------ packing

// grid.x: chunks of 1024 rows, grid.y: jobs (strided).  dst[i] = src[perm[i]] or src[i]; pad +inf;
// a job without a source writes a zero column (zeros in the n rows, +inf padding).
// A gather index outside [0, n) is never dereferenced: the row becomes NaN and bit 1 of
// *flag is set (the finite check then reports the batch as invalid).
__global__ __launch_bounds__(256) void pack_kernel(const PackJob* __restrict__ jobs, int n_jobs,
                                                   int* __restrict__ flag) {
  for (int jb = blockIdx.y; jb < n_jobs; jb += gridDim.y) {
    const PackJob job = jobs[jb];
    const int base = blockIdx.x * 1024;
    if (base >= job.n_pad) continue;
    if (!job.src) {  // a zero column (wide problems): zeros in the n rows, +inf padding
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = base + r * 256 + threadIdx.x;
        if (i < job.n_pad) job.dst[i] = i < job.n ? 0.0f : INFINITY;
      }
      continue;
    }
    bool bad = false;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = base + r * 256 + threadIdx.x;
      if (i < job.n) {
        int src = i;
        if (job.order) src = job.order[i];  // a permutation of [0, n) written by window_rank_kernel
        if (job.perm) {
          src = job.perm[src];
          if ((unsigned)src >= (unsigned)job.n) {
            bad = true;
            job.dst[i] = NAN;
            continue;
          }
        }
        job.dst[i] = job.src[src];
      } else if (i < job.n_pad) {
        job.dst[i] = INFINITY;
      }
    }
    if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(flag, 2);
  }
}

hipError_t launch_pack(const PackJob* d_jobs, int n_jobs, int max_pad, int* d_flag, hipStream_t stream) {
  if (n_jobs <= 0) return hipSuccess;
  dim3 grid((max_pad + 1023) / 1024, n_jobs < 65535 ? n_jobs : 65535);
  hipLaunchKernelGGL(pack_kernel, grid, dim3(256), 0, stream, d_jobs, n_jobs, d_flag);
  return hipGetLastError();
}

// Sets *flag = 1 when any of the first n rows of a job's destination is NaN or +-inf.
__global__ __launch_bounds__(256) void finite_kernel(const PackJob* __restrict__ jobs, int n_jobs,
                                                     int* __restrict__ flag) {
  for (int jb = blockIdx.y; jb < n_jobs; jb += gridDim.y) {
    const PackJob job = jobs[jb];
    const int base = blockIdx.x * 1024;
    if (base >= job.n) continue;
    bool bad = false;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = base + r * 256 + threadIdx.x;
      if (i < job.n) bad |= !isfinite(job.dst[i]);
    }
    if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(flag, 1);
  }
}

hipError_t launch_finite_check(const PackJob* d_jobs, int n_jobs, int max_pad, int* d_flag,
                               hipStream_t stream) {
  if (n_jobs <= 0) return hipSuccess;
  dim3 grid((max_pad + 1023) / 1024, n_jobs < 65535 ? n_jobs : 65535);
  hipLaunchKernelGGL(finite_kernel, grid, dim3(256), 0, stream, d_jobs, n_jobs, d_flag);
  return hipGetLastError();
}

// Sets bit 1 of *flag when any of the n_perm * n gather indices lies outside [0, n).
__global__ __launch_bounds__(256) void perm_check_kernel(const int32_t* __restrict__ perms, int64_t total,
                                                         int n, int* __restrict__ flag) {
  bool bad = false;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < total; i += (int64_t)gridDim.x * 256)
    bad |= (unsigned)perms[i] >= (unsigned)n;
  if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(flag, 2);
}

hipError_t launch_perm_check(const int32_t* perms, int n_perm, int n, int* d_flag, hipStream_t stream) {
  const int64_t total = (int64_t)n_perm * n;
  if (total <= 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>((total + 255) / 256, 4096);
  hipLaunchKernelGGL(perm_check_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, perms, total, n, d_flag);
  return hipGetLastError();
}

// Key order of a Y/Z set: the rank of row i among the n keys (column Z_1, or Y when m = 0)
// under the total order of the FP32 values' ordered bit patterns, ties by row index, so that
// the ranks are a permutation of [0, n) whatever the data; sigma[rank] = i, and the padding
// rows n..n_pad-1 map to themselves.  O(n^2) comparisons against LDS tiles of the keys: a
// few microseconds at n = 10^4, negligible beside the search.  grid.x: chunks of 256 rows,
// grid.y: groups (strided); only the group that writes the Y/Z block sorts.
__device__ __forceinline__ unsigned ordered_bits(float v) {
  const unsigned b = __float_as_uint(v);
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

__global__ __launch_bounds__(256) void key_order_kernel(const GroupDesc* __restrict__ descs,
                                                        int n_groups, float* __restrict__ base) {
  constexpr int kChunk = 2048;
  __shared__ __align__(16) unsigned s_key[kChunk];
  for (int gi = blockIdx.y; gi < n_groups; gi += gridDim.y) {
    const GroupDesc& gd = descs[gi];
    const int n = gd.n;
    const int i0 = blockIdx.x * 256;
    if (!gd.write_yz || i0 >= gd.n_pad) continue;  // uniform over the block
    const float* key = base + (gd.m > 0 ? gd.z_off[0] : gd.y_off);
    int32_t* sigma = reinterpret_cast<int32_t*>(base + gd.sigma_off);
    const int i = i0 + (int)threadIdx.x;
    if (i0 >= n) {
      if (i < gd.n_pad) sigma[i] = i;
      continue;
    }
    const unsigned long long ki =
        i < n ? ((unsigned long long)ordered_bits(key[i]) << 32) | (unsigned)i : ~0ull;
    int rank = 0;
    for (int j0 = 0; j0 < n; j0 += kChunk) {
      const int cnt = min(kChunk, n - j0);
      const int cnt4 = (cnt + 3) & ~3;
      __syncthreads();
      // entries cnt..cnt4-1 hold the largest key; their row index j0 + t >= n exceeds every i,
      // so they never rank below a real row
      for (int t = threadIdx.x; t < cnt4; t += 256) s_key[t] = t < cnt ? ordered_bits(key[j0 + t]) : ~0u;
      __syncthreads();
      // four keys per LDS read, several reads in flight
      const uint4* s4 = reinterpret_cast<const uint4*>(s_key);
#pragma unroll 4
      for (int t4 = 0; t4 < cnt4 / 4; ++t4) {
        const uint4 v = s4[t4];
        const unsigned j = (unsigned)(j0 + 4 * t4);
        rank += ((((unsigned long long)v.x << 32) | j) < ki) ? 1 : 0;
        rank += ((((unsigned long long)v.y << 32) | (j + 1)) < ki) ? 1 : 0;
        rank += ((((unsigned long long)v.z << 32) | (j + 2)) < ki) ? 1 : 0;
        rank += ((((unsigned long long)v.w << 32) | (j + 3)) < ki) ? 1 : 0;
      }
    }
    if (i < n) sigma[rank] = i;
    else if (i < gd.n_pad) sigma[i] = i;
  }
}

hipError_t launch_key_order(const GroupDesc* d_gdesc, int n_groups, int max_pad, float* base,
                            hipStream_t stream) {
  if (n_groups <= 0) return hipSuccess;
  dim3 grid((max_pad + 255) / 256, n_groups < 65535 ? n_groups : 65535);
  hipLaunchKernelGGL(key_order_kernel, grid, dim3(256), 0, stream, d_gdesc, n_groups, base);
  return hipGetLastError();
}

// Interleaved group blocks from packed columns (layouts in internal.h), rows in key order.
// grid.x: chunks of 64 four-row steps, grid.y: groups (strided).
__global__ __launch_bounds__(256) void interleave_kernel(const GroupDesc* __restrict__ descs,
                                                         int n_groups, float* __restrict__ base) {
  for (int gi = blockIdx.y; gi < n_groups; gi += gridDim.y) {
    const GroupDesc& gd = descs[gi];
    const int steps = gd.n_pad / 4;
    const int s0 = blockIdx.x * 64;
    if (s0 >= steps) continue;
    const int s1 = min(steps, s0 + 64);
    const int G = gd.G;
    const int32_t* sigma = reinterpret_cast<const int32_t*>(base + gd.sigma_off);
    auto src_row = [&](int row) {
      const unsigned r = (unsigned)sigma[row];
      return r < (unsigned)gd.n_pad ? (int)r : row;  // sigma is a permutation; never trust it blindly
    };
    // one row per thread: its source row is looked up once and its G (and m + 1) values are
    // gathered with independent loads
    float* xi = base + gd.xi_off;
    const int row = s0 * 4 + (int)threadIdx.x;  // 64 steps = 256 rows per block
    if (row < s1 * 4) {
      const int src = src_row(row);
      const int s = row >> 2, u = row & 3;
      float v[kGroupMax];
#pragma unroll
      for (int g = 0; g < kGroupMax; ++g)
        if (g < G) v[g] = base[gd.x_off[g] + src];
#pragma unroll
      for (int g = 0; g < kGroupMax; ++g)
        if (g < G) xi[(s * G + g) * 4 + u] = v[g];
      if (gd.write_yz) {
        const int W = gd.m + 1;
        float* yzi = base + gd.yzi_off;
        for (int a = 0; a < W; ++a) {
          const uint32_t col = a == 0 ? gd.y_off : gd.z_off[a - 1];
          yzi[(s * W + a) * 4 + u] = base[col + src];
        }
      }
    }
  }
}

hipError_t launch_interleave(const GroupDesc* d_gdesc, int n_groups, int max_pad, float* base,
                             hipStream_t stream) {
  if (n_groups <= 0) return hipSuccess;
  dim3 grid((max_pad / 4 + 63) / 64, n_groups < 65535 ? n_groups : 65535);
  hipLaunchKernelGGL(interleave_kernel, grid, dim3(256), 0, stream, d_gdesc, n_groups, base);
  return hipGetLastError();
}

// ------------------------------------------------------------------ embedding

// Candidate (v, l) row i: trial tr = i / (T - L), time t = L + i % (T - L), value x_v(t - l).
// grid.x: row chunks of 256, grid.y: columns (n_vars * L candidates + 1 target column).
__global__ __launch_bounds__(256) void embed_kernel(const float* __restrict__ data, int n_vars,
                                                    int64_t T, int n_trials, int target, int L,
                                                    float* __restrict__ cand, float* __restrict__ y,
                                                    int64_t stride) {
  const int c = blockIdx.y;
  const int64_t per_trial = T - L;
  const int64_t n = per_trial * n_trials;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= stride) return;
  const bool is_target = (c == n_vars * L);
  float* dst = is_target ? y : cand + (int64_t)c * stride;
  if (i >= n) {
    dst[i] = INFINITY;
    return;
  }
  const int v = is_target ? target : c / L;
  const int lag = is_target ? 0 : (c % L) + 1;
  const int64_t tr = i / per_trial;
  const int64_t t = L + (i - tr * per_trial);
  dst[i] = data[(tr * n_vars + v) * T + (t - lag)];
}

hipError_t launch_embed(const float* data, int n_vars, int64_t T, int n_trials, int target,
                        int max_lag, float* cand, float* y, int64_t col_stride, hipStream_t stream) {
  dim3 grid((unsigned)((col_stride + 255) / 256), n_vars * max_lag + 1);
  hipLaunchKernelGGL(embed_kernel, grid, dim3(256), 0, stream, data, n_vars, T, n_trials, target,
                     max_lag, cand, y, col_stride);
  return hipGetLastError();
}

// ------------------------------------------------------------------ finalisation

// I = C - S / N, S = compensated (Neumaier) sum of the problem's tile partials in tile order;
// C = H_{k-1} for algorithm 1, H_{k-1} - 2/k for algorithm 2 with Z and H_{k-1} - 1/k + H_{N-1}
// for algorithm 2 without Z.
__global__ __launch_bounds__(256) void finalize_kernel(const ProbDesc* __restrict__ descs, int n_probs,
                                                       const double* __restrict__ partials,
                                                       const double* __restrict__ htab,
                                                       double* __restrict__ out) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n_probs) return;
  const ProbDesc& d = descs[p];
  double s = 0.0, comp = 0.0;
  for (int t = 0; t < d.n_tiles; ++t) {
    const double v = partials[d.part_base + t];
    const double u = s + v;
    comp += (fabs(s) >= fabs(v)) ? (s - u) + v : (v - u) + s;
    s = u;
  }
  s += comp;
  double c = htab[d.k - 1];
  if (d.alg == 2) c = d.dz > 0 ? c - 2.0 / (double)d.k : (c - 1.0 / (double)d.k) + htab[d.n - 1];
  out[d.out_index] = c - s / (double)d.n;
}

static const void* pick_search_kernel(int shape, int kp) {
  if (shape == kGenericShape + kWideDims) return search_kernels_wide[kp <= 5 ? 0 : (kp <= 9 ? 1 : 2)];
  const void* const* table = kp <= 5 ? search_kernels_kp5 : (kp <= 9 ? search_kernels_kp9 : search_kernels_kp17);
  if (shape >= 0 && shape < 39) return table[shape];
  if (shape >= kGenericShape + 2 && shape <= kGenericShape + kMaxDimsCompiled)
    return table[40 + shape - kGenericShape - 2];
  return table[39];
}

hipError_t launch_ksg_search(const ProbDesc* d_desc, const WorkItem* d_items, int n_items,
                             const double* d_htab, double* d_partials, int shape, int kp,
                             hipStream_t stream, int tile_q) {
  if (n_items <= 0) return hipSuccess;
  if (tile_q != 64 && tile_q != 128 && tile_q != 256) return hipErrorInvalidValue;
  const void* fn = pick_search_kernel(shape, kp);
  const ProbDesc* a0 = d_desc;
  const WorkItem* a1 = d_items;
  const double* a2 = d_htab;
  double* a3 = d_partials;
  void* args[] = {&a0, &a1, &a2, &a3};
  return hipLaunchKernel(fn, dim3(n_items), dim3(tile_q), args, 0, stream);
}

hipError_t launch_ksg_group_radius(const float* base, const GroupDesc* d_gdesc, const WorkItem* d_items,
                                   int n_items, float* E, int m, int G, int kp,
                                   unsigned long long* d_work, hipStream_t stream) {
  if (n_items <= 0) return hipSuccess;
  // m <= 14: any group size; m = 15..30: 8 problems per group only
  if (m < 0 || m > kGroupMaxM || (G != 8 && G != 16) || (kp != 5 && kp != 9) || (G == 16 && m > kGroupMaxM16))
    return hipErrorInvalidValue;
  const void* fn;
  if (m > kGroupMaxM16) {
    fn = (kp == 5 ? group_radius_kernels_kp5_g8_wide : group_radius_kernels_kp9_g8_wide)[m - kGroupMaxM16 - 1];
  } else {
    const void* const* table = kp == 5 ? (G == 8 ? group_radius_kernels_kp5_g8 : group_radius_kernels_kp5_g16)
                                       : (G == 8 ? group_radius_kernels_kp9_g8 : group_radius_kernels_kp9_g16);
    fn = table[m];
  }
  const float* a0 = base;
  const GroupDesc* a1 = d_gdesc;
  const WorkItem* a2 = d_items;
  float* a3 = E;
  unsigned long long* a4 = d_work;
  void* args[] = {&a0, &a1, &a2, &a3, &a4};
  return hipLaunchKernel(fn, dim3(n_items), dim3(kTileQ), args, 0, stream);
}

hipError_t launch_ksg_yzcount(const float* base, const YZDesc* d_ydesc, const WorkItem* d_items,
                              int n_items, const float* E, double* T, const double* d_htab, int m,
                              unsigned long long* d_work, hipStream_t stream) {
  if (n_items <= 0) return hipSuccess;
  if (m < 0 || m > kGroupMaxM) return hipErrorInvalidValue;
  const float* a0 = base;
  const YZDesc* a1 = d_ydesc;
  const WorkItem* a2 = d_items;
  const float* a3 = E;
  double* a4 = T;
  const double* a5 = d_htab;
  unsigned long long* a6 = d_work;
  void* args[] = {&a0, &a1, &a2, &a3, &a4, &a5, &a6};
  return hipLaunchKernel(yzcount_kernels[m], dim3(n_items), dim3(256), args, 0, stream);
}

hipError_t launch_ksg_group_xcount(const float* base, const GroupDesc* d_gdesc, const WorkItem* d_items,
                                   int n_items, const float* E, const double* T, const double* d_htab,
                                   double* d_partials, int m, int G, unsigned long long* d_work,
                                   hipStream_t stream) {
  if (n_items <= 0) return hipSuccess;
  if (m < 0 || m > kGroupMaxM || (G != 8 && G != 16) || (G == 16 && m > kGroupMaxM16)) return hipErrorInvalidValue;
  const void* fn = m > kGroupMaxM16 ? group_xcount_kernels_g8_wide[m - kGroupMaxM16 - 1]
                                    : (G == 8 ? group_xcount_kernels_g8 : group_xcount_kernels_g16)[m];
  const float* a0 = base;
  const GroupDesc* a1 = d_gdesc;
  const WorkItem* a2 = d_items;
  const float* a3 = E;
  const double* a4 = T;
  const double* a5 = d_htab;
  double* a6 = d_partials;
  unsigned long long* a7 = d_work;
  void* args[] = {&a0, &a1, &a2, &a3, &a4, &a5, &a6, &a7};
  return hipLaunchKernel(fn, dim3(n_items), dim3(kTileQ), args, 0, stream);
}

hipError_t launch_finalize(const ProbDesc* d_desc, int n_probs, const double* d_partials,
                           const double* d_htab, double* d_out, hipStream_t stream) {
  hipLaunchKernelGGL(finalize_kernel, dim3((n_probs + 255) / 256), dim3(256), 0, stream, d_desc,
                     n_probs, d_partials, d_htab, d_out);
  return hipGetLastError();
}

// ------------------------------------------------------------------ max statistic

// One block.  cmi: [c][P+1], column 0 = originals.  T_p = max_c cmi[c][p]; count of T_p >= t_obs;
// thresholds by stable descending rank (rank r-1 is the r-th largest).
constexpr int kMaxPerm = 4096;

__global__ __launch_bounds__(1024) void maxstat_kernel(const double* __restrict__ cmi, int c, int P,
                                                       double alpha, MaxStatOut* __restrict__ out) {
  __shared__ double tmax[kMaxPerm];
  __shared__ int s_count;
  __shared__ int s_cstar;
  if (threadIdx.x == 0) {
    int best = 0;
    for (int i = 1; i < c; ++i)
      if (cmi[(int64_t)i * (P + 1)] > cmi[(int64_t)best * (P + 1)]) best = i;
    s_cstar = best;
    s_count = 0;
  }
  __syncthreads();
  const double t_obs = cmi[(int64_t)s_cstar * (P + 1)];
  int local = 0;
  for (int p = threadIdx.x; p < P; p += blockDim.x) {
    double m = cmi[p + 1];
    for (int i = 1; i < c; ++i) m = fmax(m, cmi[(int64_t)i * (P + 1) + p + 1]);
    tmax[p] = m;
    local += (m >= t_obs) ? 1 : 0;
  }
  atomicAdd(&s_count, local);
  __syncthreads();
  const int r05 = min(max((int)ceil(0.05 * P), 1), P);
  const int r01 = min(max((int)ceil(0.01 * P), 1), P);
  for (int p = threadIdx.x; p < P; p += blockDim.x) {
    const double v = tmax[p];
    int rank = 0;
    for (int q = 0; q < P; ++q) rank += (tmax[q] > v) || (tmax[q] == v && q < p);
    if (rank == r05 - 1) out->tau05 = v;
    if (rank == r01 - 1) out->tau01 = v;
  }
  if (threadIdx.x == 0) {
    const double pval = (double)s_count / (double)P;
    out->c_star = s_cstar;
    out->count = s_count;
    out->n_perm = P;
    out->t_obs = t_obs;
    out->pval = pval;
    out->significant = pval < alpha ? 1 : 0;
  }
}

hipError_t launch_maxstat(const double* cmi, int c, int n_perm, double alpha, MaxStatOut* out,
                          hipStream_t stream) {
  if (n_perm > kMaxPerm || n_perm < 1 || c < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(maxstat_kernel, dim3(1), dim3(1024), 0, stream, cmi, c, n_perm, alpha, out);
  return hipGetLastError();
}

}  // namespace ksg
