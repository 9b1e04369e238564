// Key-ordered window search for single problems (any shape) that share an unpermuted Z column.
//
// Same estimator as the brute-force single-problem kernel (KSG algorithm 1: joint k-th
// neighbour radius with self included, strict counts in XZ, YZ and Z, FP64 digamma partial
// sums per tile), on columns that the pack step has written in ascending order of one key
// column of the problem (rows ordered by the FP32 bit order of the key, ties by row index).
// The key is a column of Z: then d^Z >= |dkey| bounds all three counts (and the joint distance
// bounds the radius), so rows outside the window can change neither.
// Every distance is at least the key difference |fl(k_j - k_i)|, and that difference grows
// monotonically with the distance of row j from row i in key order, so a tile of 256
// consecutive rows first scans its own rows and then steps outward, right and left; a
// direction stops at the first step whose nearest key is, for every lane of the wave, at
// least the lane's bound away (the current (k+1)-th distance in the radius pass, eps_i in the
// count pass): no later row in that direction can change a result.  The estimate is a sum over
// all rows, so the row order changes it only by the order of the FP64 summation.
#include "ksg_search.inc.h"

namespace ksg {

// Rank of every key under the total order (ordered bits, then row): sigma[rank] = row; rows
// n..n_pad-1 map to themselves.
__global__ __launch_bounds__(256) void window_rank_kernel(const float* __restrict__ key, int n, int n_pad,
                                                          int32_t* __restrict__ sigma) {
  constexpr int kChunk = 2048;
  __shared__ __align__(16) unsigned s_key[kChunk];
  const int i = blockIdx.x * 256 + (int)threadIdx.x;
  auto ordered = [](float v) {
    const unsigned b = __float_as_uint(v);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
  };
  const unsigned long long ki = i < n ? ((unsigned long long)ordered(key[i]) << 32) | (unsigned)i : ~0ull;
  int rank = 0;
  for (int j0 = 0; j0 < n; j0 += kChunk) {
    const int cnt = min(kChunk, n - j0);
    const int cnt4 = (cnt + 3) & ~3;
    __syncthreads();
    for (int t = threadIdx.x; t < cnt4; t += 256) s_key[t] = t < cnt ? ordered(key[j0 + t]) : ~0u;
    __syncthreads();
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
  else if (i < n_pad) sigma[i] = i;
}

// Steps (4 rows) outward: alternately one step right (from r) and one step left (from l) while
// that direction is open.  f(s) runs a step; open_right(s) / open_left(s) test a step's nearest
// key against the lanes' bounds.
template <class Step, class OpenR, class OpenL>
__device__ __forceinline__ void window_outward(int r, int l, int steps, Step f, OpenR open_right,
                                               OpenL open_left, unsigned& n_steps) {
  bool go_r = r < steps, go_l = l >= 0;
  while (go_r || go_l) {
    if (go_r) {
      if (open_right(r)) {
        f(r);
        ++n_steps;
        go_r = ++r < steps;
      } else {
        go_r = false;
      }
    }
    if (go_l) {
      if (open_left(l)) {
        f(l);
        ++n_steps;
        go_l = --l >= 0;
      } else {
        go_l = false;
      }
    }
  }
}

// The steps [s_lo, s_hi] without a test, then outward from them.
template <class Step, class OpenR, class OpenL>
__device__ __forceinline__ void window_scan(int s_lo, int s_hi, int steps, Step f, OpenR open_right,
                                            OpenL open_left, unsigned& n_steps) {
  for (int s = s_lo; s <= s_hi; ++s) f(s);
  n_steps += (unsigned)(s_hi - s_lo + 1);
  window_outward(s_hi + 1, s_lo - 1, steps, f, open_right, open_left, n_steps);
}

// Count step with a compile-time split of the D = DX + DY + DZ columns (strict counts).
template <int DX, int DY, int DZ>
__device__ __forceinline__ void window_count_step(const cfptr (&col)[DX + DY + DZ],
                                                  const float (&q)[DX + DY + DZ], int s, float eps,
                                                  unsigned (&acc)[3]) {
  constexpr int D = DX + DY + DZ;
  constexpr int U = 4;
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int j = 4 * s + u;
    float A = fabsf(col[0][j] - q[0]);
#pragma unroll
    for (int a = 1; a < DX; ++a) A = fmaxf(A, fabsf(col[a][j] - q[a]));
    float B = fabsf(col[DX][j] - q[DX]);
#pragma unroll
    for (int a = DX + 1; a < DX + DY; ++a) B = fmaxf(B, fabsf(col[a][j] - q[a]));
    if constexpr (DZ > 0) {
      float C = fabsf(col[DX + DY][j] - q[DX + DY]);
#pragma unroll
      for (int a = DX + DY + 1; a < D; ++a) C = fmaxf(C, fabsf(col[a][j] - q[a]));
      acc[0] += (unsigned)(fmaxf(A, C) < eps);
      acc[1] += (unsigned)(fmaxf(B, C) < eps);
      acc[2] += (unsigned)(C < eps);
    } else {
      acc[0] += (unsigned)(A < eps);
      acc[1] += (unsigned)(B < eps);
    }
  }
}

// Count step for a split known only at run time (per-column selects).
template <int D>
__device__ __forceinline__ void window_count_step_split(const cfptr (&col)[D], const float (&q)[D], int s,
                                                        float eps, int dx, int dy, unsigned (&acc)[3]) {
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int j = 4 * s + u;
    float A = 0.0f, B = 0.0f, C = 0.0f;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const float t = fabsf(col[a][j] - q[a]);
      if (a < dx) A = fmaxf(A, t);
      else if (a < dx + dy) B = fmaxf(B, t);
      else C = fmaxf(C, t);
    }
    acc[0] += (unsigned)(fmaxf(A, C) < eps);
    acc[1] += (unsigned)(fmaxf(B, C) < eps);
    acc[2] += (unsigned)(C < eps);
  }
}

// Count pass for dx == 1 and a wave-uniform dy in [DY, D): one compile-time loop per dy.
template <int D, int DY, class OpenR, class OpenL>
__device__ __forceinline__ void window_count_dx1(const cfptr (&col)[D], const float (&q)[D], int dy, float eps,
                                                 int s_lo, int s_hi, int steps, OpenR open_r, OpenL open_l,
                                                 unsigned (&acc)[3], unsigned& n_steps) {
  if constexpr (DY < D - 1) {
    if (dy == DY) {
      window_scan(s_lo, s_hi, steps, [&](int s) { window_count_step<1, DY, D - 1 - DY>(col, q, s, eps, acc); },
                  open_r, open_l, n_steps);
      return;
    }
    window_count_dx1<D, DY + 1>(col, q, dy, eps, s_lo, s_hi, steps, open_r, open_l, acc, n_steps);
  } else {
    window_scan(s_lo, s_hi, steps, [&](int s) { window_count_step<1, D - 1, 0>(col, q, s, eps, acc); }, open_r,
                open_l, n_steps);
  }
}

// Count pass for dx == 2 (so dy >= 2 in the canonical split, and dz >= 1 for a window
// problem): one compile-time loop per dy in [DY, D - 3].
template <int D, int DY, class OpenR, class OpenL>
__device__ __forceinline__ void window_count_dx2(const cfptr (&col)[D], const float (&q)[D], int dy, float eps,
                                                 int s_lo, int s_hi, int steps, OpenR open_r, OpenL open_l,
                                                 unsigned (&acc)[3], unsigned& n_steps) {
  if constexpr (DY < D - 3) {
    if (dy == DY) {
      window_scan(s_lo, s_hi, steps, [&](int s) { window_count_step<2, DY, D - 2 - DY>(col, q, s, eps, acc); },
                  open_r, open_l, n_steps);
      return;
    }
    window_count_dx2<D, DY + 1>(col, q, dy, eps, s_lo, s_hi, steps, open_r, open_l, acc, n_steps);
  } else {
    window_scan(s_lo, s_hi, steps, [&](int s) { window_count_step<2, D - 3, 1>(col, q, s, eps, acc); }, open_r,
                open_l, n_steps);
  }
}

template <int D, int KP>
__global__ __launch_bounds__(kTileQ) void ksg_window_kernel(const ProbDesc* __restrict__ descs,
                                                            const WorkItem* __restrict__ items,
                                                            const double* __restrict__ htab,
                                                            double* __restrict__ partials,
                                                            unsigned long long* __restrict__ work) {
  __shared__ double s_red[kTileQ / 64];
  __shared__ unsigned long long s_ord[kTileQ];
  __shared__ float s_x[KP][kTileQ];
  const KSG_AS4 ProbDesc* d4 = (const KSG_AS4 ProbDesc*)descs;
  const KSG_AS4 WorkItem* i4 = (const KSG_AS4 WorkItem*)items;
  const int prob = i4[blockIdx.x].prob;
  if (prob < 0) return;
  const int tile = i4[blockIdx.x].tile;
  const KSG_AS4 ProbDesc* pd = d4 + prob;
  const int n = pd->n;
  const int n_pad = pd->n_pad;
  const int k = pd->k;
  const int dx = pd->dx, dy = pd->dy;
  const int qraw = tile * kTileQ + (int)threadIdx.x;
  bool valid = qraw < n;
  int qi = valid ? qraw : n - 1;
  cfptr col[D];
  float q[D];
#pragma unroll
  for (int a = 0; a < D; ++a) {
    const float* c = pd->col[a];
    col[a] = (cfptr)c;
    q[a] = c[qi];
  }
  const float* keyc = pd->col[pd->key_col];
  const cfptr kcol = (cfptr)keyc;
  float qkey = keyc[qi];
  const int steps = n_pad / 4;
  // the tile's own rows (the last tile ends at the last real row's step)
  const int s_lo = tile * (kTileQ / 4);
  const int s_hi = min((tile + 1) * (kTileQ / 4), (n + 3) / 4) - 1;
  unsigned n1 = 0, n2 = 0;

  // ---- pass 1: (k+1) smallest joint distances within the key window ----
  // Phase 1 scans the tile's rows and its neighbouring tiles' for every query, which bounds
  // each radius; the tile's queries are then handed to the waves again in ascending order of
  // that bound (the lists move through LDS), so that a wave's window is not held open by a few
  // wide queries; phase 2 scans outward from the phase-1 rows with each wave's window.
  float b[KP];
#pragma unroll
  for (int i = 0; i < KP; ++i) b[i] = (i < KP - 1 - k) ? -INFINITY : INFINITY;
  auto radius_step = [&](int s) {
    float d[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) d[u] = fabsf(col[0][4 * s + u] - q[0]);
#pragma unroll
    for (int a = 1; a < D; ++a) {
#pragma unroll
      for (int u = 0; u < 4; ++u) d[u] = fmaxf(d[u], fabsf(col[a][4 * s + u] - q[a]));
    }
    bool hit = false;
#pragma unroll
    for (int u = 0; u < 4; ++u) hit |= d[u] < b[KP - 1];
    if (hit) {
#pragma unroll
      for (int u = 0; u < 4; ++u) topk_insert<KP>(b, d[u]);
    }
  };
  const int real_steps = (n + 3) / 4;
  const int p_lo = max(s_lo - kTileQ / 4, 0);
  const int p_hi = min(s_hi + kTileQ / 4, real_steps - 1);
  for (int s = p_lo; s <= p_hi; ++s) radius_step(s);
  n1 += (unsigned)(p_hi - p_lo + 1);

  // regroup: sort the tile's (key, row) pairs in LDS; invalid lanes sort last
  const int tid = (int)threadIdx.x;
  auto regroup = [&](unsigned keybits) {
    s_ord[tid] = valid ? ((unsigned long long)keybits << 32) | (unsigned)qi : ~0ull;
    __syncthreads();
    for (int size = 2; size <= kTileQ; size <<= 1) {
      for (int stride = size >> 1; stride > 0; stride >>= 1) {
        if (tid < kTileQ / 2) {
          const int lo = 2 * tid - (tid & (stride - 1));
          const int hi = lo + stride;
          const unsigned long long a = s_ord[lo], c = s_ord[hi];
          if ((a > c) == ((lo & size) == 0)) {
            s_ord[lo] = c;
            s_ord[hi] = a;
          }
        }
        __syncthreads();
      }
    }
    const unsigned long long kk = s_ord[tid];
    __syncthreads();  // s_ord is reused by the next regroup
    return kk;
  };
  auto take_query = [&](unsigned long long kk) {
    valid = kk != ~0ull;
    qi = valid ? (int)(unsigned)(kk & 0xffffffffu) : n - 1;
#pragma unroll
    for (int a = 0; a < D; ++a) q[a] = pd->col[a][qi];
    qkey = keyc[qi];
  };
  {
    const unsigned long long kk = regroup(__float_as_uint(b[KP - 1]));
    const int src = kk != ~0ull ? (int)(unsigned)(kk & 0xffffffffu) - tile * kTileQ : tid;  // lane of the row
#pragma unroll
    for (int i = 0; i < KP; ++i) s_x[i][tid] = b[i];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < KP; ++i) b[i] = s_x[i][src];
    __syncthreads();
    take_query(kk);
  }
  auto open_r1 = [&](int s) {
    return __builtin_amdgcn_ballot_w64(fabsf(kcol[4 * s] - qkey) < b[KP - 1]) != 0;
  };
  auto open_l1 = [&](int s) {
    return __builtin_amdgcn_ballot_w64(fabsf(kcol[4 * s + 3] - qkey) < b[KP - 1]) != 0;
  };
  // phase 2: outward from the phase-1 rows (window_scan's first loop is empty)
  window_outward(p_hi + 1, p_lo - 1, steps, radius_step, open_r1, open_l1, n1);
  float eps = b[KP - 1];

  // ---- pass 2: strict counts within the key window of eps, queries regrouped by eps ----
  {
    const unsigned long long kk = regroup(valid ? __float_as_uint(eps) : 0u);
    eps = kk != ~0ull ? __uint_as_float((unsigned)(kk >> 32)) : 0.0f;  // invalid lanes widen nothing
    take_query(kk);
  }
  unsigned acc[3] = {0u, 0u, 0u};
  auto open_r2 = [&](int s) { return __builtin_amdgcn_ballot_w64(fabsf(kcol[4 * s] - qkey) < eps) != 0; };
  auto open_l2 = [&](int s) { return __builtin_amdgcn_ballot_w64(fabsf(kcol[4 * s + 3] - qkey) < eps) != 0; };
  bool counted = false;
  if (dx == 1) {
    window_count_dx1<D, 1>(col, q, dy, eps, s_lo, s_hi, steps, open_r2, open_l2, acc, n2);
    counted = true;
  }
  if constexpr (D >= 5) {
    if (dx == 2) {
      window_count_dx2<D, 2>(col, q, dy, eps, s_lo, s_hi, steps, open_r2, open_l2, acc, n2);
      counted = true;
    }
  }
  if (!counted)
    window_scan(s_lo, s_hi, steps, [&](int s) { window_count_step_split<D>(col, q, s, eps, dx, dy, acc); },
                open_r2, open_l2, n2);
  if (work && (threadIdx.x & 63) == 0)
    atomicAdd(&work[5], (unsigned long long)n1 * (unsigned)(2 * D) + (unsigned long long)n2 * (unsigned)(2 * D + 2));
  tile_epilogue(pd, tile, qi, valid, eps, (int)acc[0], (int)acc[1], (int)acc[2], dx + dy == D, htab, partials,
                s_red);
}

#define KSG_WIN(D) reinterpret_cast<const void*>(&ksg_window_kernel<D, 5>)
// [D - 2] for D in [2, 16]; top-k of 5 slots (k <= 4)
const void* window_kernels[15] = {KSG_WIN(2),  KSG_WIN(3),  KSG_WIN(4),  KSG_WIN(5),  KSG_WIN(6),
                                  KSG_WIN(7),  KSG_WIN(8),  KSG_WIN(9),  KSG_WIN(10), KSG_WIN(11),
                                  KSG_WIN(12), KSG_WIN(13), KSG_WIN(14), KSG_WIN(15), KSG_WIN(16)};

hipError_t launch_window_rank(const float* key, int n, int n_pad, int32_t* sigma, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(window_rank_kernel, dim3((n_pad + 255) / 256), dim3(256), 0, stream, key, n, n_pad, sigma);
  return hipGetLastError();
}

hipError_t launch_ksg_window(const ProbDesc* d_desc, const WorkItem* d_items, int n_items, const double* d_htab,
                             double* d_partials, int D, unsigned long long* d_work, hipStream_t stream) {
  if (n_items <= 0) return hipSuccess;
  if (D < 2 || D > kMaxDims) return hipErrorInvalidValue;
  const ProbDesc* a0 = d_desc;
  const WorkItem* a1 = d_items;
  const double* a2 = d_htab;
  double* a3 = d_partials;
  unsigned long long* a4 = d_work;
  void* args[] = {&a0, &a1, &a2, &a3, &a4};
  return hipLaunchKernel(window_kernels[D - 2], dim3(n_items), dim3(kTileQ), args, 0, stream);
}

}  // namespace ksg
