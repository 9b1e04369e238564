// KSG search kernel: brute-force max-norm k-th neighbour radius, strict subspace range
// counts and the FP64 harmonic-number partial sum of one 256-query tile.
//
// Estimator (KSG algorithm 1 in the conditional form of Frenzel & Pompe; the paper names
// the KSG estimator in its Summary, estimator paragraph, without printing it):
//   eps_i  = k-th smallest joint max-norm distance to the other points,
//   n_S(i) = #{ j != i : d^S_ij < eps_i } for S in {XZ, YZ, Z},
//   term_i = H_{n_XZ(i)} + H_{n_YZ(i)} - H_{n_Z(i)},  I = H_{k-1} - (1/N) sum_i term_i.
//
// Mapping to CDNA4.  One query per lane, 4 waves per work item.  Reference points are
// read through the scalar data path (constant address space, wave-uniform addresses), so
// every reference coordinate arrives in an SGPR and feeds v_sub_f32 as its scalar operand:
// no LDS traffic and no VGPRs are spent on references, and the VALU does only the
// estimator's own arithmetic (sub, max with |.| source modifiers folded into v_max3,
// compare).  Self is not skipped: d_ii = 0 is always among the k+1 smallest, so the
// (k+1)-th smallest of all N distances is eps_i, and every count includes self exactly
// when eps_i > 0, which the epilogue subtracts.  Padding rows are +inf in every column,
// so they never enter the top-k or a count.
//
// Top-k: KP sorted registers, ascending; the first KP-1-k hold -inf (inert), the last
// k+1 the smallest distances seen; insertion is KP-1 v_med3_f32 + 1 v_min_f32 and runs only
// when some lane of the wave has a candidate below its current radius.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

#include "internal.h"

#define KSG_AS4 __attribute__((address_space(4)))

namespace ksg {

typedef const KSG_AS4 float* cfptr;

template <int KP>
__device__ __forceinline__ void topk_insert(float (&b)[KP], float d) {
#pragma unroll
  for (int i = KP - 1; i >= 1; --i) b[i] = __builtin_amdgcn_fmed3f(b[i - 1], b[i], d);
  b[0] = __builtin_amdgcn_fmed3f(-INFINITY, b[0], d);
}

// Insertion of four candidates given as the bit patterns of non-negative floats, for waves in
// which some lane has a candidate below its radius.  The candidates are inserted in ascending
// order, and usually only the smallest is below the radius: the three others are inserted only
// when the second smallest still is, for some lane of the wave.  Inserting the values in order
// equals inserting the multiset (an insertion of a value >= the radius changes nothing), so the
// result is that of four plain insertions.  b[0] takes a signed integer minimum of the bit
// patterns, which orders -inf (an inert slot) below every non-negative value as the FP32
// minimum does, without the quieting copies an IEEE-mode minimum needs.
template <int KP>
__device__ __forceinline__ void topk_insert_sorted(float (&b)[KP], float v) {
#pragma unroll
  for (int i = KP - 1; i >= 1; --i) b[i] = __builtin_amdgcn_fmed3f(b[i - 1], b[i], v);
  b[0] = __int_as_float(min(__float_as_int(b[0]), __float_as_int(v)));
}

// s0 = min(a0, a1, a2, a3), which the caller has already computed for its test.
template <int KP>
__device__ __forceinline__ void topk_insert4(float (&b)[KP], unsigned a0, unsigned a1, unsigned a2,
                                             unsigned a3, unsigned s0) {
  const unsigned p = min(a0, a1), q = max(a0, a1), r = min(a2, a3), t = max(a2, a3);
  const unsigned mid_lo = max(p, r), mid_hi = min(q, t);
  const unsigned s1 = min(mid_lo, mid_hi);
  topk_insert_sorted<KP>(b, __uint_as_float(s0));
  if (__builtin_amdgcn_ballot_w64(s1 < __float_as_uint(b[KP - 1])) != 0) {
    topk_insert_sorted<KP>(b, __uint_as_float(s1));
    topk_insert_sorted<KP>(b, __uint_as_float(max(mid_lo, mid_hi)));
    topk_insert_sorted<KP>(b, __uint_as_float(max(q, t)));
  }
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Tile epilogue shared by all shapes: self correction, optional per-point outputs,
// FP64 digamma terms, deterministic block reduction, one partial per work item.
__device__ __forceinline__ void tile_epilogue(const KSG_AS4 ProbDesc* pd, int tile, int qi,
                                              bool valid, float eps, int cxz, int cyz, int cz,
                                              bool z_empty, const double* __restrict__ htab,
                                              double* __restrict__ partials, double* s_red) {
  const int n = pd->n;
  const int self = eps > 0.0f ? 1 : 0;
  // Clamped at 0 so that table reads stay in range even for non-finite data (whose
  // self-distance is NaN) when the finite check has been switched off.
  const int nxz = max(cxz - self, 0);
  const int nyz = max(cyz - self, 0);
  const int nz = z_empty ? (self ? n - 1 : 0) : max(cz - self, 0);
  double t = 0.0;
  if (valid) {
    t = (htab[nxz] + htab[nyz]) - htab[nz];
    float* eo = pd->eps_out;
    int32_t* co = pd->counts_out;
    double* lo = pd->local_out;
    if (eo) eo[qi] = eps;
    if (co) {
      const int sw = pd->swap_xy;
      co[qi] = sw ? nyz : nxz;
      co[n + qi] = sw ? nxz : nyz;
      co[2 * n + qi] = nz;
    }
    if (lo) lo[qi] = htab[pd->k - 1] - t;
  }
  t = wave_sum(t);
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) s_red[wave] = t;
  __syncthreads();
  // fixed-order sum over the tile's 1, 2 or 4 waves (the tile height is the block size)
  if (threadIdx.x == 0) {
    const int nw = (int)blockDim.x >> 6;
    partials[pd->part_base + tile] =
        nw == 4 ? (s_red[0] + s_red[1]) + (s_red[2] + s_red[3]) : (nw == 2 ? s_red[0] + s_red[1] : s_red[0]);
  }
}

// Pass 1: the (k+1) smallest joint distances, self included; returns eps_i.
template <int D, int KP, int U>
__device__ __forceinline__ float radius_pass(const cfptr (&col)[D], const float (&q)[D], int n_pad, int k) {
  float b[KP];
#pragma unroll
  for (int i = 0; i < KP; ++i) b[i] = (i < KP - 1 - k) ? -INFINITY : INFINITY;

  for (int j = 0; j < n_pad; j += U) {
    float d[U];
#pragma unroll
    for (int u = 0; u < U; ++u) d[u] = fabsf(col[0][j + u] - q[0]);
#pragma unroll
    for (int a = 1; a < D; ++a) {
#pragma unroll
      for (int u = 0; u < U; ++u) d[u] = fmaxf(d[u], fabsf(col[a][j + u] - q[a]));
    }
    bool hit = false;
#pragma unroll
    for (int u = 0; u < U; ++u) hit |= d[u] < b[KP - 1];
    if (hit) {
#pragma unroll
      for (int u = 0; u < U; ++u) topk_insert<KP>(b, d[u]);
    }
  }
  return b[KP - 1];
}

// Pass 2: strict counts in XZ, YZ and Z (self included, removed in the epilogue), for a
// compile-time split of the D = DX + DY + DZ columns.  One accumulator per unrolled reference
// keeps every count a compare + add-with-carry.
struct Counts {
  int xz, yz, z;
};

template <int DX, int DY, int DZ, int U>
__device__ __forceinline__ Counts count_pass(const cfptr (&col)[DX + DY + DZ], const float (&q)[DX + DY + DZ],
                                             int n_pad, float eps) {
  constexpr int D = DX + DY + DZ;
  unsigned axz[U], ayz[U], az[U];
#pragma unroll
  for (int u = 0; u < U; ++u) axz[u] = ayz[u] = az[u] = 0u;
  for (int j = 0; j < n_pad; j += U) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      float A = fabsf(col[0][j + u] - q[0]);
#pragma unroll
      for (int a = 1; a < DX; ++a) A = fmaxf(A, fabsf(col[a][j + u] - q[a]));
      float B = fabsf(col[DX][j + u] - q[DX]);
#pragma unroll
      for (int a = DX + 1; a < DX + DY; ++a) B = fmaxf(B, fabsf(col[a][j + u] - q[a]));
      if constexpr (DZ > 0) {
        float C = fabsf(col[DX + DY][j + u] - q[DX + DY]);
#pragma unroll
        for (int a = DX + DY + 1; a < D; ++a) C = fmaxf(C, fabsf(col[a][j + u] - q[a]));
        axz[u] += (unsigned)(fmaxf(A, C) < eps);
        ayz[u] += (unsigned)(fmaxf(B, C) < eps);
        az[u] += (unsigned)(C < eps);
      } else {
        axz[u] += (unsigned)(A < eps);
        ayz[u] += (unsigned)(B < eps);
      }
    }
  }
  Counts c{0, 0, 0};
#pragma unroll
  for (int u = 0; u < U; ++u) {
    c.xz += (int)axz[u];
    c.yz += (int)ayz[u];
    c.z += (int)az[u];
  }
  return c;
}

// Pass 2 for a split known only at run time: subspace membership per column by selects.
template <int D>
__device__ __forceinline__ Counts count_pass_split(const cfptr (&col)[D], const float (&q)[D], int n_pad,
                                                   float eps, int dx, int dy) {
  constexpr int U = 4;
  int cxz = 0, cyz = 0, cz = 0;
  for (int j = 0; j < n_pad; j += U) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      float A = 0.0f, B = 0.0f, C = 0.0f;
#pragma unroll
      for (int a = 0; a < D; ++a) {
        const float t = fabsf(col[a][j + u] - q[a]);
        if (a < dx) A = fmaxf(A, t);
        else if (a < dx + dy) B = fmaxf(B, t);
        else C = fmaxf(C, t);
      }
      cxz += fmaxf(A, C) < eps;
      cyz += fmaxf(B, C) < eps;
      cz += C < eps;
    }
  }
  return Counts{cxz, cyz, cz};
}

// Pass 2 for dx == 1 and a wave-uniform dy in [DY, D): one compile-time count loop per dy,
// selected once per tile, so the reference loop carries no per-column selects.
template <int D, int DY, int U>
__device__ __forceinline__ Counts count_pass_dx1(const cfptr (&col)[D], const float (&q)[D], int n_pad,
                                                 float eps, int dy) {
  if constexpr (DY < D - 1) {
    if (dy == DY) return count_pass<1, DY, D - 1 - DY, U>(col, q, n_pad, eps);
    return count_pass_dx1<D, DY + 1, U>(col, q, n_pad, eps, dy);
  } else {
    return count_pass<1, D - 1, 0, U>(col, q, n_pad, eps);  // dy == D - 1: no Z
  }
}

// Fast path: compile-time subspace dimensions.
template <int DX, int DY, int DZ, int KP, int U>
__device__ __forceinline__ void search_tile(const KSG_AS4 ProbDesc* pd, int tile,
                                            const double* __restrict__ htab,
                                            double* __restrict__ partials, double* s_red) {
  constexpr int D = DX + DY + DZ;
  const int n = pd->n;
  const int n_pad = pd->n_pad;
  const int k = pd->k;
  const int qraw = tile * (int)blockDim.x + (int)threadIdx.x;
  const bool valid = qraw < n;
  const int qi = valid ? qraw : n - 1;

  cfptr col[D];
  float q[D];
#pragma unroll
  for (int a = 0; a < D; ++a) {
    const float* c = pd->col[a];
    col[a] = (cfptr)c;
    q[a] = c[qi];
  }
  const float eps = radius_pass<D, KP, U>(col, q, n_pad, k);
  const Counts c = count_pass<DX, DY, DZ, U>(col, q, n_pad, eps);
  tile_epilogue(pd, tile, qi, valid, eps, c.xz, c.yz, c.z, DZ == 0, htab, partials, s_red);
}

// Dimension-count path: D columns with the split known at run time.  The canonical split has
// dx <= dy, so dx == 1 (the usual case: one target variable against several sources, or one
// source against several conditioning columns) gets compile-time count loops; any other split
// counts with per-column selects.
template <int D, int KP>
__device__ __forceinline__ void search_tile_dims(const KSG_AS4 ProbDesc* pd, int tile,
                                                 const double* __restrict__ htab,
                                                 double* __restrict__ partials, double* s_red) {
  constexpr int U = D <= 8 ? 8 : 4;
  const int n = pd->n;
  const int n_pad = pd->n_pad;
  const int k = pd->k;
  const int dx = pd->dx, dy = pd->dy;
  const int qraw = tile * (int)blockDim.x + (int)threadIdx.x;
  const bool valid = qraw < n;
  const int qi = valid ? qraw : n - 1;
  cfptr col[D];
  float q[D];
#pragma unroll
  for (int a = 0; a < D; ++a) {
    const float* c = pd->col[a];
    col[a] = (cfptr)c;
    q[a] = c[qi];
  }
  const float eps = radius_pass<D, KP, U>(col, q, n_pad, k);
  const Counts c = dx == 1 ? count_pass_dx1<D, 1, U>(col, q, n_pad, eps, dy)
                           : count_pass_split<D>(col, q, n_pad, eps, dx, dy);
  tile_epilogue(pd, tile, qi, valid, eps, c.xz, c.yz, c.z, dx + dy == D, htab, partials, s_red);
}

// Generic path: any split of up to kMaxDimsCompiled dimensions, subspace membership resolved
// with wave-uniform selects.  Used for shapes outside the fast table.
template <int D, int KP>
__device__ __forceinline__ void search_tile_generic(const KSG_AS4 ProbDesc* pd, int tile,
                                                    const double* __restrict__ htab,
                                                    double* __restrict__ partials,
                                                    double* s_red) {
  constexpr int U = 4;
  const int n = pd->n;
  const int n_pad = pd->n_pad;
  const int k = pd->k;
  const int dx = pd->dx, dy = pd->dy;
  const int qraw = tile * (int)blockDim.x + (int)threadIdx.x;
  const bool valid = qraw < n;
  const int qi = valid ? qraw : n - 1;
  cfptr col[D];
  float q[D];
#pragma unroll
  for (int a = 0; a < D; ++a) {
    const float* c = pd->col[a];
    col[a] = (cfptr)c;
    q[a] = c[qi];
  }
  const float eps = radius_pass<D, KP, U>(col, q, n_pad, k);
  const bool z_empty = (dx + dy == D);
  const Counts c = count_pass_split<D>(col, q, n_pad, eps, dx, dy);
  const int cxz = c.xz, cyz = c.yz, cz = c.z;
  tile_epilogue(pd, tile, qi, valid, eps, cxz, cyz, cz, z_empty, htab, partials, s_red);
}

// Fast-shape dispatch: shape = pair * (kFastMaxDz + 1) + dz.
template <int KP>
__device__ __forceinline__ void dispatch_fast(int shape, const KSG_AS4 ProbDesc* pd, int tile,
                                              const double* __restrict__ htab,
                                              double* __restrict__ partials, double* s_red);

#define KSG_FAST_CASE(PAIR, DXv, DYv, DZv)                                                      \
  case (PAIR) * (kFastMaxDz + 1) + (DZv):                                                       \
    search_tile<DXv, DYv, DZv, KP, ((DXv + DYv + DZv) <= 8 ? 8 : 4)>(pd, tile, htab, partials, \
                                                                     s_red);                    \
    break;

#define KSG_FAST_PAIR(PAIR, DXv, DYv)                                                \
  KSG_FAST_CASE(PAIR, DXv, DYv, 0) KSG_FAST_CASE(PAIR, DXv, DYv, 1)                  \
  KSG_FAST_CASE(PAIR, DXv, DYv, 2) KSG_FAST_CASE(PAIR, DXv, DYv, 3)                  \
  KSG_FAST_CASE(PAIR, DXv, DYv, 4) KSG_FAST_CASE(PAIR, DXv, DYv, 5)                  \
  KSG_FAST_CASE(PAIR, DXv, DYv, 6) KSG_FAST_CASE(PAIR, DXv, DYv, 7)                  \
  KSG_FAST_CASE(PAIR, DXv, DYv, 8) KSG_FAST_CASE(PAIR, DXv, DYv, 9)                  \
  KSG_FAST_CASE(PAIR, DXv, DYv, 10) KSG_FAST_CASE(PAIR, DXv, DYv, 11)                \
  KSG_FAST_CASE(PAIR, DXv, DYv, 12)

#define KSG_GENERIC_CASE(Dv) \
  case Dv:                   \
    search_tile_generic<Dv, KP>(pd, tile, htab, partials, s_red); \
    break;

template <int KP>
__device__ __forceinline__ void dispatch_generic(int D, const KSG_AS4 ProbDesc* pd, int tile,
                                                 const double* __restrict__ htab,
                                                 double* __restrict__ partials, double* s_red) {
  switch (D) {
    KSG_GENERIC_CASE(2) KSG_GENERIC_CASE(3) KSG_GENERIC_CASE(4) KSG_GENERIC_CASE(5)
    KSG_GENERIC_CASE(6) KSG_GENERIC_CASE(7) KSG_GENERIC_CASE(8) KSG_GENERIC_CASE(9)
    KSG_GENERIC_CASE(10) KSG_GENERIC_CASE(11) KSG_GENERIC_CASE(12) KSG_GENERIC_CASE(13)
    KSG_GENERIC_CASE(14) KSG_GENERIC_CASE(15) KSG_GENERIC_CASE(16)
    default: break;
  }
}

// Batched kernel: one work-group per work item (problem, query tile).  The tile height is the
// work-group size, 64, 128 or 256 queries (one per lane), chosen per launch by the autotuner;
// the window and algorithm-2 kernels keep 256 (their epilogue reads four waves).  The host orders
// the items longest-problem-first and the hardware dispatcher hands work-groups to compute
// units in that order as they free up, which gives the dynamic longest-first schedule of a
// work queue without a device-side queue.  SHAPE in [0, kGenericShape): every problem of the
// launch has that fast shape; SHAPE == kGenericShape + D: every problem is a generic shape of D
// columns; SHAPE == -1: mixed batch, per-problem dispatch.
template <int SHAPE, int KP>
__global__ __launch_bounds__(kTileQ) void ksg_batch_kernel(const ProbDesc* __restrict__ descs,
                                                           const WorkItem* __restrict__ items,
                                                           const double* __restrict__ htab,
                                                           double* __restrict__ partials) {
  __shared__ double s_red[kTileQ / 64];
  const KSG_AS4 ProbDesc* d4 = (const KSG_AS4 ProbDesc*)descs;
  const KSG_AS4 WorkItem* i4 = (const KSG_AS4 WorkItem*)items;
  const int it = blockIdx.x;
  const int prob = i4[it].prob;
  if (prob < 0) return;
  const int tile = i4[it].tile;
  const KSG_AS4 ProbDesc* pd = d4 + prob;
  if constexpr (SHAPE >= kGenericShape + 2) {
    search_tile_dims<SHAPE - kGenericShape, KP>(pd, tile, htab, partials, s_red);
  } else if constexpr (SHAPE >= 0 && SHAPE < kGenericShape) {
    constexpr int PAIR = SHAPE / (kFastMaxDz + 1);
    constexpr int DZ = SHAPE % (kFastMaxDz + 1);
    constexpr int DX = PAIR == 2 ? 2 : 1;
    constexpr int DY = PAIR == 0 ? 1 : 2;
    search_tile<DX, DY, DZ, KP, ((DX + DY + DZ) <= 8 ? 8 : 4)>(pd, tile, htab, partials, s_red);
  } else {
    const int shape = pd->variant;
    if (shape >= kGenericShape) {
      dispatch_generic<KP>(pd->dx + pd->dy + pd->dz, pd, tile, htab, partials, s_red);
    } else {
      switch (shape) {
        KSG_FAST_PAIR(0, 1, 1)
        KSG_FAST_PAIR(1, 1, 2)
        KSG_FAST_PAIR(2, 2, 2)
        default: break;
      }
    }
  }
}

}  // namespace ksg
