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
#pragma once
#include <climits>

#include "ksg_search.inc.h"

namespace ksg {

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

// Per-space max-norm distances of reference row j (X, Y, Z), compile-time split.
template <int DX, int DY, int D>
__device__ __forceinline__ void space_dists(const cfptr (&col)[D], const float (&q)[D], int j, float& A, float& B,
                                            float& C) {
  A = fabsf(col[0][j] - q[0]);
#pragma unroll
  for (int a = 1; a < DX; ++a) A = fmaxf(A, fabsf(col[a][j] - q[a]));
  B = fabsf(col[DX][j] - q[DX]);
#pragma unroll
  for (int a = DX + 1; a < DX + DY; ++a) B = fmaxf(B, fabsf(col[a][j] - q[a]));
  C = 0.0f;
#pragma unroll
  for (int a = DX + DY; a < D; ++a) C = fmaxf(C, fabsf(col[a][j] - q[a]));
}

// The same for a split known only at run time (per-column selects).
template <int D>
__device__ __forceinline__ void space_dists_rt(const cfptr (&col)[D], const float (&q)[D], int j, int dx, int dy,
                                               float& A, float& B, float& C) {
  A = B = C = 0.0f;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    const float t = fabsf(col[a][j] - q[a]);
    if (a < dx) A = fmaxf(A, t);
    else if (a < dx + dy) B = fmaxf(B, t);
    else C = fmaxf(C, t);
  }
}

// KSG algorithm 2 in key order, after the (k+1)-th smallest joint distance eps (self
// included, so eps is the k-th neighbour's distance) is known for every lane:
//  sides pass: the neighbours are the rows j != i with d_ij < eps and, of those with
//    d_ij == eps, the ones with the lowest source rows (as many as make k); the rectangle
//    sides are the largest X, Y and Z distances over them.  A row with d_ij <= eps has
//    |key gap| <= eps, so the window of eps (gaps <= eps) holds them all; ties go through a
//    short list of source rows (key_order) kept sorted, taken only when a lane meets one.
//  count pass: n_S = #{j : d^S_ij <= e^S and d^Z_ij <= e^Z} with self included (subtracted
//    later); every counted row has |key gap| <= e^Z.
template <int DX, int DY, int D, int T, class OpenR, class OpenL>
__device__ __forceinline__ void alg2_sides_pass(const cfptr (&col)[D], const float (&q)[D], int dx, int dy, int qi,
                                                float eps, const int32_t* __restrict__ korder, int s_lo, int s_hi,
                                                int steps, OpenR open_r, OpenL open_l, float& ex, float& ey,
                                                float& ez, int& c_less, int (&ti)[T], float (&tx)[T],
                                                float (&ty)[T], float (&tz)[T], unsigned& n_steps) {
  auto step = [&](int s) {
    float A[4], B[4], C[4], d[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if constexpr (DX > 0) space_dists<DX, DY, D>(col, q, 4 * s + u, A[u], B[u], C[u]);
      else space_dists_rt<D>(col, q, 4 * s + u, dx, dy, A[u], B[u], C[u]);
      d[u] = fmaxf(fmaxf(A[u], B[u]), C[u]);
    }
    bool near = false;
#pragma unroll
    for (int u = 0; u < 4; ++u) near |= d[u] <= eps;
    if (__builtin_amdgcn_ballot_w64(near) == 0) return;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int j = 4 * s + u;
      if (j == qi) continue;
      if (d[u] < eps) {
        ex = fmaxf(ex, A[u]);
        ey = fmaxf(ey, B[u]);
        ez = fmaxf(ez, C[u]);
        ++c_less;
      } else if (d[u] == eps) {
        // keep the T lowest source rows among the ties, sorted
        int r = korder[j];
        float a = A[u], bb = B[u], c = C[u];
#pragma unroll
        for (int t = 0; t < T; ++t) {
          if (r < ti[t]) {
            const int r0 = ti[t];
            const float a0 = tx[t], b0 = ty[t], c0 = tz[t];
            ti[t] = r;
            tx[t] = a;
            ty[t] = bb;
            tz[t] = c;
            r = r0;
            a = a0;
            bb = b0;
            c = c0;
          }
        }
      }
    }
  };
  window_scan(s_lo, s_hi, steps, step, open_r, open_l, n_steps);
}

template <int DX, int DY, int D, class OpenR, class OpenL>
__device__ __forceinline__ void alg2_count_pass(const cfptr (&col)[D], const float (&q)[D], int dx, int dy,
                                                float ex, float ey, float ez, int s_lo, int s_hi, int steps,
                                                OpenR open_r, OpenL open_l, unsigned (&acc)[3],
                                                unsigned& n_steps) {
  auto step = [&](int s) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      float A, B, C;
      if constexpr (DX > 0) space_dists<DX, DY, D>(col, q, 4 * s + u, A, B, C);
      else space_dists_rt<D>(col, q, 4 * s + u, dx, dy, A, B, C);
      const bool cz = C <= ez;
      acc[0] += (unsigned)((A <= ex) & cz);
      acc[1] += (unsigned)((B <= ey) & cz);
      acc[2] += (unsigned)cz;
    }
  };
  window_scan(s_lo, s_hi, steps, step, open_r, open_l, n_steps);
}

// Sides pass, the ties that complete the k neighbours, then the count pass, for one split.
template <int DX, int DY, int D, int T, class OpenR3, class OpenL3, class OpenRC, class OpenLC>
__device__ __forceinline__ void alg2_rect(const cfptr (&col)[D], const float (&q)[D], int dx, int dy, int qi, int k,
                                          float eps, const int32_t* __restrict__ korder, int s_lo, int s_hi,
                                          int steps, OpenR3 open_r3, OpenL3 open_l3, OpenRC open_rc,
                                          OpenLC open_lc, float& ez, unsigned (&acc)[3], unsigned& n3,
                                          unsigned& n2) {
  float ex = 0.0f, ey = 0.0f;
  ez = 0.0f;
  int c_less = 0;
  int ti[T];
  float tx[T], ty[T], tz[T];
#pragma unroll
  for (int t = 0; t < T; ++t) {
    ti[t] = INT_MAX;
    tx[t] = ty[t] = tz[t] = 0.0f;
  }
  alg2_sides_pass<DX, DY, D>(col, q, dx, dy, qi, eps, korder, s_lo, s_hi, steps, open_r3, open_l3, ex, ey, ez,
                             c_less, ti, tx, ty, tz, n3);
  // the ties with the lowest source rows complete the k neighbours
  const int need = k - c_less;
#pragma unroll
  for (int t = 0; t < T; ++t) {
    if (t < need && ti[t] != INT_MAX) {
      ex = fmaxf(ex, tx[t]);
      ey = fmaxf(ey, ty[t]);
      ez = fmaxf(ez, tz[t]);
    }
  }
  alg2_count_pass<DX, DY, D>(col, q, dx, dy, ex, ey, ez, s_lo, s_hi, steps, open_rc, open_lc, acc, n2);
}

// dx == 1 and a wave-uniform dy in [DY, D - 2] (dz >= 1): one compile-time split per dy.
template <int D, int DY, int T, class OpenR3, class OpenL3, class OpenRC, class OpenLC>
__device__ __forceinline__ void alg2_rect_dx1(const cfptr (&col)[D], const float (&q)[D], int dy, int qi, int k,
                                              float eps, const int32_t* __restrict__ korder, int s_lo, int s_hi,
                                              int steps, OpenR3 open_r3, OpenL3 open_l3, OpenRC open_rc,
                                              OpenLC open_lc, float& ez, unsigned (&acc)[3], unsigned& n3,
                                              unsigned& n2) {
  if constexpr (DY < D - 2) {
    if (dy == DY) {
      alg2_rect<1, DY, D, T>(col, q, 1, dy, qi, k, eps, korder, s_lo, s_hi, steps, open_r3, open_l3, open_rc,
                             open_lc, ez, acc, n3, n2);
      return;
    }
    alg2_rect_dx1<D, DY + 1, T>(col, q, dy, qi, k, eps, korder, s_lo, s_hi, steps, open_r3, open_l3, open_rc,
                                open_lc, ez, acc, n3, n2);
  } else {
    alg2_rect<1, D - 2, D, T>(col, q, 1, dy, qi, k, eps, korder, s_lo, s_hi, steps, open_r3, open_l3, open_rc,
                              open_lc, ez, acc, n3, n2);
  }
}

template <int D, int KP, int ALG>
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
  if constexpr (ALG == 1) {
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
    // per-point outputs are indexed by the problem's own rows: row qi of the key order is row
    // key_order[qi] of the problem
    const bool outputs = pd->eps_out || pd->counts_out || pd->local_out;
    const int orow = valid && outputs ? pd->key_order[qi] : qi;
    tile_epilogue(pd, tile, orow, valid, eps, (int)acc[0], (int)acc[1], (int)acc[2], dx + dy == D, htab, partials,
                  s_red);
  } else {
    constexpr int T = KP - 1;  // >= k: ties kept at the k-th distance
    const int32_t* korder = pd->key_order;
    // rows at a gap equal to eps can tie with it, so the windows keep gaps <= eps (sides) and
    // <= e^Z (counts, e^Z is per lane)
    float ez = 0.0f;
    auto open_r3 = [&](int s) { return __builtin_amdgcn_ballot_w64(fabsf(kcol[4 * s] - qkey) <= eps) != 0; };
    auto open_l3 = [&](int s) { return __builtin_amdgcn_ballot_w64(fabsf(kcol[4 * s + 3] - qkey) <= eps) != 0; };
    auto open_rc = [&](int s) { return __builtin_amdgcn_ballot_w64(fabsf(kcol[4 * s] - qkey) <= ez) != 0; };
    auto open_lc = [&](int s) { return __builtin_amdgcn_ballot_w64(fabsf(kcol[4 * s + 3] - qkey) <= ez) != 0; };
    unsigned acc[3] = {0u, 0u, 0u};
    unsigned n3 = 0;
    bool done = false;
    if constexpr (D >= 3) {  // a window problem has dy >= 1 and dz >= 1
      if (dx == 1) {
        alg2_rect_dx1<D, 1, T>(col, q, dy, qi, k, eps, korder, s_lo, s_hi, steps, open_r3, open_l3, open_rc,
                               open_lc, ez, acc, n3, n2);
        done = true;
      }
    }
    if (!done)
      alg2_rect<0, 0, D, T>(col, q, dx, dy, qi, k, eps, korder, s_lo, s_hi, steps, open_r3, open_l3, open_rc,
                            open_lc, ez, acc, n3, n2);
    if (work && (threadIdx.x & 63) == 0)
      atomicAdd(&work[5], (unsigned long long)(n1 + n3) * (unsigned)(2 * D) +
                              (unsigned long long)n2 * (unsigned)(2 * D + 2));
    // self is inside every rectangle; clamped as in the brute-force kernel
    const int nxz = max((int)acc[0] - 1, 1);
    const int nyz = max((int)acc[1] - 1, 1);
    const int nz = max((int)acc[2] - 1, 1);
    double t = 0.0;
    if (valid)
      t = -(((htab[nz - 1] - htab[nxz - 1]) - htab[nyz - 1]) + (1.0 / (double)nxz + 1.0 / (double)nyz));
    t = wave_sum(t);
    if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = t;
    __syncthreads();
    if (threadIdx.x == 0) partials[pd->part_base + tile] = (s_red[0] + s_red[1]) + (s_red[2] + s_red[3]);
  }
}

}  // namespace ksg
