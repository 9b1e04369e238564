// Grouped search kernels: G CMI problems that share Y, Z, N and k and differ only in their
// one-dimensional X column (the candidates and permutation surrogates of one greedy step)
// are searched together, one 256-query tile per work-group.
//
// For every ordered pair (i, j) the Y/Z part of the max-norm distance,
//   d^YZ_ij = max(|y_j - y_i|, |z_j1 - z_i1|, ..., |z_jm - z_im|),
// is the same for all G problems, so it is computed once per pair and reused:
//   joint  d_ij(g)    = max(|x_g,j - x_g,i|, d^YZ_ij)          (radius eps_i(g))
//   counts d^XZ_ij(g) = max(|x_g,j - x_g,i|, d^Z_ij)           (n_XZ)
// The counts n_YZ and n_Z do not involve X at all: they are functions of the query and the
// radius only, evaluated for every problem of the Y/Z set at once by the Y/Z count kernel
// (ksg_yzcount.hip), which hands each problem's H(n_YZ) - H(n_Z) term to the X count kernel
// below.  So a greedy step runs three launches: radius (eps of every problem and row, to a
// buffer E), Y/Z counts (terms to a buffer T), X counts (n_XZ, the sum of the terms).
// Every distance, radius and count is bit-identical to the single-problem kernel (the same
// FP32 subtractions and exact maxima, only evaluated once instead of G times).  The rows are
// searched in the order of a key column, which bounds each wave's scan to a window of rows
// (below) without changing any radius or count; only the order in which the FP64 per-point
// terms are summed differs from the single-problem kernel.  Column data come from one device
// pool through 32-bit offsets held in SGPRs; references arrive through the scalar data path
// as in the single-problem kernel.
#pragma once

#include "ksg_search.inc.h"

namespace ksg {

typedef float ksg_f4 __attribute__((ext_vector_type(4)));
typedef const KSG_AS4 ksg_f4* cf4ptr;

// Interleaved group blocks (written by the interleave kernel from the packed columns):
//   X block  [n_pad/4][G][4]:   the G candidate columns, four references at a time,
//   YZ block [n_pad/4][M+1][4]: Y then the M conditioning columns, four references at a time.
// One step of U = 4 references reads G + M + 1 consecutive float4 values from two pointers,
// so the scalar loads of a step share two base registers and are issued together.
//
// Key window.  The rows are in ascending order of the key column (Z_1, or Y when m = 0),
// and the 64 queries of a wave are consecutive rows.  Every distance of the search is at
// least |k_j - k_i| (a coordinate difference in the max norm), and because FP32 rounding is
// monotone, fl(k_j - k_i) >= fl(k_b - k_i) for every row j beyond a boundary row b on the
// far side of the query.  So once the first key of a step to the right (the last key of a
// step to the left) is at least a lane's bound away from that lane's key, for every lane, no
// later step in that direction can change the wave's results: the scan in that direction
// ends there.  The radius kernel scans the wave's own rows first, then alternates right and
// left (so that the radii shrink early); the X count kernel scans right, then left.
struct WaveRange {
  int s_lo, s_hi;  // the wave's own reference steps (inclusive), s_hi < s_lo when idle
  bool live;
};

__device__ __forceinline__ WaveRange wave_range(int tile, int n) {
  const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
  const int w0 = tile * kTileQ + wave * 64;
  WaveRange r;
  r.live = w0 < n;
  r.s_lo = r.live ? (w0 >> 2) : 0;
  r.s_hi = r.live ? (min(w0 + 63, n - 1) >> 2) : -1;
  return r;
}

// ---- radius kernel: (k+1) smallest joint distances per problem, self included ----
// max(|t|, dyz) is taken as med3(|t|, dyz, +inf) and the "any candidate below the radius"
// test as an unsigned minimum of the (non-negative) distance bit patterns: neither form needs
// the NaN-quieting copies that an IEEE-mode maximum of a value from another basic block would
// get, and both give exactly the maximum / comparison of the values.
// Exact skips: d(g) = max(|dx_g|, dyz) >= dyz, so when dyz >= radius_g for all four
// references and every lane of the wave, problem g cannot gain a neighbour in the step; when
// that holds for bmax = max_g radius_g the whole step is skipped.
// Two phases.  Phase 1: every wave scans all rows of its tile and of the two neighbouring
// tiles for its own 64 queries, which leaves each query's top-(k+1) lists over those rows and
// so an upper bound on each radius.
// Then the tile's queries are handed to the waves again in ascending order of their largest
// bound (the lists travel through LDS), so that a wave's window is not widened by a few wide
// queries among narrow ones.  Phase 2: each wave scans outward from the tile, alternating right
// and left, with the key window of its current radii.  Every row is examined exactly once per
// query, so the radii are those of a full scan.
// Output: E[e_off + row * G + g] = eps of problem g at (key-ordered) row, rows < n.
constexpr int kXchg = 20;  // floats per lane per LDS exchange round
template <int M, int G, int KP>
__device__ __forceinline__ void group_radius_tile(const float* __restrict__ base,
                                                  const KSG_AS4 GroupDesc* gd, int tile,
                                                  float* __restrict__ E,
                                                  unsigned long long* __restrict__ s_ord,
                                                  float (*s_x)[kTileQ],
                                                  unsigned long long* __restrict__ work) {
  constexpr int U = 4;
  constexpr int W = M + 1;
  constexpr int KC = M > 0 ? 1 : 0;  // key column in the YZ block
  const int n = gd->n;
  const int n_pad = gd->n_pad;
  const int k = gd->k;
  const int ng = gd->ng;
  const int tid = (int)threadIdx.x;
  int qi = min(tile * kTileQ + tid, n - 1);
  bool valid = tile * kTileQ + tid < n;

  const float* xi = base + gd->xi_off;
  const float* yzi = base + gd->yzi_off;
  const cf4ptr px = (cf4ptr)xi;
  const cf4ptr pyz = (cf4ptr)yzi;
  float qx[G], qz[M > 0 ? M : 1], qy, qkey;
  auto load_query = [&]() {
    const int qs = qi >> 2, ql = qi & 3;
#pragma unroll
    for (int g = 0; g < G; ++g) qx[g] = xi[(qs * G + g) * 4 + ql];
    qy = yzi[(qs * W) * 4 + ql];
#pragma unroll
    for (int a = 0; a < M; ++a) qz[a] = yzi[(qs * W + 1 + a) * 4 + ql];
    qkey = M > 0 ? qz[0] : qy;
  };
  load_query();
  const int steps = n_pad / U;
  const WaveRange wr = wave_range(tile, n);

  float b[G][KP];
#pragma unroll
  for (int g = 0; g < G; ++g)
#pragma unroll
    for (int i = 0; i < KP; ++i) b[g][i] = (i < KP - 1 - k) ? -INFINITY : INFINITY;

  unsigned bmax = __float_as_uint(INFINITY);
  unsigned done = 0;    // problem-steps whose per-problem work ran (wave-uniform)
  const unsigned gmask = (1u << ng) - 1u;  // the group's real problems (ng <= 16)
  unsigned shared = 0;  // shared-part operations / 256 (wave-uniform)

  // One reference step s; dir != 0: a window step, skipped (returns true) when every lane's
  // key gap reaches its bound.
  auto step = [&](int s, int dir) -> bool {
    // the step's X block is requested first so that its latency overlaps the Y/Z work
    ksg_f4 rx[G];
#pragma unroll
    for (int g = 0; g < G; ++g) rx[g] = px[s * G + g];
    // |key differences| first: they give the window test (a step to the right starts with
    // its smallest key, a step to the left ends with its largest, and fl(a - b) = -fl(b - a))
    // and are the first term of d^YZ
    const ksg_f4 rk = pyz[s * W + KC];
    float dyz[U] = {fabsf(rk.x - qkey), fabsf(rk.y - qkey), fabsf(rk.z - qkey), fabsf(rk.w - qkey)};
    if (dir != 0) {
      const float gap = dir > 0 ? dyz[0] : dyz[3];
      if (__builtin_amdgcn_ballot_w64(__float_as_uint(gap) < bmax) == 0) return true;
    }
    shared += 2 * M + 2;
    if constexpr (M > 0) {
      const ksg_f4 ry = pyz[s * W];
      dyz[0] = fmaxf(dyz[0], fabsf(ry.x - qy));
      dyz[1] = fmaxf(dyz[1], fabsf(ry.y - qy));
      dyz[2] = fmaxf(dyz[2], fabsf(ry.z - qy));
      dyz[3] = fmaxf(dyz[3], fabsf(ry.w - qy));
    }
#pragma unroll
    for (int a = 1; a < M; ++a) {
      const ksg_f4 rz = pyz[s * W + 1 + a];
      dyz[0] = fmaxf(dyz[0], fabsf(rz.x - qz[a]));
      dyz[1] = fmaxf(dyz[1], fabsf(rz.y - qz[a]));
      dyz[2] = fmaxf(dyz[2], fabsf(rz.z - qz[a]));
      dyz[3] = fmaxf(dyz[3], fabsf(rz.w - qz[a]));
    }
    const unsigned dmin = min(min(__float_as_uint(dyz[0]), __float_as_uint(dyz[1])),
                              min(__float_as_uint(dyz[2]), __float_as_uint(dyz[3])));
    if (__builtin_amdgcn_ballot_w64(dmin < bmax) == 0) return false;
    unsigned act = 0;  // problems whose work ran in this step (bit g; wave-uniform, kept scalar)
#pragma unroll
    for (int g = 0; g < G; ++g) {
      if (__builtin_amdgcn_ballot_w64(dmin < __float_as_uint(b[g][KP - 1])) == 0) continue;
      act |= 1u << g;
      float d[U];
      d[0] = __builtin_amdgcn_fmed3f(fabsf(rx[g].x - qx[g]), dyz[0], INFINITY);
      d[1] = __builtin_amdgcn_fmed3f(fabsf(rx[g].y - qx[g]), dyz[1], INFINITY);
      d[2] = __builtin_amdgcn_fmed3f(fabsf(rx[g].z - qx[g]), dyz[2], INFINITY);
      d[3] = __builtin_amdgcn_fmed3f(fabsf(rx[g].w - qx[g]), dyz[3], INFINITY);
      // chained so that it is one v_min_u32 and one v_min3_u32
      const unsigned lo = min(min(min(__float_as_uint(d[0]), __float_as_uint(d[1])), __float_as_uint(d[2])),
                              __float_as_uint(d[3]));
      if (lo < __float_as_uint(b[g][KP - 1]))
        topk_insert4<KP>(b[g], __float_as_uint(d[0]), __float_as_uint(d[1]), __float_as_uint(d[2]),
                         __float_as_uint(d[3]), lo);
    }
    done += __builtin_popcount(__builtin_amdgcn_readfirstlane(act) & gmask);
    bmax = __float_as_uint(b[0][KP - 1]);
#pragma unroll
    for (int g = 1; g < G; ++g) bmax = max(bmax, __float_as_uint(b[g][KP - 1]));
    return false;
  };

  // ---- phase 1: the tile's rows and those of its two neighbouring tiles ----
  const int real_steps = (n + U - 1) / U;                  // steps holding real rows
  const int t_lo = max(tile * (kTileQ / U) - kTileQ / U, 0);
  const int t_hi = min(tile * (kTileQ / U) + 2 * (kTileQ / U), real_steps) - 1;
  if (wr.live)
    for (int s = t_lo; s <= t_hi; ++s) step(s, 0);

  // ---- regroup the tile's queries by their largest bound ----
  {
    unsigned ub = __float_as_uint(b[0][KP - 1]);
#pragma unroll
    for (int g = 1; g < G; ++g) ub = max(ub, __float_as_uint(b[g][KP - 1]));
    s_ord[tid] = valid ? ((unsigned long long)ub << 32) | (unsigned)qi : ~0ull;
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
    const bool nvalid = kk != ~0ull;
    const int nrow = nvalid ? (int)(unsigned)(kk & 0xffffffffu) : n - 1;
    const int src = nvalid ? nrow - tile * kTileQ : tid;  // lane that held the row's lists
    constexpr int PR = kXchg / KP;                         // problems per exchange round
#pragma unroll
    for (int g0 = 0; g0 < G; g0 += PR) {
#pragma unroll
      for (int g = g0; g < g0 + PR && g < G; ++g)
#pragma unroll
        for (int i = 0; i < KP; ++i) s_x[(g - g0) * KP + i][tid] = b[g][i];
      __syncthreads();
#pragma unroll
      for (int g = g0; g < g0 + PR && g < G; ++g)
#pragma unroll
        for (int i = 0; i < KP; ++i) b[g][i] = s_x[(g - g0) * KP + i][src];
      __syncthreads();
    }
    valid = nvalid;
    qi = nrow;
    load_query();
    bmax = __float_as_uint(b[0][KP - 1]);
#pragma unroll
    for (int g = 1; g < G; ++g) bmax = max(bmax, __float_as_uint(b[g][KP - 1]));
  }

  // ---- phase 2: outward from the tile, alternating right and left ----
  {
    int r = t_hi + 1, l = t_lo - 1;
    bool ract = wr.live && r < steps, lact = wr.live && l >= 0, right_turn = true;
    for (;;) {
      int s, dir;
      if (ract && (right_turn || !lact)) {
        s = r;
        dir = 1;
      } else if (lact) {
        s = l;
        dir = -1;
      } else {
        break;
      }
      if (step(s, dir)) {
        if (dir > 0) ract = false;
        else lact = false;
        continue;
      }
      if (dir > 0) ract = ++r < steps;
      else lact = --l >= 0;
      right_turn = !right_turn;
    }
  }

  if (valid) {
    float* e = E + gd->e_off + (size_t)qi * G;
#pragma unroll
    for (int g = 0; g < G; g += 4)
      *reinterpret_cast<ksg_f4*>(e + g) = ksg_f4{b[g][KP - 1], b[g + 1][KP - 1], b[g + 2][KP - 1], b[g + 3][KP - 1]};
  }
  if (work && (threadIdx.x & 63) == 0) {
    // work executed by this wave, in units of 4 references x 64 lanes
    atomicAdd(&work[0], (unsigned long long)done);
    atomicAdd(&work[2], (unsigned long long)shared);
  }
}

// ---- X count kernel: n_XZ = #{ j : max(|dx_g|, d^Z) < eps_g }, self included ----
// Every such pair has d^Z < eps_g, so a step in which d^Z >= eps_g for all references and
// lanes contributes nothing to problem g, and with d^Z >= |dk| the key window bounds the scan
// exactly.  Without Z (m = 0) the X counts are not bounded by the key (Y), and the scan
// covers every row.  Epilogue: term = H(n_XZ) + T[row][g] (T holds H(n_YZ) - H(n_Z)), summed
// over the tile into one partial per problem.
template <int M, int G>
__device__ __forceinline__ void group_xcount_tile(const float* __restrict__ base,
                                                  const KSG_AS4 GroupDesc* gd, int tile,
                                                  const float* __restrict__ E,
                                                  const double* __restrict__ T,
                                                  const double* __restrict__ htab,
                                                  double* __restrict__ partials,
                                                  double (*s_red)[G],
                                                  unsigned long long* __restrict__ s_ord,
                                                  unsigned long long* __restrict__ work) {
  constexpr int U = 4;
  constexpr int W = M + 1;
  const int n = gd->n;
  const int n_pad = gd->n_pad;
  const int ng = gd->ng;

  // Query regrouping: the tile's rows are handed to its four waves in ascending order of
  // their largest radius (ties by row), so that each wave's window, set by its largest
  // radius, is not widened by a few wide rows among narrow ones.  The rows of a wave are no
  // longer consecutive: its own steps span the rows from its smallest to its largest, and
  // the window scans start beyond them, which keeps the bounds exact.
  auto load_eps = [&](int row, float (&eps)[G]) {
    const float* e = E + gd->e_off + (size_t)row * G;
#pragma unroll
    for (int g = 0; g < G; g += 4) {
      const ksg_f4 v = *reinterpret_cast<const ksg_f4*>(e + g);
      eps[g] = v.x;
      eps[g + 1] = v.y;
      eps[g + 2] = v.z;
      eps[g + 3] = v.w;
    }
  };
  float eps[G];
  int qi;
  bool valid;
  {
    const int own = tile * kTileQ + (int)threadIdx.x;
    const bool own_valid = own < n;
    load_eps(own_valid ? own : n - 1, eps);
    unsigned em = __float_as_uint(eps[0]);
#pragma unroll
    for (int g = 1; g < G; ++g) em = max(em, __float_as_uint(eps[g]));
    s_ord[threadIdx.x] = own_valid ? ((unsigned long long)em << 32) | (unsigned)own : ~0ull;
    __syncthreads();
    for (int size = 2; size <= kTileQ; size <<= 1) {
      for (int stride = size >> 1; stride > 0; stride >>= 1) {
        const int t = threadIdx.x;
        if (t < kTileQ / 2) {
          const int lo = 2 * t - (t & (stride - 1));
          const int hi = lo + stride;
          const unsigned long long a = s_ord[lo], b = s_ord[hi];
          if ((a > b) == ((lo & size) == 0)) {
            s_ord[lo] = b;
            s_ord[hi] = a;
          }
        }
        __syncthreads();
      }
    }
    const unsigned long long kk = s_ord[threadIdx.x];
    valid = kk != ~0ull;
    qi = valid ? (int)(unsigned)(kk & 0xffffffffu) : n - 1;
    load_eps(qi, eps);
  }

  const float* xi = base + gd->xi_off;
  const float* yzi = base + gd->yzi_off;
  const cf4ptr px = (cf4ptr)xi;
  const cf4ptr pyz = (cf4ptr)yzi;
  float qx[G], qz[M > 0 ? M : 1];
  const int qs = qi >> 2, ql = qi & 3;
#pragma unroll
  for (int g = 0; g < G; ++g) qx[g] = xi[(qs * G + g) * 4 + ql];
#pragma unroll
  for (int a = 0; a < M; ++a) qz[a] = yzi[(qs * W + 1 + a) * 4 + ql];
  const int steps = n_pad / U;
  WaveRange wr = wave_range(tile, n);
  {
    // the wave's rows span [rmin, rmax]; invalid lanes (row n-1) only widen it
    int rmin = qi, rmax = qi;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
      rmin = min(rmin, __shfl_xor(rmin, off, 64));
      rmax = max(rmax, __shfl_xor(rmax, off, 64));
    }
    if (wr.live) {
      wr.s_lo = __builtin_amdgcn_readfirstlane(rmin) >> 2;
      wr.s_hi = __builtin_amdgcn_readfirstlane(rmax) >> 2;
    }
  }

  unsigned cxz[G];
#pragma unroll
  for (int g = 0; g < G; ++g) cxz[g] = 0u;
  unsigned emax = __float_as_uint(eps[0]);
#pragma unroll
  for (int g = 1; g < G; ++g) emax = max(emax, __float_as_uint(eps[g]));
  unsigned done = 0;
  unsigned shared = 0;
  const unsigned gmask = (1u << gd->ng) - 1u;  // the group's real problems (ng <= 16)
  int own = wr.s_lo, r = wr.s_hi + 1, l = wr.s_lo - 1;
  bool ract = wr.live && r < steps, lact = wr.live && l >= 0;
  for (;;) {
    int s, dir;
    if (own <= wr.s_hi) {
      s = own++;
      dir = 0;
    } else if (ract) {
      s = r;
      dir = 1;
    } else if (lact) {
      s = l;
      dir = -1;
    } else {
      break;
    }
    float dz[U];
    unsigned zmin = 0;
    if constexpr (M > 0) {
      // |key differences| first: the window test and the first term of d^Z
      const ksg_f4 r0 = pyz[s * W + 1];
      dz[0] = fabsf(r0.x - qz[0]);
      dz[1] = fabsf(r0.y - qz[0]);
      dz[2] = fabsf(r0.z - qz[0]);
      dz[3] = fabsf(r0.w - qz[0]);
      if (dir != 0) {
        const float gap = dir > 0 ? dz[0] : dz[3];
        if (__builtin_amdgcn_ballot_w64(__float_as_uint(gap) < emax) == 0) {
          if (dir > 0) ract = false;
          else lact = false;
          continue;
        }
        if (dir > 0) ract = ++r < steps;
        else lact = --l >= 0;
      }
      shared += 2 * M;
#pragma unroll
      for (int a = 1; a < M; ++a) {
        const ksg_f4 rz = pyz[s * W + 1 + a];
        dz[0] = fmaxf(dz[0], fabsf(rz.x - qz[a]));
        dz[1] = fmaxf(dz[1], fabsf(rz.y - qz[a]));
        dz[2] = fmaxf(dz[2], fabsf(rz.z - qz[a]));
        dz[3] = fmaxf(dz[3], fabsf(rz.w - qz[a]));
      }
      zmin = min(min(__float_as_uint(dz[0]), __float_as_uint(dz[1])),
                 min(__float_as_uint(dz[2]), __float_as_uint(dz[3])));
      if (__builtin_amdgcn_ballot_w64(zmin < emax) == 0) continue;
    } else {
      if (dir > 0) ract = ++r < steps;
      else if (dir < 0) lact = --l >= 0;
    }
    // the whole X block of the step is requested at once (one wait, not one per problem)
    ksg_f4 rx[G];
#pragma unroll
    for (int g = 0; g < G; ++g) rx[g] = px[s * G + g];
    unsigned act = 0;  // problems whose work ran in this step (bit g; wave-uniform, kept scalar)
#pragma unroll
    for (int g = 0; g < G; ++g) {
      if constexpr (M > 0) {
        if (__builtin_amdgcn_ballot_w64(zmin < __float_as_uint(eps[g])) == 0) continue;
      }
      act |= 1u << g;
      const float t[U] = {fabsf(rx[g].x - qx[g]), fabsf(rx[g].y - qx[g]), fabsf(rx[g].z - qx[g]),
                          fabsf(rx[g].w - qx[g])};
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const float dxz = M > 0 ? fmaxf(t[u], dz[u]) : t[u];
        // dxz < eps exactly when fl(dxz - eps) is negative (denormals kept, so the difference
        // of two distinct values is never zero): the sign bit is the count increment, with a
        // subtract and a shift that both read only VGPRs
        cxz[g] += __float_as_uint(dxz - eps[g]) >> 31;
      }
    }
    done += __builtin_popcount(__builtin_amdgcn_readfirstlane(act) & gmask);
  }

  // ---- epilogue: self correction, digamma terms, one partial per (problem, tile) ----
  // The terms go back to their rows' places before the fixed-order sum, so the partial does
  // not depend on how the rows were handed to the waves (nor on the group size).
  const int wave = threadIdx.x >> 6;
  const double* trow = T + gd->e_off + (size_t)qi * G;
  double* s_term = reinterpret_cast<double*>(s_ord);
  const int slot = valid ? qi - tile * kTileQ : (int)threadIdx.x;  // invalid rows sort last
#pragma unroll
  for (int g = 0; g < G; ++g) {
    const int self = eps[g] > 0.0f ? 1 : 0;
    const int nxz = max((int)cxz[g] - self, 0);
    __syncthreads();
    s_term[slot] = valid ? htab[nxz] + trow[g] : 0.0;
    __syncthreads();
    const double t = wave_sum(s_term[threadIdx.x]);
    if ((threadIdx.x & 63) == 0) s_red[wave][g] = t;
  }
  if (work && (threadIdx.x & 63) == 0) {
    atomicAdd(&work[1], (unsigned long long)done);
    atomicAdd(&work[4], (unsigned long long)shared);
  }
  __syncthreads();
  if ((int)threadIdx.x < ng)
    partials[gd->part_base + threadIdx.x * gd->n_tiles + tile] =
        (s_red[0][threadIdx.x] + s_red[1][threadIdx.x]) + (s_red[2][threadIdx.x] + s_red[3][threadIdx.x]);
}

// One work-group per work item (group, tile); items with group < 0 are XCD padding.
template <int M, int G, int KP>
__global__ __launch_bounds__(kTileQ) void ksg_group_radius_kernel(const float* __restrict__ base,
                                                                  const GroupDesc* __restrict__ descs,
                                                                  const WorkItem* __restrict__ items,
                                                                  float* __restrict__ E,
                                                                  unsigned long long* __restrict__ work) {
  __shared__ unsigned long long s_ord[kTileQ];
  __shared__ float s_x[kXchg][kTileQ];
  const KSG_AS4 WorkItem* i4 = (const KSG_AS4 WorkItem*)items;
  const int grp = i4[blockIdx.x].prob;
  if (grp < 0) return;
  const int tile = i4[blockIdx.x].tile;
  const KSG_AS4 GroupDesc* gd = (const KSG_AS4 GroupDesc*)descs + grp;
  group_radius_tile<M, G, KP>(base, gd, tile, E, s_ord, s_x, work);
}

template <int M, int G>
__global__ __launch_bounds__(kTileQ) void ksg_group_xcount_kernel(const float* __restrict__ base,
                                                                  const GroupDesc* __restrict__ descs,
                                                                  const WorkItem* __restrict__ items,
                                                                  const float* __restrict__ E,
                                                                  const double* __restrict__ T,
                                                                  const double* __restrict__ htab,
                                                                  double* __restrict__ partials,
                                                                  unsigned long long* __restrict__ work) {
  __shared__ double s_red[kTileQ / 64][G];
  __shared__ unsigned long long s_ord[kTileQ];
  const KSG_AS4 WorkItem* i4 = (const KSG_AS4 WorkItem*)items;
  const int grp = i4[blockIdx.x].prob;
  if (grp < 0) return;
  const int tile = i4[blockIdx.x].tile;
  const KSG_AS4 GroupDesc* gd = (const KSG_AS4 GroupDesc*)descs + grp;
  group_xcount_tile<M, G>(base, gd, tile, E, T, htab, partials, s_red, s_ord, work);
}

}  // namespace ksg
