// X count kernel in the transposed layout: one query per wave, 64 references per instruction.
//
// The grouped X count (n_XZ of the G problems of a group, then the tile's digamma partial
// sums) has the same inputs, outputs and summation order as ksg_group_xcount_kernel, so the
// partials are bit-identical.  The work is laid out the other way round:
//   - a wave takes the 64 query rows of its quarter of the tile one after the other;
//   - for a query, the lanes hold 64 consecutive reference rows (a block) and the query's
//     coordinates are copied once into VGPRs, so every subtract reads VGPRs only;
//   - per problem g and block, the comparison d < eps_g gives a 64-bit mask whose population
//     count is added on the scalar unit: n_XZ(g) = sum over blocks of popcount(mask);
//   - the key window is the query's own: blocks are scanned outward from the query's block and
//     a direction ends at the first block whose nearest key lies at least the query's largest
//     radius away (every distance is at least the key gap, and FP32 rounding is monotone).
// d^Z = max over the Z columns of |z_j - z_q| is computed once per (query, block) and shared by
// the G problems; a problem whose eps_g no reference of the block beats in d^Z is skipped.
#pragma once

#include "ksg_group.inc.h"

namespace ksg {

// A wave-uniform value copied into a VGPR (so that VALU arithmetic reads VGPRs only).
__device__ __forceinline__ float to_vgpr(float s) {
  float v;
  asm volatile("v_mov_b32 %0, %1" : "=v"(v) : "s"(s));
  return v;
}

template <int M, int G>
__device__ __forceinline__ void group_xcount_t_tile(const float* __restrict__ base, const KSG_AS4 GroupDesc* gd,
                                                    int tile, const float* __restrict__ E,
                                                    const double* __restrict__ T, const double* __restrict__ htab,
                                                    double* __restrict__ partials, double (*s_red)[G],
                                                    unsigned long long* __restrict__ work) {
  constexpr int W = M + 1;
  const int n = gd->n;
  const int nblk = gd->n_pad >> 6;  // blocks of 64 rows (n_pad is a multiple of 64)
  const int lane = (int)threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
  const float* xi = base + gd->xi_off;
  const float* yzi = base + gd->yzi_off;
  const KSG_AS4 float* xs = (const KSG_AS4 float*)xi;   // scalar reads of a query's values
  const KSG_AS4 float* yzs = (const KSG_AS4 float*)yzi;
  const KSG_AS4 float* es = (const KSG_AS4 float*)(E + gd->e_off);
  const KSG_AS4 double* ts = (const KSG_AS4 double*)(T + gd->e_off);
  const KSG_AS4 double* hs = (const KSG_AS4 double*)htab;

  double my_term[G];  // lane i: the terms of the wave's i-th query
#pragma unroll
  for (int g = 0; g < G; ++g) my_term[g] = 0.0;
  unsigned done = 0;  // (query, block, problem) units of 64 pairs whose work ran

  const int q0 = tile * kTileQ + wave * 64;
  const int q_end = min(q0 + 64, n);
  for (int q = q0; q < q_end; ++q) {
    // the query's radii and coordinates (wave-uniform: scalar reads), then VGPR copies
    float eps[G];
    unsigned emax = 0;
#pragma unroll
    for (int g = 0; g < G; ++g) {
      eps[g] = es[(size_t)q * G + g];
      emax = max(emax, __float_as_uint(eps[g]));
    }
    const int qs = q >> 2, ql = q & 3;
    float qx[G], qz[M > 0 ? M : 1];
#pragma unroll
    for (int g = 0; g < G; ++g) qx[g] = to_vgpr(xs[(qs * G + g) * 4 + ql]);
#pragma unroll
    for (int a = 0; a < M; ++a) qz[a] = to_vgpr(yzs[(qs * W + 1 + a) * 4 + ql]);
    unsigned cnt[G];
#pragma unroll
    for (int g = 0; g < G; ++g) cnt[g] = 0u;

    // One block of 64 rows: dir = 0 (the query's own block, no window test), +1 right, -1 left.
    // Returns false when the block lies wholly outside the window (the direction ends).
    auto block = [&](int b, int dir) -> bool {
      const int r = (b << 6) + lane;
      const int rs = r >> 2, rl = r & 3;
      float dz = 0.0f;
      if constexpr (M > 0) {
        dz = fabsf(yzi[(rs * W + 1) * 4 + rl] - qz[0]);  // the key gap, and the first term of d^Z
        if (dir != 0) {
          // the nearest row of the block: its first (right) or last (left) row
          const unsigned gap = (unsigned)__builtin_amdgcn_readlane(__float_as_int(dz), dir > 0 ? 0 : 63);
          if (gap >= emax) return false;  // non-negative floats order like their bit patterns
        }
#pragma unroll
        for (int a = 1; a < M; ++a) dz = fmaxf(dz, fabsf(yzi[(rs * W + 1 + a) * 4 + rl] - qz[a]));
      }
      float rx[G];
#pragma unroll
      for (int g = 0; g < G; ++g) rx[g] = xi[(rs * G + g) * 4 + rl];
#pragma unroll
      for (int g = 0; g < G; ++g) {
        if constexpr (M > 0) {
          if (__builtin_amdgcn_ballot_w64(dz < eps[g]) == 0) continue;  // no reference can count
        }
        ++done;
        const float d = M > 0 ? fmaxf(fabsf(rx[g] - qx[g]), dz) : fabsf(rx[g] - qx[g]);
        cnt[g] += (unsigned)__builtin_popcountll(__builtin_amdgcn_ballot_w64(d < eps[g]));
      }
      return true;
    };

    const int qb = q >> 6;
    block(qb, 0);
    if constexpr (M > 0) {
      for (int b = qb + 1; b < nblk && block(b, 1); ++b) {
      }
      for (int b = qb - 1; b >= 0 && block(b, -1); --b) {
      }
    } else {  // without Z the X counts are not bounded by the key (Y): every block
      for (int b = 0; b < nblk; ++b)
        if (b != qb) block(b, 0);
    }

    // the query's terms H(n_XZ) + T (self removed), kept by the lane of the query's slot
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int self = eps[g] > 0.0f ? 1 : 0;
      const int nxz = max((int)cnt[g] - self, 0);
      const double term = hs[nxz] + ts[(size_t)q * G + g];
      if (lane == q - q0) my_term[g] = term;
    }
  }

  // ---- one partial per (problem, tile): the fixed-order sum of the classic X count kernel ----
  const bool valid = q0 + lane < n;
#pragma unroll
  for (int g = 0; g < G; ++g) {
    const double t = wave_sum(valid ? my_term[g] : 0.0);
    if (lane == 0) s_red[wave][g] = t;
  }
  if (work && lane == 0) atomicAdd(&work[1], (unsigned long long)((done + 2) / 4));  // in 256-pair units
  __syncthreads();
  if ((int)threadIdx.x < gd->ng)
    partials[gd->part_base + threadIdx.x * gd->n_tiles + tile] =
        (s_red[0][threadIdx.x] + s_red[1][threadIdx.x]) + (s_red[2][threadIdx.x] + s_red[3][threadIdx.x]);
}

template <int M, int G>
__global__ __launch_bounds__(kTileQ) void ksg_group_xcount_t_kernel(const float* __restrict__ base,
                                                                    const GroupDesc* __restrict__ descs,
                                                                    const WorkItem* __restrict__ items,
                                                                    const float* __restrict__ E,
                                                                    const double* __restrict__ T,
                                                                    const double* __restrict__ htab,
                                                                    double* __restrict__ partials,
                                                                    unsigned long long* __restrict__ work) {
  __shared__ double s_red[kTileQ / 64][G];
  const KSG_AS4 WorkItem* i4 = (const KSG_AS4 WorkItem*)items;
  const int grp = i4[blockIdx.x].prob;
  if (grp < 0) return;
  const int tile = i4[blockIdx.x].tile;
  const KSG_AS4 GroupDesc* gd = (const KSG_AS4 GroupDesc*)descs + grp;
  group_xcount_t_tile<M, G>(base, gd, tile, E, T, htab, partials, s_red, work);
}

}  // namespace ksg
