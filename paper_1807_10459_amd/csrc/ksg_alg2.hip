// KSG algorithm 2 (conditional form): neighbour rectangles instead of a joint radius.
//
// Kraskov, Stoegbauer & Grassberger define a second estimator next to the one the other search
// kernels compute (the paper names the KSG estimator in its Summary, estimator paragraph, and
// prints neither).  For point i:
//   the k nearest neighbours = the k smallest (d_ij, j), j != i, d the joint max-norm distance,
//     ties at the k-th distance broken by the lower index (the neighbours' identities matter);
//   rectangle sides e^S_i = the largest d^S_ij over those neighbours, S in {X, Y, Z};
//   n_xz = #{j != i : d^X_ij <= e^X_i and d^Z_ij <= e^Z_i}, n_yz likewise, n_z = #{d^Z <= e^Z};
//   I = psi(k) - 2/k + <psi(n_z) - psi(n_xz) - psi(n_yz) + 1/n_xz + 1/n_yz>
//     = H_{k-1} - 2/k + <H_{n_z-1} - H_{n_xz-1} - H_{n_yz-1} + 1/n_xz + 1/n_yz>,
//   and without Z the algorithm-2 MI: I = H_{k-1} - 1/k + H_{N-1} - <H_{n_x-1} + H_{n_y-1}>.
//
// Mapping: one query per lane, references through the scalar data path as in the algorithm-1
// kernel.  Pass 1 keeps the k+1 smallest (distance, index) pairs, self included: references
// arrive in increasing index order and a candidate is inserted only below a strictly larger
// distance, so equal distances stay in index order without comparing indices.  The k
// neighbours (self skipped) are then gathered per lane (k x D loads) for the rectangle sides.
// Pass 2 counts with <= per space; self is always inside its own rectangle and is subtracted.
// The per-point FP64 term t_i is written so that I = C - (1/N) sum_i t_i, with C = H_{k-1} -
// 2/k (or H_{k-1} - 1/k + H_{N-1} without Z); the finalisation applies C.
#include "ksg_search.inc.h"

namespace ksg {

template <int KP>
__device__ __forceinline__ void topk_insert_index(float (&b)[KP], int (&bi)[KP], float v, int j) {
#pragma unroll
  for (int s = KP - 1; s >= 1; --s) {
    const bool shift = v < b[s - 1];
    const bool place = v < b[s];
    bi[s] = shift ? bi[s - 1] : (place ? j : bi[s]);
    b[s] = __builtin_amdgcn_fmed3f(b[s - 1], b[s], v);  // = shift ? b[s-1] : min(b[s], v)
  }
  if (v < b[0]) {
    b[0] = v;
    bi[0] = j;
  }
}

// Pass 2 with a compile-time split: counts inside the rectangle (self included).
template <int DX, int DY, int DZ, int U>
__device__ __forceinline__ Counts rect_count_pass(const cfptr (&col)[DX + DY + DZ],
                                                  const float (&q)[DX + DY + DZ], int n_pad, float ex,
                                                  float ey, float ez) {
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
        const bool cz = C <= ez;
        axz[u] += (unsigned)((A <= ex) & cz);
        ayz[u] += (unsigned)((B <= ey) & cz);
        az[u] += (unsigned)cz;
      } else {
        axz[u] += (unsigned)(A <= ex);
        ayz[u] += (unsigned)(B <= ey);
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

// Pass 2 for a split known only at run time (per-column selects).
template <int D>
__device__ __forceinline__ Counts rect_count_split(const cfptr (&col)[D], const float (&q)[D], int n_pad,
                                                   int dx, int dy, float ex, float ey, float ez) {
  constexpr int U = 4;
  const bool has_z = dx + dy < D;
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
      const bool cz_ = !has_z || C <= ez;  // padding rows (+inf) fail A <= ex anyway
      cxz += (A <= ex) & cz_;
      cyz += (B <= ey) & cz_;
      cz += cz_;
    }
  }
  return Counts{cxz, cyz, cz};
}

template <int D, int KP>
__global__ __launch_bounds__(kTileQ) void ksg_alg2_kernel(const ProbDesc* __restrict__ descs,
                                                          const WorkItem* __restrict__ items,
                                                          const double* __restrict__ htab,
                                                          double* __restrict__ partials) {
  __shared__ double s_red[kTileQ / 64];
  constexpr int U = D <= 8 ? 8 : 4;
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
  const bool has_z = pd->dz > 0;
  const int qraw = tile * kTileQ + (int)threadIdx.x;
  const bool valid = qraw < n;
  const int qi = valid ? qraw : n - 1;

  cfptr col[D];
  const float* gcol[D];
  float q[D];
#pragma unroll
  for (int a = 0; a < D; ++a) {
    const float* c = pd->col[a];
    col[a] = (cfptr)c;
    gcol[a] = c;
    q[a] = c[qi];
  }

  // ---- pass 1: the k+1 smallest (distance, index) pairs, self included ----
  float b[KP];
  int bi[KP];
#pragma unroll
  for (int s = 0; s < KP; ++s) {
    b[s] = (s < KP - 1 - k) ? -INFINITY : INFINITY;
    bi[s] = -1;
  }
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
      // one branch per candidate: a wave runs an insertion only when one of its lanes has that
      // candidate below its current k+1-th distance
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (d[u] < b[KP - 1]) topk_insert_index<KP>(b, bi, d[u], j + u);
    }
  }

  // ---- the k neighbours (self skipped) and the rectangle sides ----
  float ex = 0.0f, ey = 0.0f, ez = 0.0f, eps = 0.0f;
  int taken = 0;
#pragma unroll
  for (int s = 0; s < KP; ++s) {
    const int j = bi[s];
    if (j >= 0 && j != qi && taken < k) {
#pragma unroll
      for (int a = 0; a < D; ++a) {
        const float t = fabsf(gcol[a][j] - q[a]);
        if (a < dx) ex = fmaxf(ex, t);
        else if (a < dx + dy) ey = fmaxf(ey, t);
        else ez = fmaxf(ez, t);
      }
      eps = b[s];
      ++taken;
    }
  }

  // ---- pass 2: rectangle counts ----
  const Counts c = (dx == 1 && dy == 1) ? rect_count_pass<1, 1, D - 2, U>(col, q, n_pad, ex, ey, ez)
                                        : rect_count_split<D>(col, q, n_pad, dx, dy, ex, ey, ez);
  // self is inside every rectangle; every count is >= k (clamped for non-finite inputs that
  // bypassed the finite check)
  const int nxz = max(c.xz - 1, 1);
  const int nyz = max(c.yz - 1, 1);
  const int nz = has_z ? max(c.z - 1, 1) : n - 1;
  double t = 0.0;
  if (valid) {
    if (has_z)
      t = -(((htab[nz - 1] - htab[nxz - 1]) - htab[nyz - 1]) + (1.0 / (double)nxz + 1.0 / (double)nyz));
    else
      t = htab[nxz - 1] + htab[nyz - 1];
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
    if (lo) {
      const double cst = has_z ? htab[k - 1] - 2.0 / (double)k : (htab[k - 1] - 1.0 / (double)k) + htab[n - 1];
      lo[qi] = cst - t;
    }
  }
  t = wave_sum(t);
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) s_red[wave] = t;
  __syncthreads();
  if (threadIdx.x == 0) partials[pd->part_base + tile] = (s_red[0] + s_red[1]) + (s_red[2] + s_red[3]);
}

#define KSG_A2_ROW(KP)                                                                                   \
  {reinterpret_cast<const void*>(&ksg_alg2_kernel<2, KP>),  reinterpret_cast<const void*>(&ksg_alg2_kernel<3, KP>),  \
   reinterpret_cast<const void*>(&ksg_alg2_kernel<4, KP>),  reinterpret_cast<const void*>(&ksg_alg2_kernel<5, KP>),  \
   reinterpret_cast<const void*>(&ksg_alg2_kernel<6, KP>),  reinterpret_cast<const void*>(&ksg_alg2_kernel<7, KP>),  \
   reinterpret_cast<const void*>(&ksg_alg2_kernel<8, KP>),  reinterpret_cast<const void*>(&ksg_alg2_kernel<9, KP>),  \
   reinterpret_cast<const void*>(&ksg_alg2_kernel<10, KP>), reinterpret_cast<const void*>(&ksg_alg2_kernel<11, KP>), \
   reinterpret_cast<const void*>(&ksg_alg2_kernel<12, KP>), reinterpret_cast<const void*>(&ksg_alg2_kernel<13, KP>), \
   reinterpret_cast<const void*>(&ksg_alg2_kernel<14, KP>), reinterpret_cast<const void*>(&ksg_alg2_kernel<15, KP>), \
   reinterpret_cast<const void*>(&ksg_alg2_kernel<16, KP>)}

// [kp class][D - 2]: kp class 0 = 5 slots (k <= 4), 1 = 9 (k <= 8), 2 = 17 (k <= 16).
const void* alg2_kernels[3][15] = {KSG_A2_ROW(5), KSG_A2_ROW(9), KSG_A2_ROW(17)};

hipError_t launch_ksg_alg2(const ProbDesc* d_desc, const WorkItem* d_items, int n_items,
                           const double* d_htab, double* d_partials, int D, int kp, hipStream_t stream) {
  if (n_items <= 0) return hipSuccess;
  if (D < 2 || D > kMaxDimsCompiled || (kp != 5 && kp != 9 && kp != 17)) return hipErrorInvalidValue;
  const void* fn = alg2_kernels[kp == 5 ? 0 : (kp == 9 ? 1 : 2)][D - 2];
  const ProbDesc* a0 = d_desc;
  const WorkItem* a1 = d_items;
  const double* a2 = d_htab;
  double* a3 = d_partials;
  void* args[] = {&a0, &a1, &a2, &a3};
  return hipLaunchKernel(fn, dim3(n_items), dim3(kTileQ), args, 0, stream);
}

}  // namespace ksg
