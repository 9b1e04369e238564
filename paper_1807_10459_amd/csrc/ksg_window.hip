// Key-ordered window search: the key-order (rank) kernel, the KSG algorithm-1 kernels and
// the launchers.  The search itself is in ksg_window.inc.h.
#include "ksg_window.inc.h"

namespace ksg {

extern const void* window_kernels_alg2[15];

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

#define KSG_WIN(D) reinterpret_cast<const void*>(&ksg_window_kernel<D, 5, 1>)
// [D - 2] for D in [2, 16]; top-k of 5 slots (k <= 4); KSG algorithm 1.  The algorithm-2
// table is in ksg_window_alg2.hip.
const void* window_kernels_alg1[15] = {KSG_WIN(2),  KSG_WIN(3),  KSG_WIN(4),  KSG_WIN(5),  KSG_WIN(6),
                                       KSG_WIN(7),  KSG_WIN(8),  KSG_WIN(9),  KSG_WIN(10), KSG_WIN(11),
                                       KSG_WIN(12), KSG_WIN(13), KSG_WIN(14), KSG_WIN(15), KSG_WIN(16)};

hipError_t launch_window_rank(const float* key, int n, int n_pad, int32_t* sigma, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(window_rank_kernel, dim3((n_pad + 255) / 256), dim3(256), 0, stream, key, n, n_pad, sigma);
  return hipGetLastError();
}

hipError_t launch_ksg_window(const ProbDesc* d_desc, const WorkItem* d_items, int n_items, const double* d_htab,
                             double* d_partials, int D, int alg, unsigned long long* d_work, hipStream_t stream) {
  if (n_items <= 0) return hipSuccess;
  if (D < 2 || D > kMaxDimsCompiled || (alg != 1 && alg != 2)) return hipErrorInvalidValue;
  const ProbDesc* a0 = d_desc;
  const WorkItem* a1 = d_items;
  const double* a2 = d_htab;
  double* a3 = d_partials;
  unsigned long long* a4 = d_work;
  void* args[] = {&a0, &a1, &a2, &a3, &a4};
  const void* kern = alg == 1 ? window_kernels_alg1[D - 2] : window_kernels_alg2[D - 2];
  return hipLaunchKernel(kern, dim3(n_items), dim3(kTileQ), args, 0, stream);
}

}  // namespace ksg
