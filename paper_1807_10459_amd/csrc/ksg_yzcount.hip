// Y/Z count kernel: the counts n_YZ and n_Z of every problem of a Y/Z set, for one query row.
//
// For a query i the two counts are step functions of the radius alone,
//   F_YZ(e) = #{ j : d^YZ_ij < e },   F_Z(e) = #{ j : d^Z_ij < e }   (self included),
// and every problem p of the set (a candidate or surrogate of one greedy step) needs them at
// its own radius eps_p(i).  So instead of counting per problem, the work-group sorts the radii
// of up to kYZSlots problems once, ranks every reference's d^Z and d^YZ among them by binary
// search (pos_j = #{ radii <= d_j }), histograms the ranks in LDS, and turns the histogram
// into the counts with one prefix sum: the r-th smallest radius has F(radius_(r)) =
// #{ j : pos_j <= r }.  Ties are exact (equal radii get equal counts), the distances are the
// same FP32 subtractions and exact maxima as in the search kernels, so the counts equal a
// per-problem count bit for bit.  The output is the problem's FP64 term H(n_YZ) - H(n_Z)
// (self removed), written to T[row][slot] for the X count kernel.
//
// Only references within the key window can count: d^Z >= |k_j - k_i| (the key is Z_1;
// without Z it is Y, and d^YZ = |dy| >= |k_j - k_i|), so the scan runs outward from the query
// row in chunks of 256 rows and stops at the first chunk lying entirely outside the largest
// radius, exactly as the search kernels' windows do.
#include "ksg_search.inc.h"

namespace ksg {

constexpr int kYZThreads = 256;
constexpr int kYZBuckets = 256;  // radius buckets of the rank search

template <int M>
__global__ __launch_bounds__(kYZThreads) void ksg_yzcount_kernel(const float* __restrict__ base,
                                                                 const YZDesc* __restrict__ descs,
                                                                 const WorkItem* __restrict__ items,
                                                                 const float* __restrict__ E,
                                                                 double* __restrict__ T,
                                                                 const double* __restrict__ htab,
                                                                 unsigned long long* __restrict__ work) {
  __shared__ unsigned long long s_key[kYZSlots];  // (radius bits << 32) | slot, sorted
  __shared__ unsigned s_hz[kYZSlots + 1];
  __shared__ unsigned s_hyz[kYZSlots + 1];
  __shared__ unsigned s_part[2][kYZThreads];
  __shared__ int s_start[kYZBuckets + 2];  // first sorted slot of each radius bucket
  constexpr int W = M + 1;
  const int tid = threadIdx.x;
  const WorkItem it = items[blockIdx.x];
  if (it.prob < 0) return;
  const YZDesc d = descs[it.prob];
  const int i = it.tile;
  const int n = d.n;
  const float* yzi = base + d.yzi_off;
  auto at = [&](int j, int a) { return yzi[((j >> 2) * W + a) * 4 + (j & 3)]; };
  const float qy = at(i, 0);
  float qz[M > 0 ? M : 1];
#pragma unroll
  for (int a = 0; a < M; ++a) qz[a] = at(i, 1 + a);
  const float qkey = M > 0 ? qz[0] : qy;

  // ---- the radii of this descriptor's slots, sorted ascending (invalid slots last) ----
  int P2 = 64;
  while (P2 < d.n_slots) P2 <<= 1;
  const int nv = d.n_slots;  // every slot of a descriptor is a real problem, nv >= 1
  for (int s = tid; s < P2; s += kYZThreads) {
    unsigned long long kk = ~0ull;
    if (s < nv) {
      const int rs = d.slot0 + s;  // slot within the run of groups
      const float r = E[d.e_off + (size_t)(rs / d.G) * ((size_t)d.n_pad * d.G) + (size_t)i * d.G + rs % d.G];
      kk = ((unsigned long long)__float_as_uint(r) << 32) | (unsigned)s;
    }
    s_key[s] = kk;
  }
  for (int s = tid; s <= P2; s += kYZThreads) {
    s_hz[s] = 0u;
    s_hyz[s] = 0u;
  }
  __syncthreads();
  for (int size = 2; size <= P2; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int t = tid; t < (P2 >> 1); t += kYZThreads) {
        const int lo = 2 * t - (t & (stride - 1));
        const int hi = lo + stride;
        const unsigned long long a = s_key[lo], b = s_key[hi];
        const bool up = (lo & size) == 0;
        if ((a > b) == up) {
          s_key[lo] = b;
          s_key[hi] = a;
        }
      }
      __syncthreads();
    }
  }
  const float rmax = __uint_as_float((unsigned)(s_key[nv - 1] >> 32));

  // pos(d) = number of radii <= d.  The radii are non-negative, so their bit patterns order
  // like their values; bucket(x) = (x - r_lo) >> shift maps [r_lo, r_hi] monotonically onto at
  // most kYZBuckets buckets, s_start[b] = the first sorted slot whose bucket is >= b.  Every
  // radius of a lower bucket is < d and every radius of a higher bucket is > d, so pos(d) =
  // s_start[b] + #{radii of bucket b that are <= d}, found by a short binary search.
  const unsigned r_lo = (unsigned)(s_key[0] >> 32), r_hi = (unsigned)(s_key[nv - 1] >> 32);
  const unsigned span = r_hi - r_lo;  // r_hi >= r_lo
  int shift = 0;
  while ((span >> shift) >= (unsigned)kYZBuckets) ++shift;
  for (int i = tid; i < nv; i += kYZThreads) {
    const int b = (int)(((unsigned)(s_key[i] >> 32) - r_lo) >> shift);
    const int bp = i == 0 ? -1 : (int)(((unsigned)(s_key[i - 1] >> 32) - r_lo) >> shift);
    for (int q = bp + 1; q <= b; ++q) s_start[q] = i;  // buckets (bp, b] start at slot i
  }
  const int b_last = (int)((r_hi - r_lo) >> shift);
  for (int q = b_last + 1 + tid; q <= kYZBuckets + 1; q += kYZThreads) s_start[q] = nv;
  __syncthreads();
  auto rank = [&](float dist) {
    const unsigned db = __float_as_uint(dist);
    if (db < r_lo) return 0;
    if (db >= r_hi) return nv;
    const int b = (int)((db - r_lo) >> shift);  // b < b_last + 1 <= kYZBuckets
    int lo = s_start[b], hi = s_start[b + 1];
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if ((unsigned)(s_key[mid] >> 32) <= db) lo = mid + 1;
      else hi = mid;
    }
    return lo;
  };
  unsigned c0z = 0, c0yz = 0, visited = 0;
  auto visit = [&](int j) {
    float dz = 0.0f;
    if constexpr (M > 0) {
      dz = fabsf(at(j, 1) - qz[0]);
#pragma unroll
      for (int a = 1; a < M; ++a) dz = fmaxf(dz, fabsf(at(j, 1 + a) - qz[a]));
      const int pz = rank(dz);
      if (pz == 0) ++c0z;
      else if (pz < nv) atomicAdd(&s_hz[pz], 1u);
    }
    const float dyz = fmaxf(fabsf(at(j, 0) - qy), dz);
    const int py = rank(dyz);
    if (py == 0) ++c0yz;
    else if (py < nv) atomicAdd(&s_hyz[py], 1u);
    ++visited;
  };
  constexpr int KC = M > 0 ? 1 : 0;
  for (int j0 = i;; j0 += kYZThreads) {  // right of the query (the query row included)
    const int j = j0 + tid;
    bool in = false;
    if (j < n) {
      in = at(j, KC) - qkey < rmax;
      if (in) visit(j);
    }
    if (!__syncthreads_or(in)) break;
  }
  for (int j0 = i - 1;; j0 -= kYZThreads) {  // left of the query
    const int j = j0 - tid;
    bool in = false;
    if (j >= 0) {
      in = qkey - at(j, KC) < rmax;
      if (in) visit(j);
    }
    if (!__syncthreads_or(in)) break;
  }
  if (c0z) atomicAdd(&s_hz[0], c0z);
  if (c0yz) atomicAdd(&s_hyz[0], c0yz);
  __syncthreads();

  // ---- inclusive prefix sums over the first nv bins ----
  const int chunk = (nv + kYZThreads - 1) / kYZThreads;
  const int b0 = min(nv, tid * chunk), b1 = min(nv, b0 + chunk);
  unsigned sz = 0, syz = 0;
  for (int q = b0; q < b1; ++q) {
    sz += s_hz[q];
    syz += s_hyz[q];
  }
  // exclusive scan of the threads' chunk sums: inclusive within each wave by shuffles, then the
  // totals of the lower waves
  const int lane = tid & 63, wave = tid >> 6;
  unsigned iz = sz, iyz = syz;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const unsigned tz = __shfl_up(iz, off, 64), tyz = __shfl_up(iyz, off, 64);
    if (lane >= off) {
      iz += tz;
      iyz += tyz;
    }
  }
  if (lane == 63) {
    s_part[0][wave] = iz;
    s_part[1][wave] = iyz;
  }
  __syncthreads();
  unsigned az = iz - sz, ayz = iyz - syz;
  for (int w = 0; w < wave; ++w) {
    az += s_part[0][w];
    ayz += s_part[1][w];
  }
  for (int q = b0; q < b1; ++q) {
    az += s_hz[q];
    ayz += s_hyz[q];
    s_hz[q] = az;
    s_hyz[q] = ayz;
  }
  __syncthreads();

  // ---- terms H(n_YZ) - H(n_Z) of every slot, self removed ----
  for (int r = tid; r < nv; r += kYZThreads) {
    const unsigned long long kk = s_key[r];
    const int rs = d.slot0 + (int)(unsigned)(kk & 0xffffffffu);
    const float eps = __uint_as_float((unsigned)(kk >> 32));
    const int self = eps > 0.0f ? 1 : 0;
    const int nyz = max((int)s_hyz[r] - self, 0);
    const int nz = M > 0 ? max((int)s_hz[r] - self, 0) : (self ? n - 1 : 0);
    T[d.e_off + (size_t)(rs / d.G) * ((size_t)d.n_pad * d.G) + (size_t)i * d.G + rs % d.G] = htab[nyz] - htab[nz];
  }
  if (work) {
    // per visited reference: d^Z and d^YZ (2m+1 sub/max, or 1) and one or two rank searches
    int levels = 0;
    for (int b = P2; b >= 1; b >>= 1) ++levels;
    unsigned long long ops =
        (unsigned long long)visited * (unsigned)((M > 0 ? 2 * M + 1 : 1) + (M > 0 ? 2 : 1) * levels);
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) ops += __shfl_xor(ops, off, 64);
    if ((tid & 63) == 0) atomicAdd(&work[3], ops);
  }
}

#define KSG_YZ(M) reinterpret_cast<const void*>(&ksg_yzcount_kernel<M>)
// [m] for m = 0..kGroupMaxM
const void* yzcount_kernels[kGroupMaxM + 1] = {
    KSG_YZ(0),  KSG_YZ(1),  KSG_YZ(2),  KSG_YZ(3),  KSG_YZ(4),  KSG_YZ(5),  KSG_YZ(6),  KSG_YZ(7),
    KSG_YZ(8),  KSG_YZ(9),  KSG_YZ(10), KSG_YZ(11), KSG_YZ(12), KSG_YZ(13), KSG_YZ(14), KSG_YZ(15),
    KSG_YZ(16), KSG_YZ(17), KSG_YZ(18), KSG_YZ(19), KSG_YZ(20), KSG_YZ(21), KSG_YZ(22), KSG_YZ(23),
    KSG_YZ(24), KSG_YZ(25), KSG_YZ(26), KSG_YZ(27), KSG_YZ(28), KSG_YZ(29), KSG_YZ(30)};
static_assert(kGroupMaxM == 30, "one instantiation per conditioning dimension");

}  // namespace ksg
