// cmi_ksg_noalloc: the single estimate of cmi_ksg without any allocation, for callers that
// cannot allocate device memory (code under stream capture, tight serving loops).
//
// Every buffer the estimate needs beyond the caller's inputs and output -- the +inf-padded
// columns, the problem descriptor, the work items, the per-tile partial sums, the pack jobs,
// a status flag and the harmonic-number table -- lives in one file-scope device array,
// `scratch`, of a fixed size (kNoAllocBytes per device, held until the process ends).  The
// device address of the array is looked up once per device when a context is created on it
// (hipGetSymbolAddress) and kept per device; host code passes that address to the kernels and
// never the array's name.  The harmonic table part is written at that set-up and never again.
//
// A call: one set-up kernel writes the descriptor, items and pack jobs (passed by value as
// kernel arguments) and clears the flag; then the pack, the finite check, the brute-force
// search (the kernels of the batched path), the finalisation and a last kernel that turns the
// estimate into NaN when the data held a non-finite value.  All of it is queued on the
// context's stream: no allocation, no host synchronisation, no memset.  Calls on one device
// share the array, so calls that overlap on one GPU (two streams, two threads) race.
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>
#include <vector>

#include "../../include/ksgcmi.h"
#include "internal.h"
#include "runtime.h"

namespace ksg {

constexpr int64_t kNoAllocMaxN = KSG_NOALLOC_MAX_N;
constexpr int kNoAllocMaxDims = kMaxDimsCompiled;
constexpr int64_t kNoAllocMaxPad = (kNoAllocMaxN + kPad - 1) / kPad * kPad;
constexpr int kNoAllocMaxTiles = (int)((kNoAllocMaxN + kTileQ - 1) / kTileQ);

constexpr size_t align256(size_t v) { return (v + 255) & ~size_t(255); }
// Byte offsets of the parts of the array.
constexpr size_t kOffHtab = 0;
constexpr size_t kOffPool = align256(kOffHtab + sizeof(double) * (kNoAllocMaxN + 1));
constexpr size_t kOffDesc = align256(kOffPool + sizeof(float) * kNoAllocMaxDims * kNoAllocMaxPad);
constexpr size_t kOffItems = align256(kOffDesc + sizeof(ProbDesc));
constexpr size_t kOffPartials = align256(kOffItems + sizeof(WorkItem) * kNoAllocMaxTiles);
constexpr size_t kOffJobs = align256(kOffPartials + sizeof(double) * kNoAllocMaxTiles);
constexpr size_t kOffFlag = align256(kOffJobs + sizeof(PackJob) * kNoAllocMaxDims);
constexpr size_t kNoAllocBytes = align256(kOffFlag + sizeof(int));

static_assert(kNoAllocBytes < (size_t(8) << 20), "the scratch array stays modest (under 8 MiB)");

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

// Kernel arguments of the set-up kernel: the descriptor and the pack jobs by value.
struct NoAllocSetup {
  ProbDesc desc;
  PackJob jobs[kNoAllocMaxDims];
  int n_jobs;
  int n_tiles;
};

__global__ __launch_bounds__(256) void noalloc_setup_kernel(NoAllocSetup s, unsigned char* base) {
  ProbDesc* d = reinterpret_cast<ProbDesc*>(base + kOffDesc);
  WorkItem* items = reinterpret_cast<WorkItem*>(base + kOffItems);
  PackJob* jobs = reinterpret_cast<PackJob*>(base + kOffJobs);
  int* flag = reinterpret_cast<int*>(base + kOffFlag);
  const int t = threadIdx.x;
  if (t == 0) {
    *d = s.desc;
    *flag = 0;
  }
  if (t < s.n_jobs) jobs[t] = s.jobs[t];
  for (int i = t; i < s.n_tiles; i += blockDim.x) items[i] = WorkItem{0, i};
}

// out = NaN when the finite check (bit 0) or a gather (bit 1) flagged the data.
__global__ void noalloc_flag_kernel(const unsigned char* base, double* out) {
  if (*reinterpret_cast<const int*>(base + kOffFlag) != 0) *out = NAN;
}

// Per-device address of `scratch` (nullptr until looked up) and the outcome of the lookup.
constexpr int kMaxDevices = 64;
static unsigned char* g_scratch[kMaxDevices];
static hipError_t g_scratch_err[kMaxDevices];
static bool g_scratch_done[kMaxDevices];
static std::mutex g_scratch_mu;

// Called with `device` current: look up the array's address on this device and write the
// harmonic table into it, once per device.
hipError_t noalloc_init(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_done[device]) return g_scratch_err[device];
  void* ptr = nullptr;
  hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e == hipSuccess && ptr == nullptr) e = hipErrorInvalidSymbol;
  if (e == hipSuccess) {
    std::vector<double> h(kNoAllocMaxN + 1);
    ksg_build_harmonic(kNoAllocMaxN, h.data());
    e = hipMemcpy(static_cast<unsigned char*>(ptr) + kOffHtab, h.data(), sizeof(double) * h.size(),
                  hipMemcpyHostToDevice);
  }
  if (e != hipSuccess) (void)hipGetLastError();
  g_scratch[device] = e == hipSuccess ? static_cast<unsigned char*>(ptr) : nullptr;
  g_scratch_err[device] = e;
  g_scratch_done[device] = true;
  return e;
}

static unsigned char* noalloc_base(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return g_scratch_done[device] ? g_scratch[device] : nullptr;
}

}  // namespace ksg

using namespace ksg;

extern "C" int cmi_ksg_noalloc(ksg_ctx* c, const float* x, const float* y, const float* z, int64_t N,
                               const int32_t dims[3], int32_t k, double* out_nats) {
  if (!c) return KSG_EINVAL;
  if (!dims || !x || !y || !out_nats) return c->fail(KSG_EINVAL, "cmi_ksg_noalloc: null argument");
  const int dx = dims[0], dy = dims[1], dz = dims[2];
  const int D = dx + dy + dz;
  if (dx < 1 || dy < 1 || dz < 0 || D > kNoAllocMaxDims)
    return c->fail(KSG_EINVAL, "cmi_ksg_noalloc: dims (%d,%d,%d) outside d_x>=1, d_y>=1, d_z>=0, sum<=%d", dx, dy,
                   dz, kNoAllocMaxDims);
  if (dz > 0 && !z) return c->fail(KSG_EINVAL, "cmi_ksg_noalloc: z is NULL with d_z > 0");
  if (k < 1 || k > KSG_MAX_K) return c->fail(KSG_EINVAL, "cmi_ksg_noalloc: k=%d outside [1, %d]", k, KSG_MAX_K);
  if (N > kNoAllocMaxN)
    return c->fail(KSG_EINVAL, "cmi_ksg_noalloc: N=%lld above the limit %lld of the static scratch array",
                   (long long)N, (long long)kNoAllocMaxN);
  if (N <= k) return c->fail(KSG_ETOOFEW, "cmi_ksg_noalloc: N=%lld <= k=%d", (long long)N, k);
  unsigned char* base = noalloc_base(c->device);
  if (!base) return c->fail(KSG_EDEVICE, "cmi_ksg_noalloc: the scratch array of device %d is not set up", c->device);
  KSG_HIP(c, hipSetDevice(c->device));

  const int n = (int)N;
  const int n_pad = (int)((N + kPad - 1) / kPad * kPad);
  const int n_tiles = (n + kTileQ - 1) / kTileQ;
  float* pool = reinterpret_cast<float*>(base + kOffPool);

  // Canonical split: d_x <= d_y (the estimator is symmetric in X and Y), columns X, Y, Z.
  const bool swap = dx > dy;
  const int cdx = swap ? dy : dx, cdy = swap ? dx : dy;
  NoAllocSetup s;
  std::memset(&s, 0, sizeof s);
  for (int a = 0; a < D; ++a) {
    int src = a;
    if (swap) {
      if (a < cdx) src = dx + a;
      else if (a < cdx + cdy) src = a - cdx;
    }
    const float* col = src < dx ? x + (int64_t)src * N
                                : (src < dx + dy ? y + (int64_t)(src - dx) * N : z + (int64_t)(src - dx - dy) * N);
    PackJob& j = s.jobs[a];
    j.src = col;
    j.perm = nullptr;
    j.dst = pool + (int64_t)a * n_pad;
    j.n = n;
    j.n_pad = n_pad;
    j.order = nullptr;
    s.desc.col[a] = j.dst;
  }
  s.n_jobs = D;
  s.n_tiles = n_tiles;
  ProbDesc& d = s.desc;
  d.n = n;
  d.n_pad = n_pad;
  d.dx = cdx;
  d.dy = cdy;
  d.dz = dz;
  d.k = k;
  d.n_tiles = n_tiles;
  d.part_base = 0;
  d.variant = shape_id(cdx, cdy, dz);
  d.out_index = 0;
  d.swap_xy = swap ? 1 : 0;
  d.alg = 1;
  d.key_col = -1;
  const int shape = d.variant >= kGenericShape ? kGenericShape + D : d.variant;
  const int kp = k + 1 <= 5 ? 5 : (k + 1 <= 9 ? 9 : 17);

  const ProbDesc* d_desc = reinterpret_cast<const ProbDesc*>(base + kOffDesc);
  const WorkItem* d_items = reinterpret_cast<const WorkItem*>(base + kOffItems);
  double* d_partials = reinterpret_cast<double*>(base + kOffPartials);
  const PackJob* d_jobs = reinterpret_cast<const PackJob*>(base + kOffJobs);
  int* d_flag = reinterpret_cast<int*>(base + kOffFlag);
  const double* d_htab = reinterpret_cast<const double*>(base + kOffHtab);

  hipLaunchKernelGGL(noalloc_setup_kernel, dim3(1), dim3(256), 0, c->stream, s, base);
  KSG_HIP(c, hipGetLastError());
  KSG_HIP(c, launch_pack(d_jobs, D, n_pad, d_flag, c->stream));
  KSG_HIP(c, launch_finite_check(d_jobs, D, n_pad, d_flag, c->stream));
  KSG_HIP(c, launch_ksg_search(d_desc, d_items, n_tiles, d_htab, d_partials, shape, kp, c->stream));
  KSG_HIP(c, launch_finalize(d_desc, 1, d_partials, d_htab, out_nats, c->stream));
  hipLaunchKernelGGL(noalloc_flag_kernel, dim3(1), dim3(1), 0, c->stream, (const unsigned char*)base, out_nats);
  KSG_HIP(c, hipGetLastError());
  return KSG_OK;
}
