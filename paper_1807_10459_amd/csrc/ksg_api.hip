// Host runtime behind the C ABI: context, workspace, harmonic-number table, work queue,
// batched launches, max-statistic test and the greedy parent-selection driver.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <map>
#include <unordered_map>
#include <vector>

#include "../../include/ksgcmi.h"
#include "internal.h"
#include "runtime.h"

using namespace ksg;

// ============================================================== errors

int ksg_ctx::fail(int status, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  err = buf;
  return status;
}

int ksg_ctx::hip_fail(hipError_t e, const char* what) {
  return fail(e == hipErrorOutOfMemory ? KSG_ENOMEM : KSG_EDEVICE, "%s: %s", what,
              hipGetErrorString(e));
}


// ============================================================== device buffers

int ksg_ctx::reserve(DevBuf& b, size_t bytes, const char* what) {
  if (b.cap >= bytes) return KSG_OK;
  // Pending work may still read the old buffer.
  KSG_HIP(this, hipStreamSynchronize(stream));
  if (b.ptr) {
    KSG_HIP(this, hipFree(b.ptr));
    b.ptr = nullptr;
    b.cap = 0;
  }
  size_t want = std::max(bytes, b.cap + b.cap / 2);
  want = (want + 4095) & ~size_t(4095);
  hipError_t e = hipMalloc(&b.ptr, want);
  if (e != hipSuccess) {
    want = (bytes + 4095) & ~size_t(4095);
    (void)hipGetLastError();
    e = hipMalloc(&b.ptr, want);
  }
  if (e != hipSuccess) {
    b.ptr = nullptr;
    (void)hipGetLastError();
    return fail(KSG_ENOMEM, "cannot allocate %zu bytes for %s", bytes, what);
  }
  b.cap = want;
  return KSG_OK;
}

int ksg_ctx::reserve_host(size_t bytes) {
  if (staging_cap >= bytes) return wait_staging();
  int st = wait_staging();
  if (st) return st;
  if (staging) KSG_HIP(this, hipHostFree(staging));
  staging = nullptr;
  size_t want = std::max(bytes, staging_cap * 2);
  want = (want + 4095) & ~size_t(4095);
  hipError_t e = hipHostMalloc(&staging, want, hipHostMallocDefault);
  if (e != hipSuccess) {
    staging = nullptr;
    staging_cap = 0;
    (void)hipGetLastError();
    return fail(KSG_ENOMEM, "cannot allocate %zu bytes of pinned host memory", want);
  }
  staging_cap = want;
  return KSG_OK;
}

int ksg_ctx::wait_staging() {
  if (staging_pending) {
    KSG_HIP(this, hipEventSynchronize(staging_done));
    staging_pending = false;
  }
  return KSG_OK;
}

// Harmonic numbers H_0..H_nmax in FP64 from a double-double running sum of 1/m (the
// remainder of each reciprocal comes from an exact fused multiply-add), rounded once.
void ksg_build_harmonic(int64_t nmax, double* out) {
  double hi = 0.0, lo = 0.0;
  out[0] = 0.0;
  for (int64_t m = 1; m <= nmax; ++m) {
    const double dm = (double)m;
    const double r = 1.0 / dm;
    const double e = std::fma(-r, dm, 1.0) / dm;  // 1/m = r + e (to ~2^-106 relative)
    // (hi, lo) += (r, e): two-sum of the leading parts, then renormalise.
    const double s = hi + r;
    const double bb = s - hi;
    const double err = (hi - (s - bb)) + (r - bb);
    const double t = err + lo + e;
    hi = s + t;
    lo = t - (hi - s);
    out[m] = hi;
  }
}

int ksg_ctx::ensure_htab(int64_t n) {
  if (htab_n >= n) return KSG_OK;
  int64_t want = std::max<int64_t>(std::max<int64_t>(n, 2 * htab_n), 65536);
  std::vector<double> h(want + 1);
  ksg_build_harmonic(want, h.data());
  int st = reserve(htab, sizeof(double) * (want + 1), "harmonic table");
  if (st) return st;
  KSG_HIP(this, hipMemcpy(htab.ptr, h.data(), sizeof(double) * (want + 1), hipMemcpyHostToDevice));
  htab_n = want;
  return KSG_OK;
}

// ============================================================== context

extern "C" int ksg_version(void) { return 10000; }

extern "C" const char* ksg_status_string(int s) {
  switch (s) {
    case KSG_OK: return "ok";
    case KSG_EINVAL: return "invalid argument";
    case KSG_ETOOFEW: return "too few points (N <= k)";
    case KSG_ENONFINITE: return "non-finite input data";
    case KSG_ENOMEM: return "out of memory";
    case KSG_EDEVICE: return "HIP runtime error";
    case KSG_ENODEV: return "no HIP device";
    case KSG_EBUFSMALL: return "output buffer too small";
    default: return "unknown status";
  }
}

extern "C" int ksg_device_count(void) {
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  return n;
}

extern "C" int ksg_device_props_get(int32_t device, ksg_device_props* out) {
  if (!out) return KSG_EINVAL;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) {
    (void)hipGetLastError();
    return KSG_ENODEV;
  }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) {
    (void)hipGetLastError();
    return KSG_ENODEV;
  }
  std::memset(out, 0, sizeof *out);
  std::snprintf(out->name, sizeof out->name, "%s", prop.name);
  std::snprintf(out->arch, sizeof out->arch, "%s", prop.gcnArchName);
  out->cus = prop.multiProcessorCount;
  out->clock_khz = prop.clockRate;
  out->mem_clock_khz = prop.memoryClockRate;
  out->mem_bus_bits = prop.memoryBusWidth;
  out->total_mem = (int64_t)prop.totalGlobalMem;
  out->l2_bytes = prop.l2CacheSize;
  out->lds_per_cu = (int32_t)prop.maxSharedMemoryPerMultiProcessor;
  out->lds_per_block = (int32_t)prop.sharedMemPerBlock;
  out->wave_size = prop.warpSize;
  return KSG_OK;
}

extern "C" int ksg_harmonic_table(int64_t nmax, double* out) {
  if (nmax < 0 || !out) return KSG_EINVAL;
  ksg_build_harmonic(nmax, out);
  return KSG_OK;
}

extern "C" int ksg_ctx_create(ksg_ctx** out, int device, void* hip_stream) {
  if (!out) return KSG_EINVAL;
  *out = nullptr;
  const int nd = ksg_device_count();
  if (nd <= 0) return KSG_ENODEV;
  if (device < 0 || device >= nd) return KSG_EINVAL;
  if (hipSetDevice(device) != hipSuccess) {
    (void)hipGetLastError();
    return KSG_ENODEV;
  }
  ksg_ctx* c = new ksg_ctx();
  c->device = device;
  c->stream = (hipStream_t)hip_stream;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) {
    delete c;
    return KSG_EDEVICE;
  }
  c->cus = prop.multiProcessorCount;
  std::snprintf(c->arch, sizeof c->arch, "%s", prop.gcnArchName);
  if (hipMalloc(&c->d_counter, sizeof(int) * 4) != hipSuccess ||
      hipMemset(c->d_counter, 0, sizeof(int) * 4) != hipSuccess ||
      hipMalloc(&c->d_ms, sizeof(MaxStatOut) * 2) != hipSuccess ||
      hipEventCreateWithFlags(&c->staging_done, hipEventDisableTiming) != hipSuccess ||
      hipHostMalloc(&c->h_ms, sizeof(MaxStatOut) * 2, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    ksg_ctx_destroy(c);
    return KSG_ENOMEM;
  }
  c->d_flag = c->d_counter + 1;
  // cmi_ksg_noalloc's static array on this device: located once; a failure only disables that
  // entry point (it reports KSG_EDEVICE)
  (void)noalloc_init(device);
  *out = c;
  return KSG_OK;
}

extern "C" void ksg_ctx_destroy(ksg_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  for (DevBuf* b : {&c->htab, &c->pool, &c->desc, &c->items, &c->partials, &c->jobs, &c->tmp, &c->ebuf, &c->tbuf,
                    &c->embed, &c->cmi, &c->aux, &c->feat})
    if (b->ptr) (void)hipFree(b->ptr);
  if (c->d_counter) (void)hipFree(c->d_counter);
  if (c->d_ms) (void)hipFree(c->d_ms);
  if (c->d_work) (void)hipFree(c->d_work);
  if (c->h_ms) (void)hipHostFree(c->h_ms);
  if (c->staging) (void)hipHostFree(c->staging);
  if (c->staging_done) (void)hipEventDestroy(c->staging_done);
  for (int i = 0; i < ksg_ctx::kAuxStreams; ++i) {
    if (c->aux_streams[i]) {
      (void)hipStreamSynchronize(c->aux_streams[i]);
      (void)hipStreamDestroy(c->aux_streams[i]);
    }
    if (c->join_ev[i]) (void)hipEventDestroy(c->join_ev[i]);
  }
  if (c->fork_ev) (void)hipEventDestroy(c->fork_ev);
  for (auto& pr : c->timed) c->event_pool.insert(c->event_pool.end(), {pr.first, pr.second});
  for (auto& sp : c->spans) c->event_pool.insert(c->event_pool.end(), {sp.a, sp.b});
  for (hipEvent_t e : c->event_pool) (void)hipEventDestroy(e);
  (void)hipGetLastError();
  delete c;
}

extern "C" const char* ksg_last_error(const ksg_ctx* c) { return c ? c->err.c_str() : "null context"; }

extern "C" int ksg_ctx_set_option(ksg_ctx* c, int option, int64_t value) {
  if (!c) return KSG_EINVAL;
  switch (option) {
    case KSG_OPT_CHECK_FINITE: c->check_finite = value != 0; return KSG_OK;
    case KSG_OPT_GROUP_SIZE:
      if (value != -1 && value != 0 && value != 8 && value != 16)
        return c->fail(KSG_EINVAL, "group size must be -1 (tuned), 0 (off), 8 or 16");
      c->group_size = (int)value;
      return KSG_OK;
    case KSG_OPT_USE_GRAPH: c->use_graph = value != 0; return KSG_OK;
    case KSG_OPT_WINDOWS: c->use_windows = value != 0; return KSG_OK;
    case KSG_OPT_ALGORITHM:
      if (value != 1 && value != 2) return c->fail(KSG_EINVAL, "KSG algorithm must be 1 or 2");
      c->algorithm = (int)value;
      return KSG_OK;
    case KSG_OPT_TIMING:
      c->timing = value != 0;
      if (c->timing && !c->d_work) {
        if (hipMalloc(&c->d_work, 6 * sizeof(unsigned long long)) != hipSuccess ||
            hipMemset(c->d_work, 0, 6 * sizeof(unsigned long long)) != hipSuccess) {
          (void)hipGetLastError();
          c->d_work = nullptr;
          c->timing = false;
          return c->fail(KSG_ENOMEM, "timing counters");
        }
      }
      return KSG_OK;
    default: return c->fail(KSG_EINVAL, "unknown option %d", option);
  }
}

// ============================================================== batch engine

static int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

int ksg_ctx::validate(const Problem& p, int index) {
  const int D = p.dx + p.dy + p.dz;
  if (p.dx < 1 || p.dy < 1 || p.dz < 0 || D > KSG_MAX_DIMS)
    return fail(KSG_EINVAL, "problem %d: dims (%d,%d,%d) outside d_x>=1, d_y>=1, d_z>=0, sum<=%d",
                index, p.dx, p.dy, p.dz, KSG_MAX_DIMS);
  if (p.k < 1 || p.k > KSG_MAX_K)
    return fail(KSG_EINVAL, "problem %d: k=%d outside [1, %d]", index, p.k, KSG_MAX_K);
  if (algorithm == 2 && D > kMaxDimsCompiled)
    return fail(KSG_EINVAL, "problem %d: %d columns; KSG algorithm 2 supports at most %d", index, D,
                kMaxDimsCompiled);
  if (p.n > (int64_t)INT32_MAX - 1024)
    return fail(KSG_EINVAL, "problem %d: N=%lld too large", index, (long long)p.n);
  if (p.n <= p.k)
    return fail(KSG_ETOOFEW, "problem %d: N=%lld <= k=%d", index, (long long)p.n, p.k);
  for (int a = 0; a < D; ++a)
    if (!p.col[a]) return fail(KSG_EINVAL, "problem %d: null column %d", index, a);
  return KSG_OK;
}

namespace {

// A unit of scheduling: one problem (ungrouped) or one group, with all its tiles.
struct Unit {
  int id;
  int n_tiles;
  double cost;
};

// Work items for a list of units (already in longest-first order).  With many units, each
// unit goes whole to one of the 8 XCDs (least-loaded first) and the items are interleaved
// so that work-group b, which the dispatcher places on XCD b % 8, takes the next item of
// that XCD's list: a problem's columns are then read into one XCD's L2 only.  Empty slots
// (prob = -1) return at once.  With few units the plain order keeps every XCD busy.
std::vector<WorkItem> order_items(const std::vector<Unit>& units) {
  constexpr int kXcd = 8;
  std::vector<WorkItem> out;
  if ((int)units.size() < 4 * kXcd) {
    for (const Unit& u : units)
      for (int t = 0; t < u.n_tiles; ++t) out.push_back(WorkItem{u.id, t});
    return out;
  }
  std::vector<std::vector<WorkItem>> bins(kXcd);
  std::vector<double> load(kXcd, 0.0);
  for (const Unit& u : units) {
    int x = 0;
    for (int i = 1; i < kXcd; ++i)
      if (load[i] < load[x]) x = i;
    load[x] += u.cost;
    for (int t = 0; t < u.n_tiles; ++t) bins[x].push_back(WorkItem{u.id, t});
  }
  size_t L = 0;
  for (auto& b : bins) L = std::max(L, b.size());
  out.assign(L * kXcd, WorkItem{-1, 0});
  for (int x = 0; x < kXcd; ++x)
    for (size_t s = 0; s < bins[x].size(); ++s) out[s * kXcd + x] = bins[x][s];
  return out;
}

}  // namespace

// Problems that share Y, Z, N and k and differ only in a 1-D X column can be searched as a
// group (Y/Z distances computed once per pair for the whole group).
static bool groupable(const Problem& p) {
  if (p.dx != 1 || p.dy != 1 || p.dz > kGroupMaxM || p.k + 1 > 9) return false;
  if (p.eps_out || p.counts_out || p.local_out) return false;
  for (int a = 1; a < 2 + p.dz; ++a)
    if (p.perm[a]) return false;
  return true;
}

int ksg_ctx::run_batch(const std::vector<Problem>& probs, double* d_out) {
  const int np = (int)probs.size();
  if (np == 0) return KSG_OK;
  int64_t nmax = 0;
  for (int i = 0; i < np; ++i) {
    int st = validate(probs[i], i);
    if (st) return st;
    nmax = std::max<int64_t>(nmax, probs[i].n);
  }
  int st = ensure_htab(nmax);
  if (st) return st;

  // ---- grouping: problems with identical (N, k, Y, Z) and 1-D X ----
  std::vector<int> group_of(np, -1);
  std::vector<std::vector<int>> groups;  // member problem indices
  std::vector<int> group_size_of;        // G of each group's kernel
  if (group_size != 0 && algorithm == 1) {
    std::map<std::vector<intptr_t>, std::vector<int>> by_key;
    for (int i = 0; i < np; ++i) {
      const Problem& p = probs[i];
      if (!groupable(p)) continue;
      std::vector<intptr_t> key = {(intptr_t)p.n, p.k, p.dz, (intptr_t)p.col[1]};
      for (int a = 0; a < p.dz; ++a) key.push_back((intptr_t)p.col[2 + a]);
      by_key[key].push_back(i);
    }
    for (auto& kv : by_key) {
      const std::vector<int>& members = kv.second;
      if (members.size() < 2) continue;
      const int m = probs[members[0]].dz;
      int G = group_size > 0 ? group_size : tuned_group_size(m, probs[members[0]].k);
      if (m > kGroupMaxM16) G = 8;  // the wider conditioning sets are compiled for groups of 8
      for (size_t s = 0; s < members.size(); s += G) {
        std::vector<int> g(members.begin() + s, members.begin() + std::min(members.size(), s + (size_t)G));
        for (int i : g) group_of[i] = (int)groups.size();
        groups.push_back(g);
        group_size_of.push_back(G);
      }
    }
  }

  // ---- key-ordered windows: ungrouped problems (k <= 4, no per-point outputs, N large enough)
  // that share an unpermuted Z column are searched in the order of that column ----
  std::vector<int> win_of(np, -1), win_key(np, -1);  // window set, key column (original index)
  std::vector<std::pair<const float*, int64_t>> wsets;  // (key column, N)
  if (use_windows) {
    std::map<std::pair<const float*, int64_t>, int> by_key;
    for (int i = 0; i < np; ++i) {
      const Problem& p = probs[i];
      if (group_of[i] >= 0 || p.k + 1 > 5 || p.n < kWindowMinN || p.dz < 1 ||
          p.dx + p.dy + p.dz > kMaxDimsCompiled)
        continue;
      if (p.eps_out || p.counts_out || p.local_out) continue;
      int a_key = -1;
      for (int a = p.dx + p.dy; a < p.dx + p.dy + p.dz && a_key < 0; ++a)
        if (!p.perm[a]) a_key = a;
      if (a_key < 0) continue;
      const auto kk = std::make_pair(p.col[a_key], p.n);
      auto it = by_key.find(kk);
      if (it == by_key.end()) {
        it = by_key.emplace(kk, (int)wsets.size()).first;
        wsets.push_back(kk);
      }
      win_of[i] = it->second;
      win_key[i] = a_key;
    }
  }

  // ---- column pool: pack every column that is not already a padded device column ----
  // Grouped problems address all their columns through one pool, so they always pack; so do
  // window problems, in their set's key order.
  struct Key {
    const float* src;
    const int32_t* perm;
    int64_t n;
    int wset;
    bool operator==(const Key& o) const { return src == o.src && perm == o.perm && n == o.n && wset == o.wset; }
  };
  struct KeyHash {
    size_t operator()(const Key& k) const {
      return std::hash<const void*>()(k.src) * 31u ^ std::hash<const void*>()(k.perm) ^ (size_t)k.n ^
             ((size_t)(k.wset + 1) << 20);
    }
  };
  std::unordered_map<Key, int64_t, KeyHash> slot;
  std::vector<PackJob> jobs;
  int64_t pool_floats = 0;
  int max_pad = 0;
  std::vector<std::array<int64_t, kMaxDims>> col_off(np);
  for (int i = 0; i < np; ++i) {
    const Problem& p = probs[i];
    const int D = p.dx + p.dy + p.dz;
    const int64_t n_pad = round_up(p.n, kPad);
    max_pad = std::max<int>(max_pad, (int)n_pad);
    for (int a = 0; a < D; ++a) {
      if (p.padded[a] && !p.perm[a] && group_of[i] < 0 && win_of[i] < 0) {
        col_off[i][a] = -1;  // used in place
        continue;
      }
      Key key{p.col[a], p.perm[a], p.n, win_of[i]};
      auto it = slot.find(key);
      if (it == slot.end()) {
        it = slot.emplace(key, pool_floats).first;
        PackJob j;
        j.src = p.col[a];
        j.perm = p.perm[a];
        j.dst = reinterpret_cast<float*>(pool_floats);  // offset for now
        j.n = (int)p.n;
        j.n_pad = (int)n_pad;
        // window set index + 1 for now (the key order's address is known after the pool is reserved)
        j.order = win_of[i] >= 0 ? reinterpret_cast<const int32_t*>((intptr_t)(win_of[i] + 1)) : nullptr;
        jobs.push_back(j);
        pool_floats += n_pad;
      }
      col_off[i][a] = it->second;
    }
  }
  // ---- wide problems (16 < D <= 32, not grouped): searched as problems of kWideDims columns,
  // their Z filled up with a zero column of the pool (exact: see ksg_search_wide.hip).  The
  // column is zero in the N rows and +inf in the padding rows, like every column, so that the
  // padding never enters a count: one per distinct N. ----
  std::vector<char> wide(np, 0);
  std::vector<int64_t> zero_off(np, -1);
  bool any_wide = false;
  {
    std::map<int64_t, int64_t> zero_of_n;
    for (int i = 0; i < np; ++i) {
      const Problem& p = probs[i];
      wide[i] = group_of[i] < 0 && p.dx + p.dy + p.dz > kMaxDimsCompiled;
      if (!wide[i]) continue;
      any_wide = true;
      auto it = zero_of_n.find(p.n);
      if (it == zero_of_n.end()) {
        it = zero_of_n.emplace(p.n, pool_floats).first;
        PackJob j;
        std::memset(&j, 0, sizeof j);
        j.src = nullptr;                                // zeros, +inf padding
        j.dst = reinterpret_cast<float*>(pool_floats);  // offset for now
        j.n = (int)p.n;
        j.n_pad = (int)round_up(p.n, kPad);
        jobs.push_back(j);
        pool_floats += j.n_pad;
      }
      zero_off[i] = it->second;
    }
  }
  // key orders of the window sets (int32, n_pad entries each) follow the packed columns
  std::vector<int64_t> wsigma_off(wsets.size());
  for (size_t w = 0; w < wsets.size(); ++w) {
    wsigma_off[w] = pool_floats;
    pool_floats += round_up(wsets[w].second, kPad);
  }
  // Interleaved blocks of the groups follow the packed columns in the same pool.
  std::vector<int64_t> xi_off(groups.size()), yzi_off(groups.size()), sigma_off(groups.size());
  std::vector<int> write_yz(groups.size(), 0);
  {
    std::map<std::vector<int64_t>, std::pair<int64_t, int64_t>> yz_sets;  // block, key order
    for (size_t gi = 0; gi < groups.size(); ++gi) {
      const int i0 = groups[gi][0];
      const int64_t n_pad = round_up(probs[i0].n, kPad);
      xi_off[gi] = pool_floats;
      pool_floats += (int64_t)group_size_of[gi] * n_pad;
      std::vector<int64_t> key = {n_pad};
      for (int a = 1; a < 2 + probs[i0].dz; ++a) key.push_back(col_off[i0][a]);
      auto it = yz_sets.find(key);
      if (it == yz_sets.end()) {
        const int64_t block = pool_floats;
        pool_floats += (int64_t)(probs[i0].dz + 1) * n_pad;
        const int64_t order = pool_floats;  // int32 row indices, one per padded row
        pool_floats += n_pad;
        it = yz_sets.emplace(key, std::make_pair(block, order)).first;
        write_yz[gi] = 1;
      }
      yzi_off[gi] = it->second.first;
      sigma_off[gi] = it->second.second;
    }
  }
  if (!groups.empty() && pool_floats > (int64_t)UINT32_MAX)
    return fail(KSG_ENOMEM, "batch needs %lld pool floats, above the 2^32 addressable by groups",
                (long long)pool_floats);
  st = reserve(pool, sizeof(float) * std::max<int64_t>(pool_floats, 1), "column pool");
  if (st) return st;
  float* pool_base = static_cast<float*>(pool.ptr);
  for (PackJob& j : jobs) {
    j.dst = pool_base + reinterpret_cast<int64_t>(j.dst);
    if (j.order) j.order = reinterpret_cast<const int32_t*>(pool_base + wsigma_off[(intptr_t)j.order - 1]);
  }

  auto cost = [&](int i) {
    const Problem& p = probs[i];
    return (double)p.n * (double)p.n * (4.0 * (p.dx + p.dy + p.dz) + 2.0);
  };
  auto n_tiles_of = [&](int i) { return (int)((probs[i].n + kTileQ - 1) / kTileQ); };

  // ---- per-problem descriptors (search of ungrouped problems + finalisation of all) ----
  std::vector<int> order;
  for (int i = 0; i < np; ++i) order.push_back(i);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost(a) > cost(b); });
  std::vector<ProbDesc> descs(np);
  std::vector<int> desc_of(np);
  int part = 0;
  // Group partial slots first (contiguous per group), then ungrouped problems.
  std::vector<int> group_part(groups.size());
  for (size_t gi = 0; gi < groups.size(); ++gi) {
    group_part[gi] = part;
    part += (int)groups[gi].size() * n_tiles_of(groups[gi][0]);
  }
  int common_shape = -2;
  int kp = 5;
  int wide_kp = 5;
  for (int r = 0; r < np; ++r) {
    const int i = order[r];
    const Problem& p = probs[i];
    desc_of[i] = r;
    ProbDesc& d = descs[r];
    std::memset(&d, 0, sizeof d);
    const bool swap = p.dx > p.dy;
    const int dx = swap ? p.dy : p.dx, dy = swap ? p.dx : p.dy;
    const int D = p.dx + p.dy + p.dz;
    for (int a = 0; a < D; ++a) {
      int src = a;
      if (swap) {
        if (a < dx) src = p.dx + a;          // canonical X = original Y
        else if (a < dx + dy) src = a - dx;  // canonical Y = original X
      }
      d.col[a] = col_off[i][src] < 0 ? p.col[src] : pool_base + col_off[i][src];
    }
    if (wide[i])
      for (int a = D; a < kWideDims; ++a) d.col[a] = pool_base + zero_off[i];
    d.n = (int)p.n;
    d.n_pad = (int)round_up(p.n, kPad);
    d.dx = dx;
    d.dy = dy;
    d.dz = wide[i] ? kWideDims - dx - dy : p.dz;
    d.k = p.k;
    d.n_tiles = n_tiles_of(i);
    d.eps_out = p.eps_out;
    d.counts_out = p.counts_out;
    d.local_out = p.local_out;
    d.variant = shape_id(dx, dy, p.dz);
    d.out_index = p.out_index;
    d.swap_xy = swap ? 1 : 0;
    d.alg = algorithm;
    d.key_col = win_key[i];  // a Z column: its index is the same in the canonical order
    d.key_order = win_of[i] >= 0 ? reinterpret_cast<const int32_t*>(pool_base + wsigma_off[win_of[i]]) : nullptr;
    if (group_of[i] >= 0) {
      const int gi = group_of[i];
      const int g = (int)(std::find(groups[gi].begin(), groups[gi].end(), i) - groups[gi].begin());
      d.part_base = group_part[gi] + g * d.n_tiles;
    } else if (win_of[i] >= 0) {
      d.part_base = part;
      part += d.n_tiles;
    } else if (wide[i]) {
      d.part_base = part;
      part += d.n_tiles;
      wide_kp = std::max(wide_kp, p.k + 1 <= 5 ? 5 : (p.k + 1 <= 9 ? 9 : 17));
    } else {
      d.part_base = part;
      part += d.n_tiles;
      kp = std::max(kp, p.k + 1 <= 5 ? 5 : (p.k + 1 <= 9 ? 9 : 17));
      // generic shapes share a kernel when their column counts agree
      const int launch_shape = d.variant >= kGenericShape ? kGenericShape + D : d.variant;
      if (common_shape == -2) common_shape = launch_shape;
      else if (common_shape != launch_shape) common_shape = -1;
    }
  }

  // ungrouped work items (algorithm 2: one launch per column count, items in D order)
  struct Segment {
    int D, kp, off, count;
    double cost;  // brute-force operations of its problems (launch scheduling)
  };
  double plain_cost = 0.0;
  std::vector<Segment> segments;
  std::vector<WorkItem> items;
  if (algorithm == 2) {
    std::map<int, std::vector<Unit>> by_d;
    std::map<int, int> kp_of;
    for (int r = 0; r < np; ++r) {
      const Problem& p = probs[order[r]];
      if (win_of[order[r]] >= 0) continue;  // searched in key order below
      const int D = p.dx + p.dy + p.dz;
      by_d[D].push_back(Unit{r, descs[r].n_tiles, cost(order[r])});
      const int need = p.k + 1 <= 5 ? 5 : (p.k + 1 <= 9 ? 9 : 17);
      kp_of[D] = std::max(kp_of[D], need);
    }
    for (auto& kv : by_d) {
      std::vector<WorkItem> seg = order_items(kv.second);
      double c = 0.0;
      for (const Unit& u : kv.second) c += u.cost;
      segments.push_back(Segment{kv.first, kp_of[kv.first], (int)items.size(), (int)seg.size(), c});
      items.insert(items.end(), seg.begin(), seg.end());
    }
  } else {
    std::vector<Unit> units;
    for (int r = 0; r < np; ++r)
      if (group_of[order[r]] < 0 && win_of[order[r]] < 0 && !wide[order[r]])
        units.push_back(Unit{r, descs[r].n_tiles, cost(order[r])});
    for (const Unit& u : units) plain_cost += u.cost;
    items = order_items(units);
  }
  // items before the window and wide segments (brute-force items, or the algorithm-2 segments)
  const int n_plain_items = (int)items.size();
  // window problems: one launch per column count, after the other ungrouped items
  std::vector<Segment> wsegments;
  {
    std::map<int, std::vector<Unit>> by_d;
    for (int r = 0; r < np; ++r) {
      const Problem& p = probs[order[r]];
      if (win_of[order[r]] >= 0) by_d[p.dx + p.dy + p.dz].push_back(Unit{r, descs[r].n_tiles, cost(order[r])});
    }
    for (auto& kv : by_d) {
      std::vector<WorkItem> seg = order_items(kv.second);
      double c = 0.0;
      for (const Unit& u : kv.second) c += u.cost;
      wsegments.push_back(Segment{kv.first, 5, (int)items.size(), (int)seg.size(), c});
      items.insert(items.end(), seg.begin(), seg.end());
    }
  }
  // wide problems: one launch of the kernel compiled for kWideDims columns
  Segment wide_seg{kWideDims, wide_kp, (int)items.size(), 0, 0.0};
  if (any_wide) {
    std::vector<Unit> units;
    for (int r = 0; r < np; ++r)
      if (wide[order[r]]) units.push_back(Unit{r, descs[r].n_tiles, cost(order[r])});
    std::vector<WorkItem> seg = order_items(units);
    for (const Unit& u : units) wide_seg.cost += u.cost;
    wide_seg.count = (int)seg.size();
    items.insert(items.end(), seg.begin(), seg.end());
  }

  // ---- groups: descriptors, launch chunks, Y/Z count descriptors, work items ----
  // Groups of one (m, G, KP) class run as chunks of consecutive groups, each chunk three
  // launches: radius (eps to E), Y/Z counts (terms to T), X counts (partial sums).  A chunk's
  // E (FP32) and T (FP64) hold G x n_pad elements per group, at most kChunkElems in all.
  constexpr int64_t kChunkElems = int64_t(1) << 27;
  std::vector<GroupDesc> gdescs(groups.size());
  std::map<std::array<int, 3>, std::vector<int>> class_groups;  // in creation order
  for (size_t gi = 0; gi < groups.size(); ++gi) {
    const Problem& p0 = probs[groups[gi][0]];
    GroupDesc& gd = gdescs[gi];
    std::memset(&gd, 0, sizeof gd);
    const int i0 = groups[gi][0];
    for (int g = 0; g < kGroupMax; ++g) {
      const int i = groups[gi][g < (int)groups[gi].size() ? g : 0];
      gd.x_off[g] = (uint32_t)col_off[i][0];
    }
    gd.y_off = (uint32_t)col_off[i0][1];
    for (int a = 0; a < p0.dz; ++a) gd.z_off[a] = (uint32_t)col_off[i0][2 + a];
    gd.xi_off = (uint32_t)xi_off[gi];
    gd.yzi_off = (uint32_t)yzi_off[gi];
    gd.write_yz = write_yz[gi];
    gd.sigma_off = (uint32_t)sigma_off[gi];
    gd.G = group_size_of[gi];
    gd.n = (int)p0.n;
    gd.n_pad = (int)round_up(p0.n, kPad);
    gd.k = p0.k;
    gd.m = p0.dz;
    gd.ng = (int)groups[gi].size();
    gd.n_tiles = n_tiles_of(i0);
    gd.part_base = group_part[gi];
    const int gkp = p0.k + 1 <= 5 ? 5 : 9;
    class_groups[{p0.dz, group_size_of[gi], gkp}].push_back((int)gi);
  }
  struct Chunk {
    std::array<int, 3> cls;     // m, G, KP
    std::vector<WorkItem> items;  // radius and X count launches (same items)
    size_t item_off = 0;
    size_t ydesc_off = 0, n_ydesc = 0;
    size_t yitem_off = 0, n_yitems = 0;
  };
  std::vector<Chunk> chunks;
  std::vector<YZDesc> ydescs;
  std::vector<WorkItem> yitems;
  int64_t chunk_elems_max = 0;
  for (auto& kv : class_groups) {
    const std::vector<int>& gl = kv.second;
    size_t a = 0;
    while (a < gl.size()) {
      // the chunk: groups gl[a, b)
      int64_t elems = 0;
      size_t b = a;
      while (b < gl.size()) {
        const int64_t e = (int64_t)gdescs[gl[b]].G * gdescs[gl[b]].n_pad;
        if (b > a && elems + e > kChunkElems) break;
        gdescs[gl[b]].e_off = (uint32_t)elems;
        elems += e;
        ++b;
      }
      chunk_elems_max = std::max(chunk_elems_max, elems);
      Chunk c;
      c.cls = kv.first;
      std::vector<Unit> units;
      for (size_t q = a; q < b; ++q)
        units.push_back(Unit{gl[q], gdescs[gl[q]].n_tiles, cost(groups[gl[q]][0]) * gdescs[gl[q]].ng});
      std::stable_sort(units.begin(), units.end(), [](const Unit& u, const Unit& v) { return u.cost > v.cost; });
      c.items = order_items(units);
      // runs of consecutive groups of one Y/Z set -> slot ranges of at most kYZSlots
      c.ydesc_off = ydescs.size();
      size_t r0 = a;
      while (r0 < b) {
        size_t r1 = r0 + 1;
        while (r1 < b && gdescs[gl[r1]].yzi_off == gdescs[gl[r0]].yzi_off) ++r1;
        const GroupDesc& f = gdescs[gl[r0]];
        int n_valid = 0;  // groups are filled in order, only the last of a set can be short
        for (size_t q = r0; q < r1; ++q) n_valid = (int)(q - r0) * f.G + gdescs[gl[q]].ng;
        for (int s0 = 0; s0 < n_valid; s0 += kYZSlots) {
          YZDesc y;
          std::memset(&y, 0, sizeof y);
          y.yzi_off = f.yzi_off;
          y.e_off = f.e_off;
          y.n = f.n;
          y.n_pad = f.n_pad;
          y.G = f.G;
          y.slot0 = s0;
          y.n_slots = std::min(kYZSlots, n_valid - s0);
          const int di = (int)ydescs.size();
          ydescs.push_back(y);
          for (int row = 0; row < f.n; ++row) yitems.push_back(WorkItem{di, row});
        }
        r0 = r1;
      }
      c.n_ydesc = ydescs.size() - c.ydesc_off;
      chunks.push_back(std::move(c));
      a = b;
    }
  }
  if (!groups.empty()) {
    st = reserve(ebuf, sizeof(float) * chunk_elems_max, "group radii");
    if (!st) st = reserve(tbuf, sizeof(double) * chunk_elems_max, "group count terms");
    if (st) return st;
  }

  // ---- upload: one pinned staging block, one copy per array ----
  size_t n_gitems = 0;
  for (Chunk& c : chunks) {
    c.item_off = items.size() + n_gitems;
    n_gitems += c.items.size();
  }
  {
    size_t off = items.size() + n_gitems;
    size_t yoff = 0;
    for (Chunk& c : chunks) {
      // Y/Z items of the chunk: those whose descriptor lies in the chunk's range
      c.yitem_off = off;
      size_t cnt = 0;
      while (yoff < yitems.size() && (size_t)yitems[yoff].prob < c.ydesc_off + c.n_ydesc) {
        ++cnt;
        ++yoff;
      }
      c.n_yitems = cnt;
      off += cnt;
    }
  }
  const size_t n_all_items = items.size() + n_gitems + yitems.size();
  const size_t sz_desc = sizeof(ProbDesc) * np;
  const size_t sz_g = sizeof(GroupDesc) * gdescs.size();
  const size_t sz_y = sizeof(YZDesc) * ydescs.size();
  const size_t sz_items = sizeof(WorkItem) * n_all_items;
  const size_t sz_jobs = sizeof(PackJob) * jobs.size();
  st = reserve_host(sz_desc + sz_g + sz_y + sz_items + sz_jobs + 64);
  if (st) return st;
  st = reserve(desc, sz_desc + sz_g + sz_y, "descriptors");
  if (!st) st = reserve(this->items, std::max<size_t>(sz_items, 16), "work items");
  if (!st) st = reserve(this->jobs, std::max<size_t>(sz_jobs, 16), "pack jobs");
  if (!st) st = reserve(partials, sizeof(double) * std::max(part, 1), "partial sums");
  if (st) return st;
  char* h = static_cast<char*>(staging);
  std::memcpy(h, descs.data(), sz_desc);
  if (sz_g) std::memcpy(h + sz_desc, gdescs.data(), sz_g);
  if (sz_y) std::memcpy(h + sz_desc + sz_g, ydescs.data(), sz_y);
  char* hi = h + sz_desc + sz_g + sz_y;
  WorkItem* hw = reinterpret_cast<WorkItem*>(hi);
  if (!items.empty()) std::memcpy(hw, items.data(), sizeof(WorkItem) * items.size());
  for (const Chunk& c : chunks) std::memcpy(hw + c.item_off, c.items.data(), sizeof(WorkItem) * c.items.size());
  if (!yitems.empty()) std::memcpy(hw + items.size() + n_gitems, yitems.data(), sizeof(WorkItem) * yitems.size());
  char* hj = hi + sz_items;
  if (sz_jobs) std::memcpy(hj, jobs.data(), sz_jobs);
  KSG_HIP(this, hipMemcpyAsync(desc.ptr, h, sz_desc + sz_g + sz_y, hipMemcpyHostToDevice, stream));
  if (sz_items) KSG_HIP(this, hipMemcpyAsync(this->items.ptr, hi, sz_items, hipMemcpyHostToDevice, stream));
  if (sz_jobs) KSG_HIP(this, hipMemcpyAsync(this->jobs.ptr, hj, sz_jobs, hipMemcpyHostToDevice, stream));
  KSG_HIP(this, hipEventRecord(staging_done, stream));
  staging_pending = true;

  // ---- pack, optional finite check, search, finalise ----
  if (check_finite) KSG_HIP(this, hipMemsetAsync(d_flag, 0, sizeof(int), stream));
  for (size_t w = 0; w < wsets.size(); ++w)  // key orders first: the pack step reads them
    KSG_HIP(this, launch_window_rank(wsets[w].first, (int)wsets[w].second, (int)round_up(wsets[w].second, kPad),
                                     reinterpret_cast<int32_t*>(pool_base + wsigma_off[w]), stream));
  if (!jobs.empty()) {
    KSG_HIP(this, launch_pack((const PackJob*)this->jobs.ptr, (int)jobs.size(), max_pad, d_flag, stream));
  }
  if (check_finite) {
    // In-place columns are checked through identity jobs over their first n rows.
    std::vector<PackJob> all = jobs;
    for (int i = 0; i < np; ++i) {
      const Problem& p = probs[i];
      for (int a = 0; a < p.dx + p.dy + p.dz; ++a)
        if (col_off[i][a] < 0)
          all.push_back(PackJob{p.col[a], nullptr, const_cast<float*>(p.col[a]), (int)p.n, (int)p.n});
    }
    st = check_columns_finite(all, max_pad);
    if (st) return st;
  }
  const GroupDesc* d_gdesc = (const GroupDesc*)((char*)desc.ptr + sz_desc);
  const YZDesc* d_ydesc = (const YZDesc*)((char*)desc.ptr + sz_desc + sz_g);
  if (!groups.empty()) {
    KSG_HIP(this, launch_key_order(d_gdesc, (int)groups.size(), max_pad, pool_base, stream));
    KSG_HIP(this, launch_interleave(d_gdesc, (int)groups.size(), max_pad, pool_base, stream));
  }
  hipEvent_t t0 = nullptr, t1 = nullptr;
  if (timing) {
    t0 = get_event();
    t1 = get_event();
    if (!t0 || !t1) return fail(KSG_EDEVICE, "cannot create timing events");
    KSG_HIP(this, hipEventRecord(t0, stream));
  }
  const WorkItem* d_items = (const WorkItem*)this->items.ptr;
  float* d_e = static_cast<float*>(ebuf.ptr);
  double* d_t = static_cast<double*>(tbuf.ptr);
  unsigned long long* d_w = timing ? d_work : nullptr;
  // In timing mode every launch is bracketed by its own pair of events (per-kernel times),
  // recorded on the stream the launch goes to.
  hipEvent_t span_a = nullptr;
  auto span_begin = [&](hipStream_t st_) -> int {
    if (!timing) return KSG_OK;
    span_a = get_event();
    if (!span_a) return fail(KSG_EDEVICE, "cannot create timing events");
    KSG_HIP(this, hipEventRecord(span_a, st_));
    return KSG_OK;
  };
  auto span_end = [&](int kind, hipStream_t st_) -> int {
    if (!timing) return KSG_OK;
    hipEvent_t b = get_event();
    if (!b) return fail(KSG_EDEVICE, "cannot create timing events");
    KSG_HIP(this, hipEventRecord(b, st_));
    spans.push_back(Span{span_a, b, kind});
    return KSG_OK;
  };

  // Single-problem launches (one per column count or shape; none of them reads another's
  // output) are spread over the auxiliary streams, longest first onto the least-loaded
  // stream, so that launches too small to fill the device run side by side.  Grouped chunks
  // stay on the context's stream.
  struct Launch {
    int kind;  // 0 brute-force items, 1 window segment, 2 algorithm-2 segment, 3 wide problems
    int seg;
    double cost;
  };
  std::vector<Launch> launches;
  if (algorithm == 2) {
    for (size_t g = 0; g < segments.size(); ++g) launches.push_back(Launch{2, (int)g, segments[g].cost});
  } else if (n_plain_items > 0) {
    launches.push_back(Launch{0, 0, plain_cost});
  }
  for (size_t g = 0; g < wsegments.size(); ++g) launches.push_back(Launch{1, (int)g, wsegments[g].cost});
  if (wide_seg.count > 0) launches.push_back(Launch{3, 0, wide_seg.cost});
  const bool fork = launches.size() + (chunks.empty() ? 0 : 1) > 1;
  std::vector<hipStream_t> launch_stream(launches.size(), stream);
  bool aux_used[ksg_ctx::kAuxStreams] = {false, false, false};
  if (fork) {
    if ((st = ensure_aux_streams())) return st;
    std::vector<int> by_cost(launches.size());
    for (size_t i = 0; i < launches.size(); ++i) by_cost[i] = (int)i;
    std::stable_sort(by_cost.begin(), by_cost.end(),
                     [&](int a, int b) { return launches[a].cost > launches[b].cost; });
    // candidate streams: the context's (only when it runs no grouped chunk) and the auxiliaries
    std::vector<std::pair<hipStream_t, double>> load;
    if (chunks.empty()) load.emplace_back(stream, 0.0);
    for (int i = 0; i < ksg_ctx::kAuxStreams; ++i) load.emplace_back(aux_streams[i], 0.0);
    for (int li : by_cost) {
      size_t best = 0;
      for (size_t j = 1; j < load.size(); ++j)
        if (load[j].second < load[best].second) best = j;
      load[best].second += launches[li].cost;
      launch_stream[li] = load[best].first;
      for (int i = 0; i < ksg_ctx::kAuxStreams; ++i)
        if (load[best].first == aux_streams[i]) aux_used[i] = true;
    }
    KSG_HIP(this, hipEventRecord(fork_ev, stream));
    for (int i = 0; i < ksg_ctx::kAuxStreams; ++i)
      if (aux_used[i]) KSG_HIP(this, hipStreamWaitEvent(aux_streams[i], fork_ev, 0));
  }
  // Every launch is enqueued by this lambda; whatever it returns, the auxiliary streams are
  // joined back before run_batch returns, so that later work on the context's stream (and
  // a buffer reallocation, which synchronises that stream) orders after them.
  auto enqueue_search = [&]() -> int {
    for (size_t li = 0; li < launches.size(); ++li) {
      const Launch& L = launches[li];
      const hipStream_t ls = launch_stream[li];
      if ((st = span_begin(ls))) return st;
      if (L.kind == 3) {
        KSG_HIP(this, launch_ksg_search((const ProbDesc*)desc.ptr, d_items + wide_seg.off, wide_seg.count,
                                        (const double*)htab.ptr, (double*)partials.ptr, kGenericShape + kWideDims,
                                        wide_seg.kp, ls));
      } else if (L.kind == 2) {
        const Segment& g = segments[L.seg];
        KSG_HIP(this, launch_ksg_alg2((const ProbDesc*)desc.ptr, d_items + g.off, g.count, (const double*)htab.ptr,
                                      (double*)partials.ptr, g.D, g.kp, ls));
      } else if (L.kind == 1) {
        const Segment& g = wsegments[L.seg];
        KSG_HIP(this, launch_ksg_window((const ProbDesc*)desc.ptr, d_items + g.off, g.count, (const double*)htab.ptr,
                                        (double*)partials.ptr, g.D, algorithm, d_w, ls));
      } else {
        KSG_HIP(this, launch_ksg_search((const ProbDesc*)desc.ptr, d_items, n_plain_items, (const double*)htab.ptr,
                                        (double*)partials.ptr, common_shape, kp, ls));
      }
      if ((st = span_end(3, ls))) return st;
    }
    for (const Chunk& c : chunks) {
      const int m = c.cls[0], G = c.cls[1], kp_c = c.cls[2];
      if ((st = span_begin(stream))) return st;
      KSG_HIP(this, launch_ksg_group_radius(pool_base, d_gdesc, d_items + c.item_off, (int)c.items.size(), d_e,
                                            m, G, kp_c, d_w, stream));
      if ((st = span_end(0, stream)) || (st = span_begin(stream))) return st;
      KSG_HIP(this, launch_ksg_yzcount(pool_base, d_ydesc, d_items + c.yitem_off, (int)c.n_yitems, d_e, d_t,
                                       (const double*)htab.ptr, m, d_w, stream));
      if ((st = span_end(1, stream)) || (st = span_begin(stream))) return st;
      KSG_HIP(this, launch_ksg_group_xcount(pool_base, d_gdesc, d_items + c.item_off, (int)c.items.size(), d_e,
                                            d_t, (const double*)htab.ptr, (double*)partials.ptr, m, G, d_w,
                                            stream));
      if ((st = span_end(2, stream))) return st;
    }
    return KSG_OK;
  };
  const int st_search = enqueue_search();
  if (fork) {
    for (int i = 0; i < ksg_ctx::kAuxStreams; ++i) {
      if (!aux_used[i]) continue;
      hipError_t e = hipEventRecord(join_ev[i], aux_streams[i]);
      if (e == hipSuccess) e = hipStreamWaitEvent(stream, join_ev[i], 0);
      if (e != hipSuccess) {
        (void)hipStreamSynchronize(aux_streams[i]);
        if (!st_search) return hip_fail(e, "joining an auxiliary stream");
      }
    }
  }
  if (st_search) return st_search;
  if (timing) {
    KSG_HIP(this, hipEventRecord(t1, stream));
    timed.emplace_back(t0, t1);
    // window problems are counted by their kernel over the work executed (ksg_take_timing)
    for (int i = 0; i < np; ++i)
      if (group_of[i] < 0 && win_of[i] < 0) timed_ops += algorithmic_ops(probs[i], 1);
  }
  KSG_HIP(this, launch_finalize((const ProbDesc*)desc.ptr, np, (const double*)partials.ptr,
                                (const double*)htab.ptr, d_out, stream));
  last_items = (int64_t)(items.size() + n_gitems + yitems.size());
  last_groups = (int64_t)groups.size();
  return KSG_OK;
}

// Algorithmic FP32 operations (the roofline's work count).
// Ungrouped problem: the brute-force count over ordered pairs, N(N-1)(4D+2) (radius: D sub,
// D-1 max, 1 compare; counts: D sub, D-1 max, 3 compares).
// Grouped problems are counted by the kernels themselves, over the work they executed.
// Radius and X count kernels, in units of 4 references x 64 lanes: the shared part once per
// pair for the whole group -- radius d^YZ (2m+1: m+1 sub, m max) and the skip test (1); X
// counts d^Z (2m-1) and the skip test (1), nothing when m = 0 -- and the per-problem part,
// radius 3 (sub, max, compare) and X counts 3 (sub, max, compare) per pair, for every problem
// whose step ran.  Y/Z count kernel, in operations: per visited reference d^Z and d^YZ
// (2m+1, or 1) and one binary-search compare per level per rank (two ranks, one when m = 0).
// Steps outside a wave's key window are not executed and not counted.
double ksg_ctx::algorithmic_ops(const Problem& p, int) {
  const double pairs = (double)p.n * (double)(p.n - 1);
  return pairs * (4.0 * (p.dx + p.dy + p.dz) + 2.0);
}

// Finite check over the destinations (first n rows) of the given jobs; synchronises.
int ksg_ctx::check_columns_finite(const std::vector<PackJob>& cols, int max_pad) {
  if (cols.empty()) return KSG_OK;
  const size_t sz = sizeof(PackJob) * cols.size();
  int st = reserve(aux, sz, "finite-check jobs");
  if (st) return st;
  KSG_HIP(this, hipMemcpyAsync(aux.ptr, cols.data(), sz, hipMemcpyHostToDevice, stream));
  KSG_HIP(this, launch_finite_check((const PackJob*)aux.ptr, (int)cols.size(), max_pad, d_flag, stream));
  int flag = 0;
  KSG_HIP(this, hipMemcpyAsync(&flag, d_flag, sizeof(int), hipMemcpyDeviceToHost, stream));
  KSG_HIP(this, hipStreamSynchronize(stream));
  if (flag & 2) return fail(KSG_EINVAL, "a row permutation holds an index outside [0, N)");
  if (flag) return fail(KSG_ENONFINITE, "input data contain NaN or infinity");
  return KSG_OK;
}

static void fill_problem(Problem& q, const ksg_problem& p, int out_index) {
  std::memset(&q, 0, sizeof q);
  q.n = p.n;
  q.dx = p.dx;
  q.dy = p.dy;
  q.dz = p.dz;
  q.k = p.k;
  const int D = p.dx + p.dy + p.dz;
  for (int a = 0; a < D && a < kMaxDims; ++a) {
    const float* base = a < p.dx ? p.x : (a < p.dx + p.dy ? p.y : p.z);
    const int c = a < p.dx ? a : (a < p.dx + p.dy ? a - p.dx : a - p.dx - p.dy);
    q.col[a] = base ? base + (int64_t)c * p.n : nullptr;
    q.perm[a] = a < p.dx ? p.perm_x : nullptr;
  }
  q.eps_out = p.eps_out;
  q.counts_out = p.counts_out;
  q.local_out = p.local_out;
  q.out_index = out_index;
}

extern "C" int cmi_ksg_batch(ksg_ctx* c, const ksg_problem* probs, int32_t n_probs, double* out) {
  if (!c) return KSG_EINVAL;
  if (n_probs < 0 || (n_probs > 0 && (!probs || !out)))
    return c->fail(KSG_EINVAL, "cmi_ksg_batch: null problems/output or negative count");
  std::vector<Problem> v(n_probs);
  for (int i = 0; i < n_probs; ++i) {
    if (probs[i].dx < 1 || probs[i].dy < 1 || probs[i].dz < 0 ||
        probs[i].dx + probs[i].dy + probs[i].dz > KSG_MAX_DIMS)
      return c->fail(KSG_EINVAL, "problem %d: dims (%d,%d,%d) outside d_x>=1, d_y>=1, d_z>=0, sum<=%d",
                     i, probs[i].dx, probs[i].dy, probs[i].dz, KSG_MAX_DIMS);
    if (probs[i].dz > 0 && !probs[i].z) return c->fail(KSG_EINVAL, "problem %d: z is NULL with d_z > 0", i);
    fill_problem(v[i], probs[i], i);
  }
  KSG_HIP(c, hipSetDevice(c->device));
  return c->run_batch(v, out);
}

extern "C" int cmi_ksg(ksg_ctx* c, const float* x, const float* y, const float* z, int64_t N,
                       const int32_t dims[3], int32_t k, double* out_nats) {
  if (!c) return KSG_EINVAL;
  if (!dims || !out_nats || !x || !y) return c->fail(KSG_EINVAL, "cmi_ksg: null argument");
  ksg_problem p;
  std::memset(&p, 0, sizeof p);
  p.n = N;
  p.dx = dims[0];
  p.dy = dims[1];
  p.dz = dims[2];
  p.k = k;
  p.x = x;
  p.y = y;
  p.z = z;
  int st = c->reserve(c->tmp, sizeof(double), "result");
  if (st) return st;
  st = cmi_ksg_batch(c, &p, 1, (double*)c->tmp.ptr);
  if (st) return st;
  KSG_HIP(c, hipMemcpyAsync(out_nats, c->tmp.ptr, sizeof(double), hipMemcpyDeviceToHost, c->stream));
  KSG_HIP(c, hipStreamSynchronize(c->stream));
  return KSG_OK;
}

// ============================================================== max statistic

int ksg_ctx::maxstat_async(const double* d_cmi, int cands, int P, double alpha, int slot) {
  if (cands < 1 || P < 1 || P > 4096)
    return fail(KSG_EINVAL, "max statistic: need c >= 1 and 1 <= P <= 4096 (c=%d, P=%d)", cands, P);
  if (!(alpha > 0.0 && alpha < 1.0)) return fail(KSG_EINVAL, "alpha must lie in (0, 1)");
  KSG_HIP(this, launch_maxstat(d_cmi, cands, P, alpha, d_ms + slot, stream));
  KSG_HIP(this, hipMemcpyAsync(h_ms + slot, d_ms + slot, sizeof(MaxStatOut), hipMemcpyDeviceToHost, stream));
  return KSG_OK;
}

static void to_public(const MaxStatOut& m, ksg_maxstat_result* out) {
  out->c_star = m.c_star;
  out->count = m.count;
  out->significant = m.significant;
  out->n_perm = m.n_perm;
  out->t_obs = m.t_obs;
  out->pval = m.pval;
  out->tau05 = m.tau05;
  out->tau01 = m.tau01;
}

extern "C" int ksg_maxstat(ksg_ctx* c, const double* cmi, int32_t cands, int32_t P, double alpha,
                           ksg_maxstat_result* out) {
  if (!c) return KSG_EINVAL;
  if (!cmi || !out) return c->fail(KSG_EINVAL, "ksg_maxstat: null argument");
  KSG_HIP(c, hipSetDevice(c->device));
  int st = c->maxstat_async(cmi, cands, P, alpha, 0);
  if (st) return st;
  KSG_HIP(c, hipStreamSynchronize(c->stream));
  to_public(c->h_ms[0], out);
  return KSG_OK;
}

// ============================================================== embedding

extern "C" int ksg_embed(ksg_ctx* c, const float* data, int32_t n_vars, int64_t T, int32_t n_trials,
                         int32_t target, int32_t max_lag, float* cand_out, float* y_out) {
  if (!c) return KSG_EINVAL;
  if (!data || !cand_out || !y_out) return c->fail(KSG_EINVAL, "ksg_embed: null argument");
  if (n_vars < 1 || n_trials < 1 || max_lag < 1 || T <= max_lag || target < 0 || target >= n_vars)
    return c->fail(KSG_EINVAL, "ksg_embed: bad sizes (n_vars=%d T=%lld n_trials=%d target=%d max_lag=%d)",
                   n_vars, (long long)T, n_trials, target, max_lag);
  const int64_t N = (int64_t)n_trials * (T - max_lag);
  if (N > (int64_t)INT32_MAX - 1024) return c->fail(KSG_EINVAL, "ksg_embed: N too large");
  KSG_HIP(c, hipSetDevice(c->device));
  KSG_HIP(c, launch_embed(data, n_vars, T, n_trials, target, max_lag, cand_out, y_out, N, c->stream));
  return KSG_OK;
}

// ============================================================== timing

int ksg_ctx::ensure_aux_streams() {
  if (fork_ev) return KSG_OK;
  // all or nothing: fork_ev is set last, and a failure releases what was created
  hipError_t e = hipSuccess;
  for (int i = 0; i < kAuxStreams && e == hipSuccess; ++i) {
    e = hipStreamCreateWithFlags(&aux_streams[i], hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&join_ev[i], hipEventDisableTiming);
  }
  hipEvent_t f = nullptr;
  if (e == hipSuccess) e = hipEventCreateWithFlags(&f, hipEventDisableTiming);
  if (e != hipSuccess) {
    for (int i = 0; i < kAuxStreams; ++i) {
      if (aux_streams[i]) (void)hipStreamDestroy(aux_streams[i]);
      if (join_ev[i]) (void)hipEventDestroy(join_ev[i]);
      aux_streams[i] = nullptr;
      join_ev[i] = nullptr;
    }
    return hip_fail(e, "creating the auxiliary streams");
  }
  fork_ev = f;
  return KSG_OK;
}

hipEvent_t ksg_ctx::get_event() {
  if (!event_pool.empty()) {
    hipEvent_t e = event_pool.back();
    event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return e;
}

extern "C" int ksg_take_timing(ksg_ctx* c, double* ms, int64_t* launches, double* ops) {
  if (!c) return KSG_EINVAL;
  if (!ms || !launches || !ops) return c->fail(KSG_EINVAL, "ksg_take_timing: null output");
  KSG_HIP(c, hipStreamSynchronize(c->stream));
  double total = 0.0;
  for (auto& pr : c->timed) {
    float t = 0.0f;
    KSG_HIP(c, hipEventElapsedTime(&t, pr.first, pr.second));
    total += t;
    c->event_pool.push_back(pr.first);
    c->event_pool.push_back(pr.second);
  }
  double kms[4] = {0, 0, 0, 0};
  int64_t kn[4] = {0, 0, 0, 0};
  for (auto& sp : c->spans) {
    float t = 0.0f;
    KSG_HIP(c, hipEventElapsedTime(&t, sp.a, sp.b));
    kms[sp.kind] += t;
    kn[sp.kind] += 1;
    c->event_pool.push_back(sp.a);
    c->event_pool.push_back(sp.b);
  }
  unsigned long long w[6] = {0, 0, 0, 0, 0, 0};
  if (c->d_work) {
    KSG_HIP(c, hipMemcpy(w, c->d_work, sizeof w, hipMemcpyDeviceToHost));
    KSG_HIP(c, hipMemset(c->d_work, 0, sizeof w));
  }
  for (int i = 0; i < 5; ++i) c->last_work[i] = w[i];
  // w[5]: operations / 256 executed by the key-ordered window search (single-problem kind)
  const double kops[4] = {256.0 * (3.0 * (double)w[0] + (double)w[2]), (double)w[3],
                          256.0 * (3.0 * (double)w[1] + (double)w[4]), c->timed_ops + 256.0 * (double)w[5]};
  for (int i = 0; i < 4; ++i) {
    c->last_kernel_ms[i] = kms[i];
    c->last_kernel_ops[i] = kops[i];
    c->last_kernel_launches[i] = kn[i];
  }
  *ms = total;
  *launches = (int64_t)c->timed.size();
  *ops = kops[0] + kops[1] + kops[2] + kops[3];
  c->timed.clear();
  c->spans.clear();
  c->timed_ops = 0.0;
  return KSG_OK;
}

extern "C" int ksg_last_kernels(ksg_ctx* c, double* ms, double* ops, int64_t* launches) {
  if (!c) return KSG_EINVAL;
  if (!ms || !ops || !launches) return c->fail(KSG_EINVAL, "ksg_last_kernels: null output");
  for (int i = 0; i < 4; ++i) {
    ms[i] = c->last_kernel_ms[i];
    ops[i] = c->last_kernel_ops[i];
    launches[i] = c->last_kernel_launches[i];
  }
  return KSG_OK;
}

extern "C" int ksg_last_work(ksg_ctx* c, uint64_t* counters) {
  if (!c) return KSG_EINVAL;
  if (!counters) return c->fail(KSG_EINVAL, "ksg_last_work: null output");
  for (int i = 0; i < 5; ++i) counters[i] = (uint64_t)c->last_work[i];
  return KSG_OK;
}
