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
  // captured batches hold the addresses of these work buffers: a new address retires them
  if (&b == &pool || &b == &partials || &b == &ebuf || &b == &tbuf || &b == &htab) ++buf_gen;
  const size_t old_cap = b.cap;
  if (b.ptr) {
    KSG_HIP(this, hipFree(b.ptr));
    b.ptr = nullptr;
  }
  mem_held -= old_cap;
  b.cap = 0;
  size_t want = std::max(bytes, old_cap + old_cap / 2);  // grow by half at least
  want = (want + 4095) & ~size_t(4095);
  const size_t need = (bytes + 4095) & ~size_t(4095);
  if (mem_limit > 0 && mem_held + need > (size_t)mem_limit)
    return fail(KSG_ENOMEM, "%s needs %zu bytes; the context's workspace limit is %lld (holding %zu)", what, need,
                (long long)mem_limit, mem_held);
  if (mem_limit > 0 && mem_held + want > (size_t)mem_limit) want = need;
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
  mem_held += want;
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

extern "C" int ksg_version(void) { return 10100; }

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
  c->clear_graphs();
  if (c->capture_stream) (void)hipStreamDestroy(c->capture_stream);
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
    case KSG_OPT_USE_GRAPH:
      c->use_graph = value != 0;
      if (!c->use_graph) c->clear_graphs();
      return KSG_OK;
    case KSG_OPT_MEM_LIMIT:
      if (value < 0) return c->fail(KSG_EINVAL, "workspace limit must be >= 0 bytes (0 = none)");
      c->mem_limit = value;
      return KSG_OK;
    case KSG_OPT_TILE_Q:
      if (value != 0 && value != 64 && value != 128 && value != 256)
        return c->fail(KSG_EINVAL, "tile height must be 0 (tuned), 64, 128 or 256");
      c->tile_q = (int)value;
      return KSG_OK;
    case KSG_OPT_GROUP_CHUNK:
      if (value < 0 || value > (int64_t)1 << 31)
        return c->fail(KSG_EINVAL, "group chunk must lie in [0, 2^31] elements (0 = default)");
      c->group_chunk_elems = value;
      return KSG_OK;
    case KSG_OPT_WINDOWS:
      if (value < 0 || value > 2) return c->fail(KSG_EINVAL, "windows must be 0 (off), 1 (tuned) or 2 (from N = 2048)");
      c->use_windows = value != 0;
      c->windows_untuned = value == 2;
      return KSG_OK;
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

extern "C" int ksg_graph_stats(ksg_ctx* c, int64_t* captures, int64_t* replays, int64_t* held) {
  if (!c) return KSG_EINVAL;
  if (!captures || !replays || !held) return c->fail(KSG_EINVAL, "ksg_graph_stats: null output");
  *captures = c->graph_captures;
  *replays = c->graph_replays;
  *held = (int64_t)c->graphs.size();
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
