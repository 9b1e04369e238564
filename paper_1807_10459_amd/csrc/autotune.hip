// Autotuner of the launch shapes, by timing synthetic batches on the device:
//   1. the group size G in {8, 16} of the grouped kernels, per top-k width (k <= 4, k <= 8) and
//      conditioning dimension m = 0..14 (larger m are compiled for G = 8 only);
//   2. the tile height (queries per work-group: 64, 128 or 256) of the brute-force kernels, for
//      launches that fill the device with few work-groups and for those with many;
//   3. for single problems of D = 3..16 columns sharing an unpermuted Z column, the smallest N
//      from which the key-ordered window search beats the brute-force kernel (or never).
// Results can be cached in a small text file keyed by device architecture, compute-unit count
// and library version.
#include <hip/hip_runtime.h>

#include <climits>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/ksgcmi.h"
#include "internal.h"
#include "runtime.h"

namespace ksg {

// Uniform [0, 1) floats from a counter-based hash (splitmix64 finaliser) of (seed, index);
// tuning data only.
__global__ void tune_fill_kernel(float* __restrict__ out, int64_t n, uint64_t seed) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint64_t z = seed + 0x9E3779B97F4A7C15ull * (uint64_t)(i + 1);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  out[i] = (float)(z >> 40) * (1.0f / 16777216.0f);
}

// Row permutation i -> (a * i + b) mod n with gcd(a, n) = 1 (a surrogate-like gather for tuning).
__global__ void tune_perm_kernel(int32_t* __restrict__ perm, int n, int a, int b) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) perm[i] = (int32_t)(((int64_t)a * i + b) % n);
}

}  // namespace ksg

using namespace ksg;

namespace {

constexpr int kTuneWinD0 = 3;  // window thresholds are tuned for D = 3..16
constexpr int kTuneWinN[3] = {2048, 8192, 32768};
constexpr int kTuneCand = 40;  // candidate columns of the tuning data
constexpr int kTunedInts = 30 + 2 + (kMaxDimsCompiled + 1 - kTuneWinD0);  // 46

std::string tune_key(const ksg_ctx* c) {
  char buf[128];
  std::snprintf(buf, sizeof buf, "%s:%d:%d", c->arch, c->cus, ksg_version());
  return buf;
}

// Flat form: G (k <= 4) x15, G (k <= 8) x15, tile height small / large, window N for D = 3..16.
void to_flat(const ksg_ctx* c, int* v) {
  for (int t = 0; t < 2; ++t)
    for (int m = 0; m < 15; ++m) v[t * 15 + m] = c->tuned_g[t][m];
  v[30] = c->tuned_tq[0];
  v[31] = c->tuned_tq[1];
  for (int D = kTuneWinD0; D <= kMaxDimsCompiled; ++D) v[32 + D - kTuneWinD0] = c->tuned_win_n[D];
}

bool from_flat(ksg_ctx* c, const int* v) {
  for (int i = 0; i < 30; ++i)
    if (v[i] != 8 && v[i] != 16) return false;
  for (int i = 30; i < 32; ++i)
    if (v[i] != 64 && v[i] != 128 && v[i] != 256) return false;
  for (int i = 32; i < kTunedInts; ++i)
    if (v[i] < 0) return false;
  for (int t = 0; t < 2; ++t)
    for (int m = 0; m < 15; ++m) c->tuned_g[t][m] = v[t * 15 + m];
  c->tuned_tq[0] = v[30];
  c->tuned_tq[1] = v[31];
  for (int D = kTuneWinD0; D <= kMaxDimsCompiled; ++D) c->tuned_win_n[D] = v[32 + D - kTuneWinD0];
  return true;
}

// The cache file holds one line per device key: "<key> <the integers of the flat form>".
bool load_cache(ksg_ctx* c, const char* path) {
  FILE* f = std::fopen(path, "r");
  if (!f) return false;
  char key[128];
  int v[kTunedInts];
  bool found = false;
  while (!found && std::fscanf(f, "%127s", key) == 1) {
    int got = 0;
    for (int i = 0; i < kTunedInts; ++i) got += std::fscanf(f, "%d", &v[i]);
    if (got != kTunedInts) break;
    if (tune_key(c) == key) found = from_flat(c, v);
  }
  std::fclose(f);
  return found;
}

void save_cache(const ksg_ctx* c, const char* path) {
  FILE* f = std::fopen(path, "a");
  if (!f) return;
  int v[kTunedInts];
  to_flat(c, v);
  std::fprintf(f, "%s", tune_key(c).c_str());
  for (int i = 0; i < kTunedInts; ++i) std::fprintf(f, " %d", v[i]);
  std::fprintf(f, "\n");
  std::fclose(f);
}

// The fastest of `reps` runs after one warm-up run (device time between two events).
int time_batch(ksg_ctx* c, const std::vector<Problem>& probs, double* out, int reps, double* best_ms) {
  double tmin = 1e30;
  for (int rep = 0; rep <= reps; ++rep) {
    hipEvent_t e0 = c->get_event(), e1 = c->get_event();
    if (!e0 || !e1) return c->fail(KSG_EDEVICE, "events");
    KSG_HIP(c, hipEventRecord(e0, c->stream));
    int st = c->run_batch(probs, out);
    if (st) return st;
    KSG_HIP(c, hipEventRecord(e1, c->stream));
    KSG_HIP(c, hipEventSynchronize(e1));
    float ms = 0.0f;
    KSG_HIP(c, hipEventElapsedTime(&ms, e0, e1));
    c->event_pool.push_back(e0);
    c->event_pool.push_back(e1);
    if (rep > 0) tmin = std::min(tmin, (double)ms);  // the first run warms the code object
  }
  *best_ms = tmin;
  return KSG_OK;
}

// A tuning problem: X = candidate column x_col (through perm when given), Y and dz Z columns
// shared by every problem; columns are `stride` floats apart.
Problem tune_problem(const float* d, int64_t stride, int x_col, int dz, int64_t n, int k, const int32_t* perm,
                     int out_index) {
  Problem q;
  std::memset(&q, 0, sizeof q);
  q.n = n;
  q.dx = 1;
  q.dy = 1;
  q.dz = dz;
  q.k = k;
  q.col[0] = d + (int64_t)x_col * stride;
  q.perm[0] = perm;
  q.col[1] = d + (int64_t)kTuneCand * stride;
  for (int a = 0; a < dz; ++a) q.col[2 + a] = d + (int64_t)(kTuneCand + 1 + a) * stride;
  q.out_index = out_index;
  return q;
}

}  // namespace

extern "C" int ksg_autotune(ksg_ctx* c, int64_t n, const char* cache_path, int32_t* tuned_out) {
  if (!c) return KSG_EINVAL;
  if (n < 256 || n > (1 << 20)) return c->fail(KSG_EINVAL, "ksg_autotune: n must lie in [256, 2^20]");
  KSG_HIP(c, hipSetDevice(c->device));
  const bool cached = cache_path && load_cache(c, cache_path);
  if (!cached) {
    // tuning columns: 40 candidates, then Y and 14 Z columns, each `stride` floats
    const int64_t stride = std::max<int64_t>(n, kTuneWinN[2]);
    const int cols = kTuneCand + 1 + kGroupMaxM16;
    int st = c->reserve(c->embed, sizeof(float) * (size_t)cols * stride + sizeof(int32_t) * stride, "tuning data");
    if (st) return st;
    float* d = (float*)c->embed.ptr;
    int32_t* perm = reinterpret_cast<int32_t*>(d + (int64_t)cols * stride);
    hipLaunchKernelGGL(tune_fill_kernel, dim3((unsigned)(((int64_t)cols * stride + 255) / 256)), dim3(256), 0,
                       c->stream, d, (int64_t)cols * stride, (uint64_t)0x5eed);
    KSG_HIP(c, hipGetLastError());
    st = c->reserve(c->cmi, sizeof(double) * 64, "tuning output");
    if (st) return st;
    double* out = (double*)c->cmi.ptr;
    // the context's settings come back on every exit, errors included
    struct Restore {
      ksg_ctx* c;
      bool timing, check, windows, untuned, graph;
      int group, alg, tile_q;
      ~Restore() {
        c->timing = timing;
        c->check_finite = check;
        c->use_windows = windows;
        c->windows_untuned = untuned;
        c->use_graph = graph;
        c->group_size = group;
        c->algorithm = alg;
        c->tile_q = tile_q;
      }
    } restore{c,           c->timing,     c->check_finite, c->use_windows, c->windows_untuned,
              c->use_graph, c->group_size, c->algorithm,    c->tile_q};
    c->windows_untuned = false;
    c->check_finite = false;
    c->use_graph = false;
    c->timing = false;
    c->algorithm = 1;  // every tuned launch shape belongs to algorithm 1
    c->tile_q = 0;
    c->tuned = false;  // the tuning runs use the fixed defaults

    // ---- 1. group size per (k bucket, m): 32 problems of n points sharing Y and Z ----
    const int n_x = 32;
    for (int t = 0; t < 2; ++t) {
      const int k = t == 0 ? 4 : 8;
      for (int m = 0; m <= kGroupMaxM16; ++m) {
        std::vector<Problem> probs;
        for (int i = 0; i < n_x; ++i) probs.push_back(tune_problem(d, stride, i, m, n, k, nullptr, i));
        double best = 1e30;
        int best_g = 8;
        for (int G : {8, 16}) {
          c->group_size = G;
          double ms = 0.0;
          if ((st = time_batch(c, probs, out, 2, &ms))) return st;
          if (ms < best) {
            best = ms;
            best_g = G;
          }
        }
        c->tuned_g[t][m] = best_g;
      }
    }
    c->group_size = 0;  // single problems from here on

    // ---- 2. tile height of the brute-force kernels: a launch of few work-groups (16 problems of
    // 1024 points: 64 tiles of 256) and one of many (64 problems of 4096 points: 1024 tiles) ----
    c->use_windows = false;
    const int64_t tq_n[2] = {1024, 4096};
    const int tq_p[2] = {16, 64};
    for (int cls = 0; cls < 2; ++cls) {
      std::vector<Problem> probs;
      for (int i = 0; i < tq_p[cls]; ++i) probs.push_back(tune_problem(d, stride, i % kTuneCand, 1, tq_n[cls], 4, nullptr, i));
      double best = 1e30;
      int best_tq = kTileQ;
      for (int tq : {256, 128, 64}) {
        c->tile_q = tq;
        double ms = 0.0;
        if ((st = time_batch(c, probs, out, 2, &ms))) return st;
        if (ms < 0.97 * best) {  // a smaller tile must win clearly
          best = ms;
          best_tq = tq;
        }
      }
      c->tuned_tq[cls] = best_tq;
    }
    c->tile_q = 0;

    // ---- 3. window search against brute force, per column count: 4 problems (the original and
    // three row gathers of X) sharing Y and Z, at N = 2048, 8192, 32768 ----
    for (int D = kTuneWinD0; D <= kMaxDimsCompiled; ++D) {
      int win_n = INT_MAX;
      for (int ni = 0; ni < 3 && win_n == INT_MAX; ++ni) {
        const int64_t nn = kTuneWinN[ni];
        hipLaunchKernelGGL(tune_perm_kernel, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, c->stream, perm,
                           (int)nn, 7919, 17);
        KSG_HIP(c, hipGetLastError());
        std::vector<Problem> probs;
        for (int i = 0; i < 4; ++i) probs.push_back(tune_problem(d, stride, i, D - 2, nn, 4, i == 0 ? nullptr : perm, i));
        double ms_win = 0.0, ms_bf = 0.0;
        c->use_windows = true;
        if ((st = time_batch(c, probs, out, 2, &ms_win))) return st;
        c->use_windows = false;
        if ((st = time_batch(c, probs, out, 2, &ms_bf))) return st;
        if (ms_win < ms_bf) win_n = (int)nn;
      }
      c->tuned_win_n[D] = win_n;
    }
    if (cache_path) save_cache(c, cache_path);
  }
  c->tuned = true;
  if (tuned_out) to_flat(c, tuned_out);
  return KSG_OK;
}
