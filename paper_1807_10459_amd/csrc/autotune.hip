// Autotuner of the grouped search kernel: for every conditioning dimension m and top-k width,
// time the group sizes on a synthetic batch of the device and keep the fastest.  Results
// can be cached in a small JSON file keyed by device architecture, compute-unit count and
// library version.
#include <hip/hip_runtime.h>

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

}  // namespace ksg

using namespace ksg;

static std::string tune_key(const ksg_ctx* c) {
  char buf[128];
  std::snprintf(buf, sizeof buf, "%s:%d:%d", c->arch, c->cus, ksg_version());
  return buf;
}

// The cache file holds one line per device key: "<key> <kp5 sizes x15> <kp9 sizes x15>".
static bool load_cache(ksg_ctx* c, const char* path) {
  FILE* f = std::fopen(path, "r");
  if (!f) return false;
  char key[128];
  int g[30];
  bool found = false;
  while (!found && std::fscanf(f, "%127s", key) == 1) {
    int got = 0;
    for (int i = 0; i < 30; ++i) got += std::fscanf(f, "%d", &g[i]);
    if (got != 30) break;
    if (tune_key(c) == key) {
      bool ok = true;
      for (int i = 0; i < 30; ++i) ok = ok && (g[i] == 8 || g[i] == 16);
      if (ok) {
        for (int i = 0; i < 15; ++i) {
          c->tuned_g[0][i] = g[i];
          c->tuned_g[1][i] = g[15 + i];
        }
        found = true;
      }
    }
  }
  std::fclose(f);
  return found;
}

static void save_cache(const ksg_ctx* c, const char* path) {
  FILE* f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f, "%s", tune_key(c).c_str());
  for (int t = 0; t < 2; ++t)
    for (int i = 0; i < 15; ++i) std::fprintf(f, " %d", c->tuned_g[t][i]);
  std::fprintf(f, "\n");
  std::fclose(f);
}

extern "C" int ksg_autotune(ksg_ctx* c, int64_t n, const char* cache_path, int32_t* tuned_out) {
  if (!c) return KSG_EINVAL;
  if (n < 256 || n > (1 << 20)) return c->fail(KSG_EINVAL, "ksg_autotune: n must lie in [256, 2^20]");
  KSG_HIP(c, hipSetDevice(c->device));
  bool cached = cache_path && load_cache(c, cache_path);
  if (!cached) {
    const int n_x = 32;                       // X columns (one step's candidates x rounds)
    const int cols = n_x + 1 + kGroupMaxM16;  // X..., Y, Z1..Z14 (larger m always use groups of 8)
    int st = c->reserve(c->embed, sizeof(float) * (size_t)cols * n, "tuning data");
    if (st) return st;
    float* d = (float*)c->embed.ptr;
    hipLaunchKernelGGL(tune_fill_kernel, dim3((unsigned)(((int64_t)cols * n + 255) / 256)), dim3(256), 0,
                       c->stream, d, (int64_t)cols * n, (uint64_t)0x5eed);
    KSG_HIP(c, hipGetLastError());
    st = c->reserve(c->cmi, sizeof(double) * n_x, "tuning output");
    if (st) return st;
    // the context's settings come back on every exit, errors included
    struct Restore {
      ksg_ctx* c;
      bool timing, check;
      int group, alg;
      ~Restore() {
        c->timing = timing;
        c->check_finite = check;
        c->group_size = group;
        c->algorithm = alg;
      }
    } restore{c, c->timing, c->check_finite, c->group_size, c->algorithm};
    c->check_finite = false;
    c->algorithm = 1;  // the group size only matters to algorithm 1 (algorithm 2 is not grouped)
    for (int t = 0; t < 2; ++t) {
      const int k = t == 0 ? 4 : 8;
      for (int m = 0; m <= kGroupMaxM16; ++m) {
        std::vector<Problem> probs(n_x);
        for (int i = 0; i < n_x; ++i) {
          Problem& q = probs[i];
          std::memset(&q, 0, sizeof q);
          q.n = n;
          q.dx = 1;
          q.dy = 1;
          q.dz = m;
          q.k = k;
          q.col[0] = d + (int64_t)i * n;
          q.col[1] = d + (int64_t)n_x * n;
          for (int a = 0; a < m; ++a) q.col[2 + a] = d + (int64_t)(n_x + 1 + a) * n;
          q.out_index = i;
        }
        double best = 1e30;
        int best_g = 8;
        for (int G : {8, 16}) {
          c->group_size = G;
          double tmin = 1e30;
          for (int rep = 0; rep < 3; ++rep) {
            hipEvent_t e0 = c->get_event(), e1 = c->get_event();
            if (!e0 || !e1) return c->fail(KSG_EDEVICE, "events");
            KSG_HIP(c, hipEventRecord(e0, c->stream));
            st = c->run_batch(probs, (double*)c->cmi.ptr);
            if (st) return st;
            KSG_HIP(c, hipEventRecord(e1, c->stream));
            KSG_HIP(c, hipEventSynchronize(e1));
            float ms = 0.0f;
            KSG_HIP(c, hipEventElapsedTime(&ms, e0, e1));
            c->event_pool.push_back(e0);
            c->event_pool.push_back(e1);
            if (rep > 0) tmin = std::min(tmin, (double)ms);  // first run warms the code object
          }
          if (tmin < best) {
            best = tmin;
            best_g = G;
          }
        }
        c->tuned_g[t][m] = best_g;
      }
    }
    if (cache_path) save_cache(c, cache_path);
  }
  if (tuned_out)
    for (int t = 0; t < 2; ++t)
      for (int m = 0; m < 15; ++m) tuned_out[t * 15 + m] = c->tuned_g[t][m];
  return KSG_OK;
}
