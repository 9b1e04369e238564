// Driver of the library's host-only code (csrc/host_stats.cpp) for a build with the host
// sanitizers: harmonic table, Benjamini-Hochberg, sequential max-statistic test, on edge cases
// and random inputs.  Exits non-zero on a failed check; the sanitizers abort on any memory or
// undefined-behaviour error.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "../include/ksgcmi.h"

static int failures = 0;
#define CHECK(cond)                                             \
  do {                                                          \
    if (!(cond)) {                                              \
      std::fprintf(stderr, "check failed: %s (line %d)\n", #cond, __LINE__); \
      ++failures;                                               \
    }                                                           \
  } while (0)

int main() {
  // harmonic numbers: H_0 = 0, H_1 = 1, H_3 = 11/6, increasing, H_n - ln n -> Euler's gamma
  std::vector<double> h(200001);
  CHECK(ksg_harmonic_table(200000, h.data()) == KSG_OK);
  CHECK(h[0] == 0.0 && h[1] == 1.0 && std::fabs(h[3] - 11.0 / 6.0) < 1e-15);
  for (size_t n = 1; n < h.size(); ++n) CHECK(h[n] > h[n - 1]);
  CHECK(std::fabs(h[200000] - std::log(200000.0) - 0.5772156649015329) < 1e-5);
  CHECK(ksg_harmonic_table(-1, h.data()) == KSG_EINVAL && ksg_harmonic_table(5, nullptr) == KSG_EINVAL);
  CHECK(ksg_harmonic_table(0, h.data()) == KSG_OK);

  std::mt19937_64 g(7);
  std::uniform_real_distribution<double> u(0.0, 1.0);
  // Benjamini-Hochberg: empty input, ties, random inputs; the rejected set is a prefix of the
  // sorted p-values and satisfies the step-up rule
  CHECK(ksg_fdr_bh(nullptr, 0, 0.05, nullptr) == KSG_EINVAL);
  {
    std::vector<double> p0;
    std::vector<int32_t> r0(1);
    CHECK(ksg_fdr_bh(p0.data() ? p0.data() : h.data(), 0, 0.05, r0.data()) == KSG_OK);
  }
  for (int trial = 0; trial < 500; ++trial) {
    const int n = 1 + (int)(u(g) * 60);
    std::vector<double> p(n);
    for (double& v : p) v = std::round(u(g) * 40) / 400.0;  // coarse: ties
    std::vector<int32_t> rej(n, -1);
    CHECK(ksg_fdr_bh(p.data(), n, 0.1, rej.data()) == KSG_OK);
    double max_rej = -1, min_keep = 2;
    int k = 0;
    for (int i = 0; i < n; ++i) {
      CHECK(rej[i] == 0 || rej[i] == 1);
      if (rej[i]) {
        ++k;
        max_rej = std::max(max_rej, p[i]);
      } else {
        min_keep = std::min(min_keep, p[i]);
      }
    }
    CHECK(max_rej <= min_keep);
    if (k > 0) CHECK(max_rej <= k * 0.1 / n);
  }
  CHECK(ksg_fdr_bh(h.data(), 3, 1.5, nullptr) == KSG_EINVAL);

  // sequential max statistic: random tables with ties, rows 0..8, the first rank that is not
  // significant ends the test
  for (int trial = 0; trial < 500; ++trial) {
    const int rows = (int)(u(g) * 9), P = 1 + (int)(u(g) * 50);
    std::vector<double> t((size_t)rows * (P + 1));
    for (double& v : t) v = std::round(u(g) * 20) / 20.0;
    std::vector<int32_t> sig(rows + 1, -1);
    std::vector<double> pv(rows + 1, -1.0);
    CHECK(ksg_maxstat_sequential(rows ? t.data() : h.data(), rows, P, 0.05, sig.data(), pv.data()) == KSG_OK);
    for (int i = 0; i < rows; ++i) {
      CHECK(sig[i] == 0 || sig[i] == 1);
      CHECK(pv[i] >= 0.0 && pv[i] <= 1.0);
      if (sig[i]) CHECK(pv[i] < 0.05);
    }
  }
  CHECK(ksg_maxstat_sequential(h.data(), 2, 0, 0.05, nullptr, nullptr) == KSG_EINVAL);

  if (failures) {
    std::fprintf(stderr, "%d checks failed\n", failures);
    return 1;
  }
  std::printf("host code clean under the sanitizers\n");
  return 0;
}
