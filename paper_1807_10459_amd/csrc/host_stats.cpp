// Host-only parts of the library: plain C++ with no HIP dependency, so that they also build
// with the host sanitizers (tests/test_host_sanitizers.py compiles this file with g++
// -fsanitize=address,undefined and runs a driver over it).
//   - the harmonic numbers H_n the digamma sums use (psi(n + 1) = H_n - Euler's gamma);
//   - Benjamini-Hochberg across targets;
//   - the sequential max-statistic test of the kept sources.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <functional>
#include <vector>

#include "../../include/ksgcmi.h"

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


extern "C" int ksg_harmonic_table(int64_t nmax, double* out) {
  if (nmax < 0 || !out) return KSG_EINVAL;
  ksg_build_harmonic(nmax, out);
  return KSG_OK;
}

extern "C" int ksg_fdr_bh(const double* pvals, int32_t n, double alpha, int32_t* reject) {
  if (!pvals || !reject || n < 0 || !(alpha > 0 && alpha < 1)) return KSG_EINVAL;
  std::vector<int> order(n);
  for (int i = 0; i < n; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return pvals[a] < pvals[b]; });
  int r = 0;
  for (int i = 0; i < n; ++i)
    if (pvals[order[i]] <= (double)(i + 1) * alpha / n) r = i + 1;
  for (int i = 0; i < n; ++i) reject[i] = 0;
  for (int i = 0; i < r; ++i) reject[order[i]] = 1;
  return KSG_OK;
}

extern "C" int ksg_maxstat_sequential(const double* table, int32_t rows, int32_t n_perm, double alpha,
                                      int32_t* significant, double* pval) {
  if (!table || !significant || !pval || rows < 0 || n_perm < 1 || !(alpha > 0 && alpha < 1)) return KSG_EINVAL;
  const int64_t W = (int64_t)n_perm + 1;
  std::vector<int> rank(rows);
  for (int i = 0; i < rows; ++i) rank[i] = i;
  // descending originals, the lower row first on ties
  std::stable_sort(rank.begin(), rank.end(), [&](int a, int b) { return table[a * W] > table[b * W]; });
  // every round's surrogate values in descending order: sorted[r][p] = r-th largest of round p
  std::vector<double> sorted((size_t)rows * n_perm), col(rows);
  for (int p = 0; p < n_perm; ++p) {
    for (int i = 0; i < rows; ++i) col[i] = table[i * W + 1 + p];
    std::sort(col.begin(), col.end(), std::greater<double>());
    for (int r = 0; r < rows; ++r) sorted[(size_t)r * n_perm + p] = col[r];
  }
  for (int i = 0; i < rows; ++i) {
    significant[i] = 0;
    pval[i] = 1.0;
  }
  for (int r = 0; r < rows; ++r) {
    const int i = rank[r];
    const double t = table[i * W];
    int count = 0;
    for (int p = 0; p < n_perm; ++p) count += sorted[(size_t)r * n_perm + p] >= t;
    pval[i] = (double)count / n_perm;
    if (!(pval[i] < alpha)) break;
    significant[i] = 1;
  }
  return KSG_OK;
}
