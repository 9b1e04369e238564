"""Feature vector of one greedy step for the learned-null gate, in FP64 (test infrastructure only).

The paper gives no learned null; the 16 features are the library's own choice:
the sample size, the dimensions, k, sample moments of the columns and the
candidates' CMI values.  All moments are population
moments of FP32 columns accumulated in FP64; CMI values are scaled by sqrt(N)
so that they are O(1) across sample sizes.

  0 log N          1 d_x      2 d_y        3 d_z       4 k
  5 log c          6 log P    7 sqrt(N) T_obs (largest original CMI)
  8 sqrt(N) * second-largest original CMI (= T_obs when c = 1)
  9 sqrt(N) * mean original CMI          10 sqrt(N) * population sd of original CMIs
 11 skewness(Y)   12 excess kurtosis(Y)
 13 mean over candidates of skewness(X_c)
 14 mean over candidates of excess kurtosis(X_c)
 15 mean over candidates of |lag-1 autocorrelation(X_c)| (pooled order)
"""
from __future__ import annotations

import math

import numpy as np

N_FEATURES = 16


def column_moments(col):
    """(skewness, excess kurtosis, lag-1 autocorrelation) of one FP32 column, FP64 arithmetic."""
    a = np.asarray(col, dtype=np.float64)
    n = a.size
    mu = math.fsum(a.tolist()) / n
    d = a - mu
    m2 = math.fsum((d * d).tolist()) / n
    m3 = math.fsum((d ** 3).tolist()) / n
    m4 = math.fsum((d ** 4).tolist()) / n
    c1 = math.fsum((d[:-1] * d[1:]).tolist()) / n
    if m2 <= 0.0:
        return 0.0, 0.0, 0.0
    return m3 / m2 ** 1.5, m4 / (m2 * m2) - 3.0, c1 / m2


def step_features(n: int, dx: int, dy: int, dz: int, k: int, n_perm: int, orig_cmis,
                  y_moments, cand_moments) -> np.ndarray:
    """orig_cmis: the c original CMIs of the step; *_moments from ``column_moments``."""
    cm = np.asarray(orig_cmis, dtype=np.float64)
    c = cm.size
    s = math.sqrt(n)
    srt = np.sort(cm)[::-1]
    second = srt[1] if c > 1 else srt[0]
    mean = math.fsum(cm.tolist()) / c
    sd = math.sqrt(math.fsum(((cm - mean) ** 2).tolist()) / c)
    cmom = np.asarray(cand_moments, dtype=np.float64).reshape(-1, 3)
    return np.array([
        math.log(n), dx, dy, dz, k, math.log(c), math.log(n_perm),
        s * srt[0], s * second, s * mean, s * sd,
        y_moments[0], y_moments[1],
        math.fsum(cmom[:, 0].tolist()) / c,
        math.fsum(cmom[:, 1].tolist()) / c,
        math.fsum(np.abs(cmom[:, 2]).tolist()) / c,
    ], dtype=np.float64)
