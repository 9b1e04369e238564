"""Embedding, surrogate max-statistic test and greedy parent selection (test infrastructure only).

The paper (Summary, network-inference paragraph) describes a greedy approach
that builds a parent set for each target by maximising a conditional MI
criterion over candidate past variables, with each inclusion gated - and the
inference stopped - by comparison with null distributions from surrogates;
the problem paragraph names control of errors from testing many sources.  It
gives no formulas; the readings taken here are:

* candidates: the target's own past and every source's past at lags
  1..max_lag, one pool, candidate index = var * max_lag + (lag - 1);
* embedded points: for each trial t = max_lag .. T-1, pooled trial-major;
* surrogates: uniform row permutations of the candidate column only (Y and
  the conditioning set stay fixed), one permutation per round shared by
  every candidate of a step (max-T / Westfall-Young form), supplied as data;
* max statistic: T_obs = max_c I_c (lowest index wins ties),
  T_p = max_c I_c^(p), p = #{p : T_p >= T_obs} / P, significant iff p < alpha;
* greedy: start with an empty conditioning set; include the argmax while
  the test is significant; stop at the first non-significant step or when
  the pool is empty;
* omnibus: I(selected source candidates ; Y | selected target-past
  candidates), surrogates permute the rows of the whole source block.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

from .ksg import ksg_cmi

__all__ = [
    "embed",
    "MaxStat",
    "max_statistic",
    "order_statistic_threshold",
    "greedy_select",
    "omnibus_test",
]


def embed(data, target: int, max_lag: int):
    """Lagged candidate columns [n_vars*max_lag][N] and target column [N], FP32.

    data: [n_trials][n_vars][T].  Candidate (v, l) holds x_v(t - l); Y holds
    x_target(t); t runs over max_lag .. T-1 in every trial, trials pooled in order.
    """
    data = np.asarray(data, dtype=np.float32)
    n_trials, n_vars, T = data.shape
    cols = []
    for v in range(n_vars):
        for lag in range(1, max_lag + 1):
            col = [data[tr, v, t - lag] for tr in range(n_trials) for t in range(max_lag, T)]
            cols.append(np.array(col, dtype=np.float32))
    y = np.array([data[tr, target, t] for tr in range(n_trials) for t in range(max_lag, T)],
                 dtype=np.float32)
    return np.stack(cols), y


@dataclasses.dataclass
class MaxStat:
    c_star: int
    t_obs: float
    count: int
    pval: float
    significant: bool
    tau05: float
    tau01: float
    t_max: np.ndarray  # per-round maxima T_p


def order_statistic_threshold(t_max: np.ndarray, alpha: float) -> float:
    """The ceil(alpha*P)-th largest per-round maximum (p < alpha iff T_obs > this)."""
    r = int(math.ceil(alpha * t_max.size))
    r = min(max(r, 1), t_max.size)
    return float(np.sort(t_max)[::-1][r - 1])


def max_statistic(cmi: np.ndarray, alpha: float = 0.05) -> MaxStat:
    """cmi: FP64 [c][P+1]; column 0 holds the originals, columns 1..P the surrogate rounds."""
    cmi = np.asarray(cmi, dtype=np.float64)
    orig = cmi[:, 0]
    c_star = 0
    for c in range(1, orig.size):
        if orig[c] > orig[c_star]:
            c_star = c
    t_obs = float(orig[c_star])
    t_max = cmi[:, 1:].max(axis=0)
    count = int(sum(1 for t in t_max if t >= t_obs))
    P = t_max.size
    pval = count / P
    return MaxStat(c_star, t_obs, count, pval, bool(pval < alpha),
                   order_statistic_threshold(t_max, 0.05),
                   order_statistic_threshold(t_max, 0.01), t_max)


def _step_cmis(cand, y, zcols, pool, perms, k):
    P = perms.shape[0]
    z = np.stack(zcols, axis=1) if zcols else np.zeros((y.size, 0), np.float32)
    out = np.empty((len(pool), P + 1), dtype=np.float64)
    for ci, c in enumerate(pool):
        out[ci, 0] = ksg_cmi(cand[c], y, z, k)
        for p in range(P):
            out[ci, p + 1] = ksg_cmi(cand[c][perms[p]], y, z, k)
    return out


def greedy_select(cand, y, k: int, perms, alpha: float = 0.05, max_steps: int | None = None,
                  return_cmis: bool = False):
    """Greedy CMI-maximising selection gated by the max-statistic test.

    cand: [C][N] FP32 candidate columns, y: [N] FP32, perms: int [P][N].
    Returns (selected candidate indices in inclusion order, per-step MaxStat list[, per-step CMI tables]).
    """
    cand = np.asarray(cand, dtype=np.float32)
    y = np.asarray(y, dtype=np.float32)
    perms = np.asarray(perms)
    pool = list(range(cand.shape[0]))
    selected, steps, tables = [], [], []
    while pool and (max_steps is None or len(steps) < max_steps):
        cmis = _step_cmis(cand, y, [cand[s] for s in selected], pool, perms, k)
        ms = max_statistic(cmis, alpha)
        steps.append(ms)
        tables.append(cmis)
        if not ms.significant:
            break
        c = pool[ms.c_star]
        selected.append(c)
        pool.remove(c)
    if return_cmis:
        return selected, steps, tables
    return selected, steps


def omnibus_test(cand, y, selected, target: int, max_lag: int, k: int, perms,
                 alpha: float = 0.05):
    """I(selected sources ; Y | selected target past), permutation test on the source block.

    Returns (cmi table [1][P+1], MaxStat) or None when no source candidate was selected.
    """
    cand = np.asarray(cand, dtype=np.float32)
    src = [c for c in selected if c // max_lag != target]
    tgt = [c for c in selected if c // max_lag == target]
    if not src:
        return None
    xs = np.stack([cand[c] for c in src], axis=1)
    z = np.stack([cand[c] for c in tgt], axis=1) if tgt else np.zeros((y.size, 0), np.float32)
    P = perms.shape[0]
    out = np.empty((1, P + 1))
    out[0, 0] = ksg_cmi(xs, y, z, k)
    for p in range(P):
        out[0, p + 1] = ksg_cmi(xs[perms[p]], y, z, k)
    return out, max_statistic(out, alpha)
