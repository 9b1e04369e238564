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

The selection has no size limit here: the paper stops only on the test.
Tests bound the number of steps with ``max_steps``.

The paper's network paragraph also names bivariate and multivariate
variants and post-selection statistics without defining them; the readings
taken here (network_select, min_statistic, prune_min_statistic, fdr_bh):

* multivariate TE: one pool of every variable's past (the default above);
* multivariate MI: the same without the target's own past;
* bivariate TE: first the target's own past alone, then each source on its
  own (sources in index order), its lags conditioned only on the selected
  target past and that source's own selected lags;
* min-statistic pruning of the selected sources: each selected source c
  gets I(c ; Y | every other selected candidate) and its surrogates (c's
  rows permuted, one permutation per round shared by all c); T_min = min_c
  (lowest index on ties), per-round minima T_p; p = #{p : T_p >= T_min}/P;
  if p >= alpha the minimising source is removed and the test repeats,
  otherwise every remaining source is kept;
* FDR across targets: Benjamini-Hochberg at level alpha on the targets'
  omnibus p-values;
* sequential max-statistic final test of the selected sources: every
  selected source c gets I(c ; Y | every other selected candidate) and its
  surrogates (as for pruning); the observed values are ranked in descending
  order (lowest index first on ties) and the r-th largest is compared with
  the distribution over rounds of the r-th largest surrogate value of that
  round: p_r = #{p : T_p,(r) >= I_(r)} / P; ranks are tested from r = 1 and
  the first rank with p_r >= alpha ends the test: that source and every
  later-ranked one are removed, the earlier ones are kept.
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
    "network_select",
    "MinStat",
    "min_statistic",
    "prune_min_statistic",
    "fdr_bh",
    "max_statistic_sequential",
    "sequential_final_test",
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


def _step_cmis(cand, y, zcols, pool, perms, k, estimator=ksg_cmi):
    P = perms.shape[0]
    z = np.stack(zcols, axis=1) if zcols else np.zeros((y.size, 0), np.float32)
    out = np.empty((len(pool), P + 1), dtype=np.float64)
    for ci, c in enumerate(pool):
        out[ci, 0] = estimator(cand[c], y, z, k)
        for p in range(P):
            out[ci, p + 1] = estimator(cand[c][perms[p]], y, z, k)
    return out


def greedy_select(cand, y, k: int, perms, alpha: float = 0.05, max_steps: int | None = None,
                  return_cmis: bool = False, pool=None, selected=None, estimator=ksg_cmi):
    """Greedy CMI-maximising selection gated by the max-statistic test.

    cand: [C][N] FP32 candidate columns, y: [N] FP32, perms: int [P][N].  pool: candidate
    indices to choose from (default: all); selected: the initial conditioning set (default:
    empty), extended in place of a copy.  estimator: the CMI function (X, Y, Z, k) -> nats
    (KSG algorithm 1 by default; oracle.ksg2.ksg2_cmi for algorithm 2).
    Returns (selected candidate indices in inclusion order, per-step MaxStat list[, per-step
    CMI tables]); the returned selection starts with the initial set.
    """
    cand = np.asarray(cand, dtype=np.float32)
    y = np.asarray(y, dtype=np.float32)
    perms = np.asarray(perms)
    pool = list(range(cand.shape[0])) if pool is None else list(pool)
    selected = [] if selected is None else list(selected)
    steps, tables = [], []
    while pool and (max_steps is None or len(steps) < max_steps):
        cmis = _step_cmis(cand, y, [cand[s] for s in selected], pool, perms, k, estimator)
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


def network_select(cand, y, target: int, max_lag: int, k: int, perms, alpha: float = 0.05,
                   mode: str = "mte"):
    """Parents of one target: mode "mte" (multivariate TE), "mmi" (multivariate MI) or "bte"
    (bivariate TE), readings in the module docstring.
    Returns (selected candidate indices in inclusion order, per-step MaxStat list)."""
    C = np.asarray(cand).shape[0]
    L = max_lag
    own = [c for c in range(C) if c // L == target]
    if mode == "mte":
        return greedy_select(cand, y, k, perms, alpha)
    if mode == "mmi":
        return greedy_select(cand, y, k, perms, alpha, pool=[c for c in range(C) if c // L != target])
    if mode != "bte":
        raise ValueError(mode)
    tgt, steps = greedy_select(cand, y, k, perms, alpha, pool=own)
    selected = list(tgt)
    for v in range(C // L):
        if v == target:
            continue
        sel_v, st_v = greedy_select(cand, y, k, perms, alpha, pool=[v * L + l for l in range(L)],
                                    selected=tgt)
        selected += sel_v[len(tgt):]
        steps += st_v
    return selected, steps


@dataclasses.dataclass
class MinStat:
    c_min: int
    t_min: float
    count: int
    pval: float
    significant: bool


def min_statistic(cmi: np.ndarray, alpha: float = 0.05) -> MinStat:
    """cmi: FP64 [c][P+1] (column 0 originals).  T_min = min_c (lowest index wins ties), per-round
    minima T_p, p = #{p : T_p >= T_min}/P, significant iff p < alpha."""
    cmi = np.asarray(cmi, dtype=np.float64)
    orig = cmi[:, 0]
    c_min = 0
    for c in range(1, orig.size):
        if orig[c] < orig[c_min]:
            c_min = c
    t_min = float(orig[c_min])
    t_p = cmi[:, 1:].min(axis=0)
    count = int(sum(1 for t in t_p if t >= t_min))
    pval = count / t_p.size
    return MinStat(c_min, t_min, count, pval, bool(pval < alpha))


def prune_min_statistic(cand, y, selected, target: int, max_lag: int, k: int, perms,
                        alpha: float = 0.05):
    """Min-statistic pruning of the selected sources.  Returns (kept selection in the original
    order, removed candidates in removal order, per-round MinStat list)."""
    cand = np.asarray(cand, dtype=np.float32)
    y = np.asarray(y, dtype=np.float32)
    perms = np.asarray(perms)
    kept = list(selected)
    removed, rounds = [], []
    while True:
        src = [c for c in kept if c // max_lag != target]
        if not src:
            break
        P = perms.shape[0]
        table = np.empty((len(src), P + 1))
        for i, c in enumerate(src):
            others = [cand[o] for o in kept if o != c]
            z = np.stack(others, axis=1) if others else np.zeros((y.size, 0), np.float32)
            table[i, 0] = ksg_cmi(cand[c], y, z, k)
            for p in range(P):
                table[i, p + 1] = ksg_cmi(cand[c][perms[p]], y, z, k)
        ms = min_statistic(table, alpha)
        rounds.append(ms)
        if ms.significant:
            break
        removed.append(src[ms.c_min])
        kept.remove(src[ms.c_min])
    return kept, removed, rounds


def fdr_bh(pvals, alpha: float = 0.05) -> np.ndarray:
    """Benjamini-Hochberg: reject the hypotheses with the r smallest p-values, r the largest rank
    with p_(r) <= r * alpha / m.  Returns a boolean array in the input order."""
    p = np.asarray(pvals, dtype=np.float64)
    m = p.size
    order = np.argsort(p, kind="stable")
    r = 0
    for i, idx in enumerate(order, start=1):
        if p[idx] <= i * alpha / m:
            r = i
    out = np.zeros(m, dtype=bool)
    out[order[:r]] = True
    return out


def max_statistic_sequential(cmi: np.ndarray, alpha: float = 0.05):
    """cmi: FP64 [c][P+1] (column 0 originals).  Returns (significant bool [c], pval [c]) in the
    row order; ranks after the first non-significant one keep p = 1 and are not significant."""
    cmi = np.asarray(cmi, dtype=np.float64)
    orig = cmi[:, 0]
    n, P = orig.size, cmi.shape[1] - 1
    rank_order = sorted(range(n), key=lambda c: (-orig[c], c))  # descending, lowest index on ties
    surr_sorted = -np.sort(-cmi[:, 1:], axis=0)                  # every round descending
    sig = np.zeros(n, dtype=bool)
    pval = np.ones(n)
    for r, c in enumerate(rank_order):
        count = int(np.sum(surr_sorted[r, :] >= orig[c]))
        pval[c] = count / P
        if pval[c] >= alpha:
            break
        sig[c] = True
    return sig, pval


def sequential_final_test(cand, y, selected, target: int, max_lag: int, k: int, perms,
                          alpha: float = 0.05):
    """Sequential max-statistic test of the selected sources.  Returns (kept selection in the
    original order, removed sources in rank order, {source: p-value} of every tested source,
    the [n_src][P+1] table)."""
    cand = np.asarray(cand, dtype=np.float32)
    y = np.asarray(y, dtype=np.float32)
    perms = np.asarray(perms)
    src = [c for c in selected if c // max_lag != target]
    if not src:
        return list(selected), [], {}, np.zeros((0, perms.shape[0] + 1))
    P = perms.shape[0]
    table = np.empty((len(src), P + 1))
    for i, c in enumerate(src):
        others = [cand[o] for o in selected if o != c]
        z = np.stack(others, axis=1) if others else np.zeros((y.size, 0), np.float32)
        table[i, 0] = ksg_cmi(cand[c], y, z, k)
        for p in range(P):
            table[i, p + 1] = ksg_cmi(cand[c][perms[p]], y, z, k)
    sig, pval = max_statistic_sequential(table, alpha)
    order = sorted(range(len(src)), key=lambda i: (-table[i, 0], i))
    removed = [src[i] for i in order if not sig[i]]
    kept = [c for c in selected if c not in removed]
    return kept, removed, {src[i]: float(pval[i]) for i in range(len(src))}, table
