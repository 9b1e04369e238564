"""Learned null for the greedy selection: training-set assembly, training and calibration.

The threshold network predicts, from a step's 16 features, the step's surrogate
max-statistic thresholds sqrt(N) * tau_0.05 and sqrt(N) * tau_0.01.  Its training examples
come from the method itself: every greedy step run with surrogates yields a CMI table whose
candidate subsets each have their own max-statistic null distribution (ksg_null_examples).
select_parents then gates every step on the network and pays for the surrogates only when
the observed statistic falls inside the calibrated margin around the predicted threshold;
the plain permutation test stays the fallback and the judge.

This module only sequences library calls (argument marshalling); the estimates, the
example statistics, the features, training, standardisation and calibration all run in the
library.  Randomness (which steps, conditioning sets and subsets) is supplied by the caller.
"""
from __future__ import annotations

import dataclasses
from typing import Iterable, List, Sequence

from ._binding import KSG_MAX_DIMS, Context, ThresholdNet


@dataclasses.dataclass
class StepSpec:
    """One greedy step to draw examples from.

    cand: device FP32 [C][N] candidate columns (ksg_embed layout); y: device FP32 [N];
    pool: candidate indices tested in the step; cond: conditioning candidate indices;
    perms: device int32 [P][N]; subsets: lists of positions into pool (each one example).
    """

    cand: object
    y: object
    pool: Sequence[int]
    cond: Sequence[int]
    perms: object
    subsets: Sequence[Sequence[int]]
    k: int = 4


def examples_from_step(ctx: Context, spec: StepSpec):
    """(feats [S][16], targets [S][2], obs [S][2]) device tensors for one step's subsets."""
    table, _ = ctx.greedy_step(spec.cand, spec.y, spec.pool, spec.cond, spec.perms, k=spec.k)
    return ctx.null_examples(table, list(spec.pool), spec.subsets, spec.cand, spec.y,
                             dz=len(spec.cond), k=spec.k)


def build_dataset(ctx: Context, specs: Iterable[StepSpec]):
    """Concatenated examples of many steps, plus the step id of every example."""
    import torch
    fs, ts, os_, ids = [], [], [], []
    for i, spec in enumerate(specs):
        f, t, o = examples_from_step(ctx, spec)
        fs.append(f)
        ts.append(t)
        os_.append(o)
        ids.append(torch.full((f.shape[0],), i, dtype=torch.int32, device=f.device))
    return torch.cat(fs), torch.cat(ts), torch.cat(os_), torch.cat(ids)


def greedy_path_examples(ctx: Context, cand, y, perms, subsets_for, k: int = 4,
                         alpha: float = 0.05, max_cond: int = KSG_MAX_DIMS - 2):
    """Examples from every step of the plain greedy selection on one target.

    The plain method is run step by step (ksg_greedy_step: all candidates x surrogates in one
    batched launch, then the max-statistic test), so the examples come from exactly the
    steps -- conditioning sets, candidate pools, observed statistics -- that select_parents
    meets.  subsets_for(n_pool, step) returns the candidate subsets (positions into the pool)
    to take from each step; the caller owns the randomness.  max_cond caps the conditioning
    set as select_parents does; a path that reaches it after a significant step is truncated.
    Returns (feats, targets, obs, n_steps, parents, truncated).
    """
    import torch
    C = cand.shape[0]
    pool = list(range(C))
    cond: List[int] = []
    fs, ts, os_ = [], [], []
    step = 0
    truncated = False
    while pool:
        if len(cond) > max_cond:
            truncated = True
            break
        table, res = ctx.greedy_step(cand, y, pool, cond, perms, k=k, alpha=alpha)
        f, t, o = ctx.null_examples(table, pool, subsets_for(len(pool), step), cand, y, dz=len(cond), k=k)
        fs.append(f)
        ts.append(t)
        os_.append(o)
        step += 1
        if not res["significant"]:
            break
        c = pool[res["c_star"]]
        cond.append(c)
        pool.remove(c)
    return torch.cat(fs), torch.cat(ts), torch.cat(os_), step, cond, truncated


def train_threshold_net(ctx: Context, feats, targets, init_params, epochs: int = 40,
                        batch: int = 512, lr: float = 2e-3) -> tuple[ThresholdNet, List[float]]:
    """Standardise on the training features, then Adam on the device; returns (net, loss history).

    The rows are used in the order given: shuffle them beforehand.
    """
    net = ThresholdNet(ctx, init_params)
    net.fit_norm(feats)
    hist = net.train(feats, targets, epochs=epochs, batch=batch, lr=lr)
    return net, [float(h) for h in hist]


def calibrate(net: ThresholdNet, feats, obs, rate: float = 0.0025, include_rate: float | None = None) -> dict:
    """Gate margins on held-out examples so that at most rate of them are decided wrongly
    (rate/2 per side); with include_rate, at most rate/2 wrong stops and include_rate wrong
    inclusions."""
    return net.calibrate(feats, obs, rate, include_rate)
