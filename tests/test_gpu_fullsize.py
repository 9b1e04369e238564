"""Full-size workloads in the launch configurations the benchmarks time, checked against the
oracle on sampled estimates (needs an MI355X; the oracle runs on every host core, one estimate
per process, about a minute each at N = 29,950).

* the omnibus test of the 20-node logistic network's target 0 (501 problems of 16 columns at
  N = 29,950, key-ordered window search);
* a greedy step of the same network with 14 conditioning columns (86 candidates x 501 rounds,
  grouped, split over about ten launch chunks) and ones with 22 and 30 (the grouped kernels
  compiled for 15..30 columns; 30 is the widest a greedy step can condition on);
* the 64-problem uneven batch, its three largest window-searched problems in full.
"""
import multiprocessing as mp
import os

import numpy as np
import pytest

import workloads
from oracle.ksg import ksg_cmi
from oracle.stats import embed
from tests.gpu_util import dev, soa, tol

pytestmark = pytest.mark.gpu

MAX_LAG, K = 5, 4


def _seeded_columns(count, seed, exclude=()):
    """A seeded choice of candidate columns of the 100 (conditioning sets, source blocks)."""
    pool = [c for c in range(20 * MAX_LAG) if c not in exclude]
    return [int(c) for c in workloads.rng(seed).choice(pool, count, replace=False)]


def _oracle_task(args):
    x, y, z, k = args
    return ksg_cmi(x, y, z, k)


def _oracle_many(tasks):
    """Oracle estimates of several problems, one per process (fork: the children only use NumPy)."""
    workers = min(len(tasks), os.cpu_count() or 1)
    with mp.get_context("fork").Pool(workers) as pool:
        return pool.map(_oracle_task, tasks)


@pytest.fixture(scope="module")
def ctx(lib):
    c = lib.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def logistic():
    net = workloads.logistic_network(seed=3)
    cand, y = embed(net.data, target=0, max_lag=MAX_LAG)
    perms = workloads.permutations(y.size, 500, seed=33)
    return cand, y, perms


def test_omnibus_shape_window_search(lib, ctx, logistic):
    cand, y, perms = logistic
    # the omnibus shape: 10 source columns, the target, its 5 past values (16 columns)
    tgt = list(range(MAX_LAG))
    src = _seeded_columns(10, 41, exclude=tgt)
    xs, zs = cand[src].T.copy(), cand[tgt].T.copy()
    dx, dy1, dz, dp = soa(xs), soa(y), soa(zs), dev(perms)
    probs = [lib.Problem(dx, dy1, dz, K)] + [lib.Problem(dx, dy1, dz, K, perm_x=dp[p]) for p in range(500)]
    got = ctx.cmi_batch(probs).cpu().numpy()
    rounds = [0, 1, 250, 500]
    refs = _oracle_many([(xs if p == 0 else xs[perms[p - 1]], y, zs, K) for p in rounds])
    for p, ref in zip(rounds, refs):
        assert abs(got[p] - ref) <= tol(ref), (p, got[p], ref)


@pytest.mark.parametrize("m,n_perm", [(14, 500), (22, 100), (30, 50)])
def test_logistic_greedy_step_grouped(lib, ctx, logistic, m, n_perm):
    cand, y, perms = logistic
    cond = _seeded_columns(m, 40 + m)
    pool = [c for c in range(cand.shape[0]) if c not in cond]
    tab, _ = ctx.greedy_step(dev(cand), dev(y), pool, cond, dev(perms[:n_perm]), k=K)
    tab = tab.cpu().numpy()
    z = cand[cond].T.copy()
    # candidates spread over the pool (the groups run in several launch chunks), several rounds
    picks = [(0, 0), (len(pool) // 3, 1), (len(pool) // 2, n_perm // 2), (2 * len(pool) // 3, n_perm),
             (len(pool) - 1, 3)]
    refs = _oracle_many([(cand[pool[ci]] if p == 0 else cand[pool[ci]][perms[p - 1]], y, z, K) for ci, p in picks])
    for (ci, p), ref in zip(picks, refs):
        assert abs(tab[ci, p] - ref) <= tol(ref), (m, ci, p, tab[ci, p], ref)


def test_uneven_batch_largest_window_problems(lib, ctx):
    probs, _ = workloads.uneven_batch(seed=2)
    cols = [(soa(p.x), soa(p.y), soa(p.z)) for p in probs]
    got = ctx.cmi_batch([lib.Problem(x, yy, z, p.k) for (x, yy, z), p in zip(cols, probs)]).cpu().numpy()
    win = [i for i, p in enumerate(probs) if p.k <= 4 and p.n >= 2048 and p.dims[2] >= 1]
    largest = sorted(win, key=lambda i: -probs[i].n)[:3]
    refs = _oracle_many([(probs[i].x, probs[i].y, probs[i].z, probs[i].k) for i in largest])
    for i, ref in zip(largest, refs):
        assert abs(got[i] - ref) <= tol(ref), (i, probs[i].n, probs[i].dims, got[i], ref)
