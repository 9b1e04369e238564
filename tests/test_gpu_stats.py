"""Parity of the embedding, max-statistic, greedy-step and select_parents entry points with
the CPU oracle (needs an MI355X)."""
import numpy as np
import pytest

import workloads
from oracle.ksg import ksg_cmi
from oracle.stats import embed, greedy_select, max_statistic, omnibus_test
from tests.gpu_util import dev, tol

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(lib):
    c = lib.Context(0)
    yield c
    c.close()


def test_embed_matches_oracle(lib, ctx):
    net = workloads.logistic_network(seed=3, n_nodes=6, n_trials=3, T=300)
    cand, y = ctx.embed(dev(net.data), target=2, max_lag=5)
    rc, ry = embed(net.data, target=2, max_lag=5)
    assert np.array_equal(cand.cpu().numpy(), rc)
    assert np.array_equal(y.cpu().numpy(), ry)
    # into caller-owned buffers (reused: a second target overwrites every element)
    import torch
    out = (torch.full_like(cand, float("nan")), torch.full_like(y, float("nan")))
    for tgt in (4, 2):
        c2, y2 = ctx.embed(dev(net.data), target=tgt, max_lag=5, out=out)
        assert c2.data_ptr() == out[0].data_ptr() and y2.data_ptr() == out[1].data_ptr()
        rc, ry = embed(net.data, target=tgt, max_lag=5)
        assert np.array_equal(c2.cpu().numpy(), rc) and np.array_equal(y2.cpu().numpy(), ry)
    with pytest.raises(ValueError):
        ctx.embed(dev(net.data), target=2, max_lag=4, out=out)


@pytest.mark.parametrize("c,P", [(1, 1), (1, 200), (7, 19), (25, 200), (100, 500), (3, 4096)])
def test_maxstat_matches_oracle(lib, ctx, c, P):
    g = workloads.rng(c * 1000 + P)
    t = np.round(g.standard_normal((c, P + 1)), 2)  # coarse values: ties in originals and maxima
    r = ctx.maxstat(dev(t), alpha=0.05)
    o = max_statistic(t, 0.05)
    assert r["c_star"] == o.c_star and r["count"] == o.count
    assert r["t_obs"] == o.t_obs and r["pval"] == o.pval and r["significant"] == o.significant
    assert r["tau05"] == o.tau05 and r["tau01"] == o.tau01


def test_maxstat_rejects_bad_sizes(lib, ctx):
    with pytest.raises(lib.KsgError):
        ctx.maxstat(dev(np.zeros((2, 4098))), 0.05)
    with pytest.raises(lib.KsgError):
        ctx.maxstat(dev(np.zeros((2, 5))), 1.5)


def _small_chain(seed, n_vars=4, T=260, n_trials=2):
    """y (last variable) driven by var 1 at lag 1 and var 2 at lag 2; others noise."""
    g = workloads.rng(seed)
    x = g.standard_normal((n_trials, n_vars, T))
    for tr in range(n_trials):
        for t in range(2, T):
            x[tr, -1, t] = 0.8 * x[tr, 1, t - 1] + 0.6 * x[tr, 2, t - 2] + 0.4 * g.standard_normal()
    return x.astype(np.float32)


def test_greedy_step_matches_oracle(lib, ctx):
    data = _small_chain(21)
    cand, y = embed(data, target=3, max_lag=2)
    perms = workloads.permutations(y.size, 19, seed=22)
    pool, cond = [0, 1, 2, 4, 5, 7], [3, 6]
    tab, r = ctx.greedy_step(dev(cand), dev(y), pool, cond, dev(perms), k=4)
    tab = tab.cpu().numpy()
    z = np.stack([cand[c] for c in cond], 1)
    for ci, c in enumerate(pool):
        for p in (0, 1, 19):
            x = cand[c] if p == 0 else cand[c][perms[p - 1]]
            ref = ksg_cmi(x, y, z, 4)
            assert abs(tab[ci, p] - ref) <= tol(ref), (c, p)
    o = max_statistic(tab, 0.05)
    assert r["c_star"] == o.c_star and r["count"] == o.count and r["significant"] == o.significant


def test_select_parents_matches_oracle(lib, ctx):
    data = _small_chain(31)
    L, P = 2, 19
    cand, y = embed(data, target=3, max_lag=L)
    perms = workloads.permutations(y.size, P, seed=32)
    sel, steps = greedy_select(cand, y, 4, perms, alpha=0.05)
    r = ctx.select_parents(dev(data), target=3, perms=dev(perms), k=4, max_lag=L, alpha=0.05, omnibus=True)
    assert r["candidates"] == sel
    assert r["n_steps"] == len(steps)
    for i, s in enumerate(steps[:len(sel)]):
        assert abs(r["cmi"][i] - s.t_obs) <= tol(s.t_obs)
        assert r["pval"][i] == s.pval
    assert r["n_cmi"] == sum((cand.shape[0] - i) * (P + 1) for i in range(len(steps))) + (P + 1) * r["omnibus_tested"]
    om = omnibus_test(cand, y, sel, target=3, max_lag=L, k=4, perms=perms)
    if om is None:
        assert not r["omnibus_tested"]
    else:
        assert r["omnibus_tested"] and r["omnibus_significant"] == om[1].significant
        assert abs(r["omnibus_cmi"] - om[1].t_obs) <= tol(om[1].t_obs)
        assert r["omnibus_pval"] == om[1].pval


def test_select_parents_max_steps_and_capacity(lib, ctx):
    data = _small_chain(41)
    perms = workloads.permutations(2 * 258, 9, seed=42)
    r = ctx.select_parents(dev(data), target=3, perms=dev(perms), k=4, max_lag=2, max_steps=1)
    assert r["n_steps"] == 1
    with pytest.raises(lib.KsgError) as e:
        ctx.select_parents(dev(data), target=3, perms=dev(perms), k=4, max_lag=2, capacity=0)
    assert e.value.status == 7


def test_select_parents_bad_permutation_rejected(lib, ctx):
    data = _small_chain(51)
    perms = workloads.permutations(2 * 258, 3, seed=52)
    perms[1, 7] = 10 ** 6  # outside [0, N)
    with pytest.raises(lib.KsgError) as e:
        ctx.select_parents(dev(data), target=3, perms=dev(perms), k=4, max_lag=2)
    assert e.value.status == 1
    # the context stays usable
    perms[1, 7] = 7
    ctx.select_parents(dev(data), target=3, perms=dev(perms), k=4, max_lag=2, max_steps=1)


def test_ar2_full_size_recovers_true_parents(lib, ctx):
    """Full-size AR(2) workload (N = 10,000, 25 candidates, 200 surrogates): the greedy run
    must include every true source parent and the target's own lag-1 and lag-2 past."""
    net = workloads.ar2_network(seed=1)
    perms = workloads.permutations(10000, 200, seed=11)
    r = ctx.select_parents(dev(net.data), target=0, perms=dev(perms), k=4, max_lag=5)
    got = set(r["parents"])
    want = {(src, lag) for (src, _, lag) in net.edges} | {(0, 1), (0, 2)}
    assert want <= got, (sorted(got), sorted(want))
    assert len(got) <= len(want) + 2  # few false positives at alpha = 0.05
    # the steps' p-values of included parents are below alpha
    assert all(p < 0.05 for p in r["pval"])


@pytest.mark.parametrize("mode", ["bte", "mmi", "mte"])
def test_select_parents_modes_match_oracle(lib, ctx, mode):
    """Bivariate TE, multivariate MI and multivariate TE selections equal the oracle's step by
    step (redundant driver copies: the modes give different parent sets)."""
    from oracle.stats import network_select
    data = workloads.redundant_driver_network(61)
    L, P = 2, 19
    cand, y = embed(data, target=3, max_lag=L)
    perms = workloads.permutations(y.size, P, seed=62)
    sel, steps = network_select(cand, y, 3, L, 4, perms, mode=mode)
    r = ctx.select_parents(dev(data), target=3, perms=dev(perms), k=4, max_lag=L, mode=mode)
    assert r["candidates"] == sel
    assert r["n_steps"] == len(steps)
    st = [s for s in steps if s.significant]
    for i, s in enumerate(st):
        assert abs(r["cmi"][i] - s.t_obs) <= tol(s.t_obs)
        assert r["pval"][i] == s.pval


def test_select_parents_pruning_matches_oracle(lib, ctx):
    """Min-statistic pruning after inclusion, against the oracle's (with a forced-in noise
    source, the oracle removes it: see its pins)."""
    from oracle.stats import greedy_select, prune_min_statistic
    data = workloads.redundant_driver_network(63)
    L, P = 1, 39
    cand, y = embed(data, target=3, max_lag=L)
    perms = workloads.permutations(y.size, P, seed=64)
    sel, _ = greedy_select(cand, y, 4, perms)
    kept, removed, rounds = prune_min_statistic(cand, y, sel, 3, L, 4, perms)
    r = ctx.select_parents(dev(data), target=3, perms=dev(perms), k=4, max_lag=L, prune=True, omnibus=True)
    assert r["candidates"] == kept
    assert r["pruned"] == removed
    om = omnibus_test(cand, y, kept, target=3, max_lag=L, k=4, perms=perms)
    if om is not None:
        assert r["omnibus_tested"] and r["omnibus_pval"] == om[1].pval


def test_select_parents_pruning_removal_matches_oracle(lib, ctx):
    """A case in which the min-statistic test removes a source (logistic-map network, six of
    its variables, one trial; found by searching seeds with the oracle)."""
    from oracle.stats import greedy_select, prune_min_statistic
    data = np.ascontiguousarray(workloads.logistic_network(seed=136, n_trials=1, T=260).data[:, :6])
    L, P, alpha, target = 2, 19, 0.3, 1
    cand, y = embed(data, target=target, max_lag=L)
    perms = workloads.permutations(y.size, P, seed=137)
    sel, _ = greedy_select(cand, y, 4, perms, alpha=alpha)
    kept, removed, _ = prune_min_statistic(cand, y, sel, target, L, 4, perms, alpha=alpha)
    assert removed  # the case exercises a removal
    r = ctx.select_parents(dev(data), target=target, perms=dev(perms), k=4, max_lag=L, alpha=alpha, prune=True)
    assert r["pruned"] == removed
    assert r["candidates"] == [c for c in sel if c in kept]


def test_select_parents_sequential_matches_oracle(lib, ctx):
    """Sequential max-statistic test of the selected sources against the oracle's, on a case in
    which it removes one source and keeps two (logistic-map network, six of its variables, one
    trial; found by searching seeds with the oracle)."""
    from oracle.stats import greedy_select, sequential_final_test
    data = np.ascontiguousarray(workloads.logistic_network(seed=136, n_trials=1, T=260).data[:, :6])
    L, P, alpha, target = 2, 19, 0.3, 1
    cand, y = embed(data, target=target, max_lag=L)
    perms = workloads.permutations(y.size, P, seed=137)
    sel, _ = greedy_select(cand, y, 4, perms, alpha=alpha)
    kept, removed, pv, _ = sequential_final_test(cand, y, sel, target, L, 4, perms, alpha=alpha)
    assert removed and [c for c in kept if c // L != target]  # the case removes and keeps sources
    r = ctx.select_parents(dev(data), target=target, perms=dev(perms), k=4, max_lag=L, alpha=alpha,
                           sequential=True)
    assert r["seq_removed"] == removed
    assert r["candidates"] == kept
    for c, p in zip(r["candidates"], r["seq_pval"]):
        assert p == (pv[c] if c // L != target else -1.0), c
    # with the omnibus test on, the sequential test runs only after a significant omnibus result
    r2 = ctx.select_parents(dev(data), target=target, perms=dev(perms), k=4, max_lag=L, alpha=alpha,
                            sequential=True, omnibus=True)
    if r2["omnibus_significant"]:
        assert r2["seq_removed"] == removed
    else:
        assert r2["seq_removed"] == [] and r2["candidates"] == sel


def test_select_parents_algorithm2_matches_oracle(lib, ctx):
    """select_parents under KSG algorithm 2 equals the oracle's greedy selection with the
    algorithm-2 estimator, step by step."""
    from oracle.ksg2 import ksg2_cmi
    data = _small_chain(31)
    L, P = 2, 19
    cand, y = embed(data, target=3, max_lag=L)
    perms = workloads.permutations(y.size, P, seed=32)
    sel, steps = greedy_select(cand, y, 4, perms, alpha=0.05, estimator=ksg2_cmi)
    ctx.set_option(ctx.OPT_ALGORITHM, 2)
    try:
        r = ctx.select_parents(dev(data), target=3, perms=dev(perms), k=4, max_lag=L, alpha=0.05)
    finally:
        ctx.set_option(ctx.OPT_ALGORITHM, 1)
    assert r["candidates"] == sel
    assert r["n_steps"] == len(steps)
    for i, s in enumerate(steps[:len(sel)]):
        assert abs(r["cmi"][i] - s.t_obs) <= tol(s.t_obs)
        assert r["pval"][i] == s.pval


def test_bench_configuration_sampled_parity(lib, ctx):
    """The timed workload at full size: AR(2) network, N = 10,000, 25 candidates, 200
    surrogates, greedy steps with m = 1 and m = 8 conditioning columns, one grouped batched
    launch each (as the benchmark runs them).  Sampled CMIs of every step equal the oracle's;
    the step's max-statistic result equals the oracle's test on the returned table."""
    net = workloads.ar2_network(seed=1)
    L, P = 5, 200
    perms = workloads.permutations(10000, P, seed=11)
    cand, y = embed(net.data, target=0, max_lag=L)
    dcand, dy = ctx.embed(dev(net.data), target=0, max_lag=L)
    first = [0, 1] + [src * L + (lag - 1) for (src, _, lag) in net.edges]
    order = first + [c for c in range(25) if c not in first]
    g = workloads.rng(77)
    for m in (1, 8):
        cond = order[:m]
        pool = [c for c in range(25) if c not in cond]
        table, r = ctx.greedy_step(dcand, dy, pool, cond, dev(perms), k=4)
        table = table.cpu().numpy()
        ms = max_statistic(table, 0.05)
        assert r["c_star"] == ms.c_star and r["count"] == ms.count and r["significant"] == ms.significant
        z = np.stack([cand[c] for c in cond], axis=1)
        samples = {(ms.c_star, 0), (len(pool) - 1, P)} | {(int(g.integers(len(pool))), int(g.integers(P + 1)))
                                                          for _ in range(3)}
        for ci, p in sorted(samples):
            xs = cand[pool[ci]] if p == 0 else cand[pool[ci]][perms[p - 1]]
            ref = ksg_cmi(xs, y, z, 4)
            assert abs(table[ci, p] - ref) <= tol(ref), (m, ci, p)


def test_bench_configuration_grouped_equals_brute_force(lib, ctx):
    """Every CMI of the timed workload (the AR(2) forced path, m = 1..8: 32,964 estimates at
    N = 10,000) from the grouped kernels equals the brute-force single-problem kernel's (no
    grouping, no windows), which the oracle pins elsewhere; the two differ only in the order of
    the FP64 sum."""
    net = workloads.ar2_network(seed=1)
    L, P = 5, 200
    perms = dev(workloads.permutations(10000, P, seed=11))
    dcand, dy = ctx.embed(dev(net.data), target=0, max_lag=L)
    first = [0, 1] + [src * L + (lag - 1) for (src, _, lag) in net.edges]
    order = first + [c for c in range(25) if c not in first]
    for m in range(1, 9):
        cond = order[:m]
        pool = [c for c in range(25) if c not in cond]
        grouped, rg = ctx.greedy_step(dcand, dy, pool, cond, perms, k=4)
        ctx.set_option(ctx.OPT_GROUP_SIZE, 0)
        ctx.set_option(ctx.OPT_WINDOWS, 0)
        try:
            brute, rb = ctx.greedy_step(dcand, dy, pool, cond, perms, k=4)
        finally:
            ctx.set_option(ctx.OPT_GROUP_SIZE, -1)
            ctx.set_option(ctx.OPT_WINDOWS, 1)
        g, b = grouped.cpu().numpy(), brute.cpu().numpy()
        assert np.all(np.abs(g - b) <= 1e-12 * np.maximum(np.abs(b), 1.0)), (m, float(np.max(np.abs(g - b))))
        assert rg["c_star"] == rb["c_star"] and rg["count"] == rb["count"], m


def test_select_parents_resume_from_record(lib, ctx):
    """A selection resumed from the first inclusions of an earlier run (its checkpoint) ends
    with the same parents; its new steps are the oracle's greedy steps from that set."""
    data = _small_chain(31)
    L, P = 2, 19
    cand, y = embed(data, target=3, max_lag=L)
    perms = workloads.permutations(y.size, P, seed=32)
    full = ctx.select_parents(dev(data), target=3, perms=dev(perms), k=4, max_lag=L)
    assert len(full["candidates"]) >= 2  # the case needs two inclusions
    head = full["candidates"][:1]
    r = ctx.select_parents(dev(data), target=3, perms=dev(perms), k=4, max_lag=L, resume=head)
    assert r["candidates"] == full["candidates"]
    assert r["n_steps"] == full["n_steps"] - 1
    assert np.isnan(r["cmi"][0]) and r["cmi"][1:] == full["cmi"][1:] and r["pval"][1:] == full["pval"][1:]
    pool = [c for c in range(cand.shape[0]) if c not in head]
    sel, steps = greedy_select(cand, y, 4, perms, alpha=0.05, pool=pool, selected=head)
    assert sel == r["candidates"] and len(steps) == r["n_steps"]
    with pytest.raises(lib.KsgError):
        ctx.select_parents(dev(data), target=3, perms=dev(perms), k=4, max_lag=L, resume=[999])
