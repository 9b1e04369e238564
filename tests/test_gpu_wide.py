"""Problems of 17..32 columns and greedy selections at the conditioning limit (needs an MI355X).

Single problems of more than 16 columns run the brute-force kernel compiled for 32 columns with
zero columns filling Z; grouped problems (greedy steps) with 15..30 conditioning columns run
the grouped kernels compiled for those sizes.  Radii and counts must equal the oracle's bit for
bit, estimates within 1e-12 * max(|I|, 1 nat).  A selection that reaches its conditioning limit
after a significant step reports truncated = 1 and matches the oracle step by step.
"""
import numpy as np
import pytest

import workloads
from oracle.ksg import ksg_cmi, ksg_cmi_from_counts, ksg_counts, local_terms
from oracle.stats import embed, greedy_select, max_statistic
from tests.gpu_util import dev, soa, tol

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(lib):
    c = lib.Context(0)
    yield c
    c.close()


def _full(lib, ctx, p, k, label):
    import torch
    n = p.n
    eps = torch.empty(n, dtype=torch.float32, device="cuda")
    cnt = torch.empty((3, n), dtype=torch.int32, device="cuda")
    loc = torch.empty(n, dtype=torch.float64, device="cuda")
    prob = lib.Problem(soa(p.x), soa(p.y), soa(p.z), k, eps_out=eps, counts_out=cnt, local_out=loc)
    got = float(ctx.cmi_batch([prob]).cpu()[0])
    e, a, b, c = ksg_counts(p.x, p.y, p.z, k)
    assert np.array_equal(eps.cpu().numpy(), e), label
    cn = cnt.cpu().numpy()
    assert np.array_equal(cn[0], a) and np.array_equal(cn[1], b) and np.array_equal(cn[2], c), label
    ref = ksg_cmi_from_counts(n, k, a, b, c)
    assert abs(got - ref) <= tol(ref), (label, got, ref)
    assert np.allclose(loc.cpu().numpy(), local_terms(n, k, a, b, c), rtol=0, atol=1e-13), label


@pytest.mark.parametrize("dims", [(1, 1, 15), (2, 1, 20), (1, 3, 28), (8, 9, 0), (4, 4, 24), (1, 31, 0),
                                  (1, 1, 30)])
@pytest.mark.parametrize("k", [4, 16])
def test_wide_problem_counts_match_oracle(lib, ctx, dims, k):
    # several 256-query tiles, a ragged last tile and a ragged 64-row pad
    n = 531 + 7 * sum(dims)
    p = workloads.random_problem(50 * sum(dims) + k, n, *dims, k)
    _full(lib, ctx, p, k, f"{dims} k={k}")


def test_wide_ties_and_duplicates(lib, ctx):
    """Integer-grid coordinates (heavy ties) and repeated rows (zero radii) at 20 columns."""
    g = workloads.rng(4040)
    n = 300
    pts = g.integers(0, 3, size=(n, 20)).astype(np.float32)
    pts[100:140] = pts[0]  # 41 copies of one row: radius 0 for k <= 40
    p = workloads.CmiProblemData(pts[:, :2], pts[:, 2:4], pts[:, 4:], 4)
    _full(lib, ctx, p, 4, "grid20")


def test_wide_batch_mixed_with_narrow_and_windowed(lib, ctx):
    """One batch holding wide problems (with permutation surrogates), narrow brute-force
    problems and key-window problems: the launches run side by side; every estimate matches
    the oracle."""
    import torch
    n = 2304
    pw = workloads.random_problem(71, n, 6, 1, 12, 4)   # 19 columns, Z unpermuted
    pn = workloads.random_problem(72, n, 1, 1, 3, 4)    # window search (k <= 4, N >= 2048)
    pb = workloads.random_problem(73, 700, 2, 2, 2, 8)  # brute force (k = 8)
    perms = workloads.permutations(n, 3, seed=74)
    dp = dev(perms)
    probs = [lib.Problem(soa(pw.x), soa(pw.y), soa(pw.z), 4)]
    probs += [lib.Problem(soa(pw.x), soa(pw.y), soa(pw.z), 4, perm_x=dp[q]) for q in range(3)]
    probs += [lib.Problem(soa(pn.x), soa(pn.y), soa(pn.z), 4), lib.Problem(soa(pb.x), soa(pb.y), soa(pb.z), 8)]
    got = ctx.cmi_batch(probs).cpu().numpy()
    torch.cuda.synchronize()
    refs = [ksg_cmi(pw.x, pw.y, pw.z, 4)] + [ksg_cmi(pw.x[perms[q]], pw.y, pw.z, 4) for q in range(3)]
    refs += [ksg_cmi(pn.x, pn.y, pn.z, 4), ksg_cmi(pb.x, pb.y, pb.z, 8)]
    for i, r in enumerate(refs):
        assert abs(got[i] - r) <= tol(r), (i, got[i], r)


@pytest.mark.parametrize("m,k", [(15, 4), (22, 8), (30, 4)])
def test_grouped_wide_conditioning_matches_oracle(lib, ctx, m, k):
    """Candidates x surrogates sharing Y and m = 15..30 conditioning columns: grouped (8 per
    group at these sizes, whatever the option asks) and ungrouped (the 32-column brute-force
    kernel) estimates agree to the summation-order bound and match the oracle."""
    g = workloads.rng(610 + m)
    n, n_cand, n_perm = 640, 3, 10  # 33 problems: ragged groups of 8
    p = workloads.random_problem(710 + m, n, 1, 1, m, k)
    cands = g.standard_normal((n_cand, n)).astype(np.float32)
    cands[1] = (cands[1] + 2.0 * p.y[:, 0]).astype(np.float32)
    perms = workloads.permutations(n, n_perm, seed=810 + m)
    y, z = soa(p.y), soa(p.z)
    dc, dp = dev(cands), dev(perms)
    probs = [lib.Problem(dc[c], y, z, k, perm_x=None if q == 0 else dp[q - 1])
             for c in range(n_cand) for q in range(n_perm + 1)]
    res = {}
    for gs in (0, 8, 16):
        ctx.set_option(ctx.OPT_GROUP_SIZE, gs)
        res[gs] = ctx.cmi_batch(probs).cpu().numpy()
    ctx.set_option(ctx.OPT_GROUP_SIZE, -1)
    assert np.array_equal(res[8], res[16])
    h = float(np.sum(1.0 / np.arange(1, n + 1)))
    assert np.max(np.abs(res[0] - res[8])) <= 2 * 9 * 2.0 ** -53 * 3 * h
    for idx in range(len(probs)):
        c, q = divmod(idx, n_perm + 1)
        if q not in (0, 1, n_perm):
            continue
        x = cands[c] if q == 0 else cands[c][perms[q - 1]]
        ref = ksg_cmi(x, p.y, p.z, k)
        assert abs(res[8][idx] - ref) <= tol(ref), idx


def _lag_chain(seed, n_vars=4, T=240, n_trials=2):
    """The last variable is driven by var 1 at lag 1 and var 2 at lag 2; the rest is noise."""
    g = workloads.rng(seed)
    x = g.standard_normal((n_trials, n_vars, T))
    for tr in range(n_trials):
        for t in range(2, T):
            x[tr, -1, t] = 0.8 * x[tr, 1, t - 1] + 0.7 * x[tr, 2, t - 2] + 0.3 * g.standard_normal()
    return x.astype(np.float32)


def test_greedy_step_with_thirty_conditioning_columns(lib, ctx):
    """A greedy step at the column limit (X, Y and 30 conditioning columns) against the oracle
    on every candidate and round; one more conditioning column is rejected."""
    data = workloads.logistic_network(seed=5, n_nodes=7, n_trials=1, T=405).data
    cand, y = embed(data, target=0, max_lag=5)  # 35 candidates, N = 400
    perms = workloads.permutations(y.size, 5, seed=91)
    cond = list(range(5, 35))
    pool = [0, 1, 2, 3, 4]
    tab, r = ctx.greedy_step(dev(cand), dev(y), pool, cond, dev(perms), k=4)
    tab = tab.cpu().numpy()
    z = np.stack([cand[c] for c in cond], 1)
    for ci, c in enumerate(pool):
        for q in range(perms.shape[0] + 1):
            x = cand[c] if q == 0 else cand[c][perms[q - 1]]
            ref = ksg_cmi(x, y, z, 4)
            assert abs(tab[ci, q] - ref) <= tol(ref), (c, q)
    o = max_statistic(tab, 0.05)
    assert r["c_star"] == o.c_star and r["count"] == o.count and r["significant"] == o.significant
    with pytest.raises(lib.KsgError) as e:
        ctx.greedy_step(dev(cand), dev(y), [0, 1], list(range(3, 34)), dev(perms), k=4)
    assert e.value.status == 1


@pytest.mark.parametrize("max_cond", [1, 2])
def test_select_parents_truncation_matches_oracle(lib, ctx, max_cond):
    """The conditioning set capped at max_cond columns.  On this chain the oracle's first two
    steps are significant and its third is not.  max_cond = 1: the two steps run, both parents
    are included and the selection reports the truncation.  max_cond = 2: the third step still
    fits, is not significant, and the selection ends at its statistical stop (not truncated).
    Every step matches the oracle's (which has no cap) and the uncapped selection."""
    data = _lag_chain(61)
    L, P = 2, 19
    cand, y = embed(data, target=3, max_lag=L)
    perms = workloads.permutations(y.size, P, seed=62)
    sel_all, steps_all = greedy_select(cand, y, 4, perms, alpha=0.05)
    assert [s.significant for s in steps_all] == [True, True, False]  # the case needs it
    n_run = min(max_cond + 1, len(steps_all))
    sel, steps = greedy_select(cand, y, 4, perms, alpha=0.05, max_steps=n_run)
    r = ctx.select_parents(dev(data), target=3, perms=dev(perms), k=4, max_lag=L, max_cond=max_cond)
    assert r["truncated"] == (max_cond == 1)
    assert r["candidates"] == sel and r["n_steps"] == len(steps)
    for i, s in enumerate(steps[:len(sel)]):
        assert abs(r["cmi"][i] - s.t_obs) <= tol(s.t_obs) and r["pval"][i] == s.pval
    full = ctx.select_parents(dev(data), target=3, perms=dev(perms), k=4, max_lag=L)
    assert not full["truncated"] and full["candidates"] == sel_all and full["n_steps"] == len(steps_all)
    # max_steps ends the loop without calling it a truncation
    one = ctx.select_parents(dev(data), target=3, perms=dev(perms), k=4, max_lag=L, max_steps=1)
    assert not one["truncated"] and one["n_steps"] == 1


def test_example_path_reports_truncation(lib, ctx):
    """The learned null's training paths stop at the same limit and say so."""
    from paper_1807_10459_amd.learned_null import greedy_path_examples
    data = _lag_chain(61)
    cand, y = embed(data, target=3, max_lag=2)
    perms = workloads.permutations(y.size, 19, seed=62)
    subsets = lambda n_pool, step: [list(range(n_pool))]  # noqa: E731
    f, t, o, n_steps, parents, truncated = greedy_path_examples(
        ctx, dev(cand), dev(y), dev(perms), subsets, k=4, max_cond=1)
    sel, _ = greedy_select(cand, y, 4, perms, alpha=0.05, max_steps=2)
    assert truncated and n_steps == 2 and parents == sel and f.shape[0] == 2
    *_, n_all, parents_all, trunc_all = greedy_path_examples(ctx, dev(cand), dev(y), dev(perms), subsets, k=4)
    assert not trunc_all and parents_all == greedy_select(cand, y, 4, perms, alpha=0.05)[0]


def test_algorithm2_keeps_sixteen_columns(lib, ctx):
    """KSG algorithm 2 is compiled up to 16 columns: a wider problem is rejected, the context
    stays usable, and its selections cap the conditioning set at 14 columns."""
    p = workloads.random_problem(99, 300, 1, 1, 15, 4)
    ctx.set_option(ctx.OPT_ALGORITHM, 2)
    try:
        with pytest.raises(lib.KsgError) as e:
            ctx.cmi_batch([lib.Problem(soa(p.x), soa(p.y), soa(p.z), 4)])
        assert e.value.status == 1
        q = workloads.random_problem(98, 300, 1, 1, 3, 4)
        ctx.cmi_batch([lib.Problem(soa(q.x), soa(q.y), soa(q.z), 4)])
    finally:
        ctx.set_option(ctx.OPT_ALGORITHM, 1)
