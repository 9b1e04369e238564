"""Pins of the embedding, max-statistic and greedy oracle (CPU only)."""
import numpy as np
import pytest

import workloads
from oracle.ksg import ksg_cmi
from oracle.stats import (embed, greedy_select, max_statistic, omnibus_test,
                          order_statistic_threshold)


def test_embed_hand_example():
    # 2 trials, 2 vars, T = 5, max_lag 2 -> t = 2, 3, 4 in each trial
    data = np.arange(20, dtype=np.float32).reshape(2, 2, 5)
    cand, y = embed(data, target=1, max_lag=2)
    # var 0 lag 1: trial 0 -> x0(1..3) = 1,2,3 ; trial 1 -> 11,12,13
    assert cand[0].tolist() == [1, 2, 3, 11, 12, 13]
    # var 0 lag 2: 0,1,2 ; 10,11,12
    assert cand[1].tolist() == [0, 1, 2, 10, 11, 12]
    # var 1 lag 1: 6,7,8 ; 16,17,18
    assert cand[2].tolist() == [6, 7, 8, 16, 17, 18]
    assert cand[3].tolist() == [5, 6, 7, 15, 16, 17]
    assert y.tolist() == [7, 8, 9, 17, 18, 19]


def test_max_statistic_hand_example():
    # 3 candidates, 4 rounds; candidate 1 and 2 tie on the original -> lowest index (1)
    t = np.array([[0.10, 0.05, 0.30, 0.01, 0.02],
                  [0.50, 0.20, 0.10, 0.60, 0.00],
                  [0.50, 0.40, 0.00, 0.00, 0.00]])
    ms = max_statistic(t, alpha=0.5)
    assert ms.c_star == 1 and ms.t_obs == 0.5
    assert ms.t_max.tolist() == [0.40, 0.30, 0.60, 0.02]
    assert ms.count == 1 and ms.pval == 0.25 and ms.significant
    assert not max_statistic(t, alpha=0.25).significant  # p < alpha is strict


def test_single_candidate_is_plain_permutation_test():
    g = workloads.rng(4)
    for _ in range(50):
        P = int(g.integers(5, 300))
        row = g.standard_normal(P + 1)
        ms = max_statistic(row[None, :], alpha=0.05)
        assert ms.c_star == 0
        assert ms.count == int(np.sum(row[1:] >= row[0]))
        assert ms.pval == np.mean(row[1:] >= row[0])


def test_order_statistic_identity():
    g = workloads.rng(5)
    for trial in range(400):
        P = int(g.choice([20, 100, 200, 500]))
        c = int(g.integers(1, 8))
        t = np.round(g.standard_normal((c, P + 1)), 1)  # coarse values: many ties
        for alpha in (0.05, 0.01):
            ms = max_statistic(t, alpha)
            tau = order_statistic_threshold(ms.t_max, alpha)
            assert ms.significant == (ms.t_obs > tau), (trial, alpha)


def test_pvalue_uniform_under_null():
    # exchangeable originals and surrogates -> the p-value is (discretely) uniform
    from scipy import stats
    g = workloads.rng(6)
    ps = []
    for _ in range(2000):
        t = g.standard_normal((5, 101))
        ps.append(max_statistic(t).pval)
    assert stats.kstest(ps, "uniform").pvalue > 1e-3
    assert abs(np.mean(np.array(ps) < 0.05) - 0.05) < 0.02


def _chain(seed, n=400):
    """y(t) driven by x1(t-1) only; x0 and x2 independent noise (3 vars, lag 1..2)."""
    g = workloads.rng(seed)
    T = n + 2
    x = g.standard_normal((3, T))
    x[1] = g.standard_normal(T)
    yv = np.zeros(T)
    yv[1:] = 0.9 * x[1, :-1] + 0.3 * g.standard_normal(T - 1)
    data = np.stack([x[0], x[1], x[2], yv])[None].astype(np.float32)
    return data


def test_greedy_recovers_single_driver():
    data = _chain(11)
    cand, y = embed(data, target=3, max_lag=2)
    perms = workloads.permutations(y.size, 39, seed=12)
    sel, steps = greedy_select(cand, y, 4, perms, alpha=0.05)
    assert sel[0] == 1 * 2 + 0  # var 1, lag 1
    assert steps[0].significant and steps[0].count == 0
    assert not steps[-1].significant  # stops on a non-significant step
    assert len(sel) == len(steps) - 1


def test_greedy_step_table_consistency():
    data = _chain(13, n=200)
    cand, y = embed(data, target=3, max_lag=2)
    perms = workloads.permutations(y.size, 19, seed=14)
    sel, steps, tables = greedy_select(cand, y, 4, perms, return_cmis=True, max_steps=2)
    # row 0 of the first table is the plain CMI of candidate 0 given nothing
    assert tables[0][0, 0] == ksg_cmi(cand[0], y, None, 4)
    assert tables[0][0, 3] == ksg_cmi(cand[0][perms[2]], y, None, 4)
    if len(sel) >= 1 and len(tables) > 1:
        z = cand[sel[0]][:, None]
        pool = [c for c in range(cand.shape[0]) if c != sel[0]]
        assert tables[1][0, 0] == ksg_cmi(cand[pool[0]], y, z, 4)


def test_omnibus():
    data = _chain(15, n=300)
    cand, y = embed(data, target=3, max_lag=2)
    perms = workloads.permutations(y.size, 19, seed=16)
    sel = [2, 6]  # var1 lag1 (source) and target lag 1
    tab, ms = omnibus_test(cand, y, sel, target=3, max_lag=2, k=4, perms=perms)
    assert tab[0, 0] == ksg_cmi(cand[2], y, cand[6], 4)
    assert ms.significant
    assert omnibus_test(cand, y, [6], 3, 2, 4, perms) is None


def test_omnibus_permutes_the_source_block_jointly():
    """Two identical source columns stay identical under a joint row permutation, and a
    duplicated column leaves every max-norm distance unchanged: so every surrogate of the
    two-column source block equals the one-column surrogate under the same permutation.
    Permuting the columns separately would pull the copies apart and change the values."""
    g = workloads.rng(17)
    n = 160
    zt = g.standard_normal(n)
    src = g.standard_normal(n)
    yv = 0.8 * src + 0.4 * zt + 0.3 * g.standard_normal(n)
    # max_lag 1, variables: 0 = target's past (Z), 1 and 2 = two copies of the source
    cand = np.stack([zt, src, src]).astype(np.float32)
    y = yv.astype(np.float32)
    perms = workloads.permutations(n, 12, seed=18)
    tab, ms = omnibus_test(cand, y, [1, 2, 0], target=0, max_lag=1, k=4, perms=perms)
    z = cand[0][:, None]
    assert tab[0, 0] == ksg_cmi(cand[1], y, z, 4)
    for p in range(perms.shape[0]):
        assert tab[0, p + 1] == ksg_cmi(cand[1][perms[p]], y, z, 4), p
    # a column-wise permutation (different rows for the two copies) gives other values
    split = np.stack([cand[1][perms[0]], cand[2][perms[1]]], axis=1)
    assert ksg_cmi(split, y, z, 4) != tab[0, 1]
    assert ms.significant


# ---- selection modes, min-statistic pruning, FDR (readings in oracle.stats) ----

def _copy_chain(seed):
    return workloads.redundant_driver_network(seed)


def test_selection_modes_on_redundant_sources():
    """Multivariate TE keeps one of two redundant copies of the driver; bivariate TE, which
    conditions each source only on the target's past, finds both; multivariate MI never
    selects the target's own past and, like multivariate TE, keeps one copy."""
    from oracle.stats import network_select
    data = _copy_chain(7)
    L = 1
    cand, y = embed(data, target=3, max_lag=L)  # candidates: var v at lag 1 -> index v
    perms = workloads.permutations(y.size, 39, seed=8)
    mte, _ = network_select(cand, y, 3, L, 4, perms, mode="mte")
    bte, _ = network_select(cand, y, 3, L, 4, perms, mode="bte")
    mmi, _ = network_select(cand, y, 3, L, 4, perms, mode="mmi")
    assert 3 in mte and len({0, 1} & set(mte)) == 1 and 2 not in mte
    assert 3 in bte and {0, 1} <= set(bte) and 2 not in bte
    assert bte[0] == 3  # the target's past comes first
    assert 3 not in mmi and len({0, 1} & set(mmi)) == 1


def test_bivariate_first_phase_is_restricted_greedy():
    from oracle.stats import network_select
    data = _copy_chain(9)
    cand, y = embed(data, target=3, max_lag=2)
    perms = workloads.permutations(y.size, 19, seed=10)
    sel, steps = network_select(cand, y, 3, 2, 4, perms, mode="bte")
    own, own_steps = greedy_select(cand, y, 4, perms, pool=[6, 7])
    assert sel[:len(own)] == own
    assert steps[0].t_obs == own_steps[0].t_obs


def test_min_statistic_hand_example():
    from oracle.stats import min_statistic
    # originals 0.5 and 0.3: T_min = 0.3 (candidate 1); round minima 0.1 and 0.1 -> p = 0
    t = np.array([[0.5, 0.1, 0.6], [0.3, 0.2, 0.1]])
    ms = min_statistic(t, 0.05)
    assert (ms.c_min, ms.t_min, ms.count, ms.pval, ms.significant) == (1, 0.3, 0, 0.0, True)
    # ties in the originals: the lowest index; round minima 0.4 and 0.2 -> one >= 0.3
    t2 = np.array([[0.3, 0.4, 0.9], [0.3, 0.8, 0.2]])
    ms2 = min_statistic(t2, 0.6)
    assert (ms2.c_min, ms2.count, ms2.pval, ms2.significant) == (0, 1, 0.5, True)


def test_min_statistic_single_candidate_equals_max_statistic():
    """With one candidate, min and max statistics are the same permutation test."""
    from oracle.stats import min_statistic
    g = workloads.rng(11)
    for _ in range(50):
        t = g.standard_normal((1, 21))
        a, b = min_statistic(t, 0.05), max_statistic(t, 0.05)
        assert a.pval == b.pval and a.significant == b.significant


def test_pruning_removes_a_forced_noise_candidate():
    from oracle.stats import prune_min_statistic
    data = _copy_chain(12)
    L = 1
    cand, y = embed(data, target=3, max_lag=L)
    perms = workloads.permutations(y.size, 39, seed=13)
    kept, removed, rounds = prune_min_statistic(cand, y, [3, 0, 2], 3, L, 4, perms)
    assert removed == [2] and kept == [3, 0]
    assert not rounds[0].significant and rounds[-1].significant


def test_fdr_bh_matches_library():
    from scipy.stats import false_discovery_control
    from oracle.stats import fdr_bh
    g = workloads.rng(14)
    for _ in range(200):
        m = int(g.integers(1, 30))
        p = np.where(g.random(m) < 0.3, g.random(m) * 0.01, g.random(m))
        alpha = float(g.choice([0.01, 0.05, 0.2]))
        ref = false_discovery_control(p, method="bh") <= alpha
        assert np.array_equal(fdr_bh(p, alpha), ref)
    assert fdr_bh([0.01, 0.04, 0.03, 0.2], 0.05).tolist() == [True, False, False, False]


def test_sequential_max_statistic_hand_example():
    from oracle.stats import max_statistic_sequential
    # originals 0.2, 0.9, 0.5 -> ranks: row 1 (0.9), row 2 (0.5), row 0 (0.2).
    # rounds (columns) sorted descending: round 1 (0.3, 0.1, 0.4) -> 0.4, 0.3, 0.1;
    # round 2 (0.6, 0.2, 0.1) -> 0.6, 0.2, 0.1.
    # rank 1: 0.9 vs {0.4, 0.6} -> p = 0; rank 2: 0.5 vs {0.3, 0.2} -> p = 0;
    # rank 3: 0.2 vs {0.1, 0.1} -> p = 0: all significant at any alpha > 0.
    t = np.array([[0.2, 0.3, 0.6], [0.9, 0.1, 0.2], [0.5, 0.4, 0.1]])
    sig, p = max_statistic_sequential(t, 0.05)
    assert sig.tolist() == [True, True, True] and p.tolist() == [0.0, 0.0, 0.0]
    # raise row 0's surrogate in round 2 to 0.65: sorted round 2 -> 0.65, 0.2, 0.1; still
    # rank 1: 0.9 > 0.65 (p 0); rank 2: 0.5 vs {0.3, 0.2} (p 0); rank 3: 0.2 vs {0.1, 0.1} (p 0)
    t[0, 2] = 0.65
    assert max_statistic_sequential(t, 0.05)[0].all()
    # now row 2's original drops to 0.25: ranks 1 (0.9), 2 (row 2, 0.25), 3 (row 0, 0.2);
    # rank 2: 0.25 vs {0.3, 0.2} -> p = 1/2 >= alpha: rows 2 and 0 removed, p of row 0 stays 1
    t[2, 0] = 0.25
    sig, p = max_statistic_sequential(t, 0.05)
    assert sig.tolist() == [False, True, False] and p.tolist() == [1.0, 0.0, 0.5]
    # ties in the originals rank the lower index first
    t2 = np.array([[0.5, 0.6, 0.0], [0.5, 0.0, 0.0]])
    sig2, p2 = max_statistic_sequential(t2, 0.6)
    # rank 1: row 0, 0.5 vs round maxima {0.6, 0.0} -> p = 1/2 < 0.6;
    # rank 2: row 1, 0.5 vs second largest {0.0, 0.0} -> p = 0
    assert sig2.tolist() == [True, True] and p2.tolist() == [0.5, 0.0]


def test_sequential_rank_one_is_the_max_statistic_and_counting_form():
    """Rank 1 compares the largest original with the round maxima: the max-statistic test.
    Every rank also has a counting form: the r-th largest value of a round is >= x exactly
    when at least r values of that round are >= x."""
    from oracle.stats import max_statistic_sequential
    g = workloads.rng(15)
    for _ in range(300):
        c = int(g.integers(1, 7))
        P = int(g.integers(1, 30))
        t = np.round(g.standard_normal((c, P + 1)), 1)  # coarse values: many ties
        alpha = float(g.choice([0.05, 0.2, 0.5]))
        sig, p = max_statistic_sequential(t, alpha)
        ms = max_statistic(t, alpha)
        top = max(range(c), key=lambda i: (t[i, 0], -i))
        assert top == ms.c_star and p[top] == ms.pval and sig[top] == ms.significant
        ranked = sorted(range(c), key=lambda i: (-t[i, 0], i))
        stopped = False
        for r, i in enumerate(ranked, start=1):
            if stopped:
                assert not sig[i] and p[i] == 1.0
                continue
            count = sum(1 for q in range(1, P + 1) if np.sum(t[:, q] >= t[i, 0]) >= r)
            assert p[i] == count / P
            assert sig[i] == (count / P < alpha)
            stopped = not sig[i]


def test_sequential_final_test_removes_a_noise_source():
    from oracle.stats import sequential_final_test
    data = _copy_chain(12)
    L = 1
    cand, y = embed(data, target=3, max_lag=L)
    perms = workloads.permutations(y.size, 39, seed=13)
    kept, removed, pv, table = sequential_final_test(cand, y, [3, 0, 2], 3, L, 4, perms)
    assert removed == [2] and kept == [3, 0]
    assert pv[0] < 0.05 and pv[2] >= 0.05 and table.shape == (2, 40)


def _var_exact_cmi(params, n_vars, L):
    """Exact Gaussian I(x_c ; y | x_Z) on the AR(2) network's stationary process.

    The generator is a VAR(3) in the n_vars-dim state (each node's own AR(2) terms plus the
    target's three lagged drivers), unit-variance noise.  Its companion form over the lags
    0..L gives s(t) = F s(t-1) + w(t), and the stationary covariance solves the discrete
    Lyapunov equation S = F S F^T + Q.  Candidate (v, l) is x_v(t-l), index l*n + v of s(t);
    Y is x_target(t), index target."""
    from scipy.linalg import solve_discrete_lyapunov
    n = n_vars
    A = [np.zeros((n, n)) for _ in range(3)]
    A[0][np.arange(n), np.arange(n)] = params["a1"]
    A[1][np.arange(n), np.arange(n)] = -params["a2"]
    for s in range(3):
        A[s][0, params["drivers"][s]] += params["c"][s]
    p = L + 1  # lags 0..L in the state
    F = np.zeros((n * p, n * p))
    for s in range(3):
        F[:n, s * n:(s + 1) * n] = A[s]
    F[n:, :-n] = np.eye(n * (p - 1))
    Q = np.zeros((n * p, n * p))
    Q[:n, :n] = np.eye(n)
    S = solve_discrete_lyapunov(F, Q)

    def idx(c):  # candidate index v*L + (l-1) -> state index
        v, l = divmod(c, L)
        return (l + 1) * n + v

    def logdet(ix):
        return np.linalg.slogdet(S[np.ix_(ix, ix)])[1] if ix else 0.0

    def cmi(c, Z, target=0):
        z = [idx(q) for q in Z]
        x, y = idx(c), target
        return 0.5 * (logdet([x] + z) + logdet([y] + z) - logdet(z) - logdet([x, y] + z))
    return cmi


def test_greedy_order_matches_exact_gaussian_cmi():
    """Along the greedy path on the linear AR(2) network (N = 2,000, k = 4), every candidate's
    KSG estimate lies within 0.05 nats of its exact Gaussian CMI given the path's conditioning
    set (the estimator's bias and noise at this N stay below 0.045 here), and the greedy argmax
    is the exact one wherever the exact gap between the best and second-best candidate exceeds
    0.03 nats.  Dropping or misindexing a conditioning column, or a wrong sign, moves estimates
    by more than that (e.g. I(x_0(t-1); y | x_2(t-1), x_0(t-2)) = 0.104 nats against 0.048
    without the conditioning)."""
    L, N = 5, 2000
    net = workloads.ar2_network(seed=1, T=N + L, burn=1000)
    cand, y = embed(net.data, target=0, max_lag=L)
    exact = _var_exact_cmi(net.params, net.data.shape[1], L)
    # the closed form itself: a candidate that is a lagged copy of Y given that lag is 0
    assert abs(exact(0, [0])) < 1e-10
    Z, checked = [], 0
    for _ in range(5):
        pool = [c for c in range(cand.shape[0]) if c not in Z]
        est = [ksg_cmi(cand[c], y, cand[Z].T if Z else None, 4) for c in pool]
        ex = np.array([exact(c, Z) for c in pool])
        best = pool[int(np.argmax(est))]
        order = np.argsort(ex)[::-1]
        if ex[order[0]] - ex[order[1]] > 0.03:
            assert best == pool[order[0]], (Z, best, pool[order[0]])
            checked += 1
        assert np.max(np.abs(np.array(est) - ex)) < 0.05
        Z.append(best)
    assert checked >= 2
