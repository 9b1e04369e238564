"""Parity of the HIP KSG algorithm-2 path with the CPU oracle (needs an MI355X).

Neighbour rectangles, counts and the joint k-th distance must match bit for bit; CMI values
within 1e-12 * max(|I|, 1 nat)."""
import json
import os

import numpy as np
import pytest

import workloads
from oracle.ksg import ksg_cmi
from oracle.ksg2 import ksg2_cmi, ksg2_cmi_from_counts, ksg2_counts, ksg2_local_terms
from tests.gpu_util import dev, soa, tol

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def ctx(lib):
    c = lib.Context(0)
    c.set_option(c.OPT_ALGORITHM, 2)
    yield c
    c.close()


def _run(lib, ctx, x, y, z, k, perm=None):
    import torch
    n = np.asarray(x).shape[0]
    eps = torch.empty(n, dtype=torch.float32, device="cuda")
    cnt = torch.empty((3, n), dtype=torch.int32, device="cuda")
    loc = torch.empty(n, dtype=torch.float64, device="cuda")
    p = lib.Problem(soa(x), soa(y), soa(z), k, perm_x=None if perm is None else dev(perm),
                    eps_out=eps, counts_out=cnt, local_out=loc)
    out = ctx.cmi_batch([p])
    torch.cuda.synchronize()
    return eps.cpu().numpy(), cnt.cpu().numpy(), loc.cpu().numpy(), float(out.cpu()[0])


def _check_full(lib, ctx, x, y, z, k, label=""):
    eps, cnt, loc, cmi = _run(lib, ctx, x, y, z, k)
    e, _, a, b, c = ksg2_counts(x, y, z, k)
    assert np.array_equal(eps, e), label
    assert np.array_equal(cnt[0], a) and np.array_equal(cnt[1], b) and np.array_equal(cnt[2], c), label
    n = np.asarray(x).shape[0]
    has_z = z is not None and np.asarray(z).size > 0
    ref = ksg2_cmi_from_counts(n, k, a, b, c, has_z)
    assert abs(cmi - ref) <= tol(ref), (label, cmi, ref)
    assert np.allclose(loc, ksg2_local_terms(n, k, a, b, c, has_z), rtol=0, atol=1e-13), label
    return cmi


def test_worked_example(lib, ctx):
    g = json.load(open(os.path.join(GOLD, "ksg2_tiny_ties.json")))
    x, y, z = (np.array(g[c], np.float32) for c in "xyz")
    assert abs(_check_full(lib, ctx, x, y, z, g["k"]) - 13 / 36) < 1e-15
    assert abs(_check_full(lib, ctx, x, y, None, g["k"]) - 19 / 45) < 1e-15


@pytest.mark.parametrize("dims", [(1, 1, 0), (1, 1, 1), (1, 1, 5), (1, 2, 3), (2, 1, 2), (2, 2, 4),
                                  (1, 1, 12), (3, 1, 2), (1, 4, 0), (2, 3, 5), (5, 5, 6), (1, 1, 14)])
@pytest.mark.parametrize("k", [1, 4, 7, 12])
def test_shapes_ragged(lib, ctx, dims, k):
    n = 700 + 13 * sum(dims)
    p = workloads.random_problem(sum(dims) * 11 + k, n, *dims, k)
    _check_full(lib, ctx, p.x, p.y, p.z, k, str(dims))


@pytest.mark.parametrize("k", [1, 2, 4, 8])
def test_ties_and_duplicates(lib, ctx, k):
    """Integer grids: many equal distances, so the index tie-break decides the neighbours."""
    for dims in [(1, 1, 1), (2, 1, 0), (1, 2, 2)]:
        p = workloads.random_problem(40 + k, 900, *dims, k, kind="grid")
        _check_full(lib, ctx, p.x, p.y, p.z, k, str(dims))


@pytest.mark.parametrize("n", [2, 3, 5, 64, 65, 255, 256, 257])
def test_smallest_sizes(lib, ctx, n):
    k = 1 if n < 5 else 4
    p = workloads.random_problem(60 + n, n, 1, 1, 1, k)
    _check_full(lib, ctx, p.x, p.y, p.z, k, str(n))


def test_mixed_width_batch_with_surrogates(lib, ctx):
    """One batch: problems of several column counts (one launch each) and X permutations."""
    import torch
    specs = [(1, 1, 2, 4), (1, 1, 0, 3), (2, 2, 3, 8), (1, 1, 2, 4), (1, 3, 6, 5)]
    data, probs = [], []
    perms = workloads.permutations(1500, 3, seed=71)
    for i, (dx, dy, dz, k) in enumerate(specs):
        pr = workloads.random_problem(70 + i, 1500, dx, dy, dz, k)
        data.append(pr)
        probs.append(lib.Problem(soa(pr.x), soa(pr.y), soa(pr.z), k))
        probs.append(lib.Problem(soa(pr.x), soa(pr.y), soa(pr.z), k, perm_x=dev(perms[i % 3])))
    out = ctx.cmi_batch(probs).cpu().numpy()
    for i, pr in enumerate(data):
        ref = ksg2_cmi(pr.x, pr.y, pr.z, pr.k)
        assert abs(out[2 * i] - ref) <= tol(ref), i
        ref_s = ksg2_cmi(pr.x[perms[i % 3]], pr.y, pr.z, pr.k)
        assert abs(out[2 * i + 1] - ref_s) <= tol(ref_s), i


def test_full_size_n10000(lib, ctx):
    """N = 10,000, D = 3 (one conditioning column) in full against the oracle."""
    p = workloads.random_problem(81, 10000, 1, 1, 1, 4)
    _check_full(lib, ctx, p.x, p.y, p.z, 4, "n10000")


def test_greedy_step_table_and_switch_back(lib, ctx):
    """A greedy step under algorithm 2 against the oracle; switching back gives algorithm 1."""
    from oracle.stats import embed
    net = workloads.ar2_network(seed=5, T=1505, burn=200)
    cand, y = embed(net.data, target=0, max_lag=5)
    perms = workloads.permutations(y.size, 9, seed=82)
    dcand, dy = ctx.embed(dev(net.data), target=0, max_lag=5)
    pool, cond = [1, 7, 12, 20], [0, 5]
    table, r = ctx.greedy_step(dcand, dy, pool, cond, dev(perms), k=4)
    table = table.cpu().numpy()
    z = np.stack([cand[c] for c in cond], axis=1)
    for ci, c in enumerate(pool):
        for p in (0, 3, 9):
            xs = cand[c] if p == 0 else cand[c][perms[p - 1]]
            ref = ksg2_cmi(xs, y, z, 4)
            assert abs(table[ci, p] - ref) <= tol(ref), (c, p)
    ctx.set_option(ctx.OPT_ALGORITHM, 1)
    try:
        t1, _ = ctx.greedy_step(dcand, dy, pool, cond, dev(perms), k=4)
        ref1 = ksg_cmi(cand[pool[0]], y, z, 4)
        assert abs(float(t1[0, 0]) - ref1) <= tol(ref1)
    finally:
        ctx.set_option(ctx.OPT_ALGORITHM, 2)


def test_bad_algorithm_rejected(lib, ctx):
    with pytest.raises(lib.KsgError):
        ctx.set_option(ctx.OPT_ALGORITHM, 3)


def test_autotune_keeps_algorithm(lib, ctx):
    """The autotuner times algorithm-1 groups and leaves the context on algorithm 2."""
    ctx.autotune(1024)
    p = workloads.random_problem(91, 800, 1, 1, 2, 4)
    _check_full(lib, ctx, p.x, p.y, p.z, 4, "after autotune")


def _alg2_window_case(case):
    """Problems that take the key-ordered window search under algorithm 2 (k <= 4, N >= 2048,
    a Z column, no per-point outputs)."""
    g = workloads.rng(1700 + case)
    if case == 0:  # compile-time (1, 1) split, continuous data
        p = workloads.random_problem(1710, 2500, 1, 1, 2, 4)
    elif case == 1:  # integer grid 0..20: many ties at the k-th distance
        pts = g.integers(0, 21, size=(2300, 3)).astype(np.float32)
        p = workloads.CmiProblemData(pts[:, :1].copy(), pts[:, 1:2].copy(), pts[:, 2:].copy(), 4)
    elif case == 2:  # run-time split (1, 2, 3) after the X/Y exchange, k = 3
        p = workloads.random_problem(1712, 2600, 2, 1, 3, 3)
    elif case == 3:  # values in {0, 1}: every point has duplicates, the k-th distance is 0
        pts = g.integers(0, 2, size=(2200, 4)).astype(np.float32)
        p = workloads.CmiProblemData(pts[:, :1].copy(), pts[:, 1:2].copy(), pts[:, 2:].copy(), 4)
    elif case == 4:  # constant key column: every row in every window
        p = workloads.random_problem(1714, 2048, 1, 1, 2, 2)
        p.z[:, 0] = 0.5
    else:  # (2, 2, 4) in [1, 2), k = 1
        p = workloads.random_problem(1715, 2100, 2, 2, 4, 1, kind="unit12")
    return p


@pytest.mark.parametrize("case", range(6))
def test_window_search_matches_oracle(lib, ctx, case):
    """Algorithm 2 on the key-ordered window search: the estimates equal the algorithm-2
    oracle's, and the brute-force kernel's up to the FP64 summation order; the window path
    runs (its operation count stays below the brute force's except for a constant key)."""
    p = _alg2_window_case(case)
    n = p.n
    perms = workloads.permutations(n, 2, seed=1720 + case)
    xd, yd, zd = soa(p.x), soa(p.y), soa(p.z)
    dp = dev(perms)
    probs = [lib.Problem(xd, yd, zd, p.k)] + [lib.Problem(xd, yd, zd, p.k, perm_x=dp[q]) for q in range(2)]
    got, ops = {}, {}
    ctx.set_option(ctx.OPT_TIMING, 1)
    try:
        for w in (1, 0):  # 2: windows from N = 2048 whatever an earlier autotune found
            ctx.set_option(ctx.OPT_WINDOWS, 2 * w)
            ctx.take_timing()
            got[w] = ctx.cmi_batch(probs).cpu().numpy()
            ops[w] = ctx.take_timing()[2]
    finally:
        ctx.set_option(ctx.OPT_WINDOWS, 1)
        ctx.set_option(ctx.OPT_TIMING, 0)
    h = float(np.sum(1.0 / np.arange(1, n + 1)))
    bound = 2 * 9 * 2.0 ** -53 * 4 * (h + 2.0)  # per-point terms bounded by 3 H_n + 2
    assert np.max(np.abs(got[1] - got[0])) <= bound, (case, got[1] - got[0])
    if case != 4:
        assert 0 < ops[1] < ops[0], (case, ops)
    for q in range(3):
        xs = p.x if q == 0 else p.x[perms[q - 1]]
        ref = ksg2_cmi(xs, p.y, p.z, p.k)
        assert abs(got[1][q] - ref) <= tol(ref), (case, q, got[1][q], ref)


def test_mixed_window_and_brute_force_batch(lib, ctx):
    """One algorithm-2 batch whose problems split between the window search (k <= 4, N >= 2048,
    a Z column), the brute-force kernel (k = 8; N < 2048; no Z) and several column counts, so
    that its launches run side by side on the auxiliary streams: every estimate equals the
    oracle's."""
    specs = [(2500, (1, 1, 2), 4), (2300, (1, 1, 2), 8), (1500, (1, 2, 1), 4), (2400, (2, 1, 3), 3),
             (2200, (1, 1, 0), 4), (2600, (1, 1, 1), 2)]
    probs, data = [], []
    for i, (n, dims, k) in enumerate(specs):
        p = workloads.random_problem(1800 + i, n, *dims, k)
        data.append(p)
        probs.append(lib.Problem(soa(p.x), soa(p.y), soa(p.z), k))
    out = ctx.cmi_batch(probs).cpu().numpy()
    for i, p in enumerate(data):
        ref = ksg2_cmi(p.x, p.y, p.z, p.k)
        assert abs(out[i] - ref) <= tol(ref), (i, out[i], ref)
