"""Parity of the HIP estimator with the CPU oracle (needs an MI355X).

Counts and radii must match bit for bit; CMI values within 1e-12 * max(|I|, 1 nat).
"""
import json
import os

import numpy as np
import pytest

import workloads
from oracle.ksg import ksg_cmi, ksg_cmi_from_counts, ksg_counts, ksg_point_counts, local_terms
from tests.gpu_util import dev, soa, tol

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def ctx(lib):
    c = lib.Context(0)
    yield c
    c.close()


def _run(lib, ctx, x, y, z, k, perm=None):
    """GPU eps, counts, local terms and CMI of one problem via the batch entry point."""
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
    e, a, b, c = ksg_counts(x, y, z, k)
    assert np.array_equal(eps, e), label
    assert np.array_equal(cnt[0], a), label
    assert np.array_equal(cnt[1], b), label
    assert np.array_equal(cnt[2], c), label
    n = np.asarray(x).shape[0]
    ref = ksg_cmi_from_counts(n, k, a, b, c)
    assert abs(cmi - ref) <= tol(ref), (label, cmi, ref)
    lt = local_terms(n, k, a, b, c)
    assert np.allclose(loc, lt, rtol=0, atol=1e-13), label
    return cmi


def test_worked_example(lib, ctx):
    g = json.load(open(os.path.join(GOLD, "ksg_tiny_ties.json")))
    x, y, z = (np.array(g[c], np.float32) for c in "xyz")
    cmi = _check_full(lib, ctx, x, y, z, g["k"])
    assert abs(cmi - 137 / 180) < 1e-15
    assert abs(_check_full(lib, ctx, x, y, None, g["k"]) - 161 / 180) < 1e-15


def test_fp32_discriminator(lib, ctx):
    g = json.load(open(os.path.join(GOLD, "fp32_discriminator.json")))
    x, y = np.array(g["x"], np.float32), np.array(g["y"], np.float32)
    eps, cnt, _, _ = _run(lib, ctx, x, y, None, 1)
    assert eps[0] == g["eps0"] and cnt[0][0] == g["n_x0"]


def test_single_entry_point_c0(lib, ctx):
    p, _, _ = workloads.gaussian_trivariate(seed=0, n_perm=0)
    ref = ksg_cmi(p.x, p.y, p.z, 4)
    got = ctx.cmi(soa(p.x), soa(p.y), soa(p.z), 4)
    assert abs(got - ref) <= tol(ref)
    _check_full(lib, ctx, p.x, p.y, p.z, 4, "c0")


@pytest.mark.parametrize("dims", [(1, 1, 0), (1, 1, 1), (1, 1, 5), (1, 2, 3), (2, 1, 2), (2, 2, 4),
                                  (1, 1, 12), (3, 1, 2), (1, 4, 0), (2, 3, 5), (5, 5, 6), (1, 1, 14)])
@pytest.mark.parametrize("k", [4, 8])
def test_shapes_ragged(lib, ctx, dims, k):
    # N spans several 256-query tiles and ends in a ragged tile and a ragged 64-row pad
    n = 777 + 13 * sum(dims)
    p = workloads.random_problem(sum(dims) * 7 + k, n, *dims, k)
    _check_full(lib, ctx, p.x, p.y, p.z, k, str(dims))


@pytest.mark.parametrize("kind", ["grid", "unit12"])
@pytest.mark.parametrize("k", [1, 2, 3, 5, 16])
def test_ties_and_small_k(lib, ctx, kind, k):
    p = workloads.random_problem(40 + k, 300, 1, 2, 2, k, kind=kind)
    _check_full(lib, ctx, p.x, p.y, p.z, k, kind)


def test_duplicates_and_zero_radius(lib, ctx):
    g = workloads.rng(77)
    x = g.integers(0, 3, size=(500, 1)).astype(np.float32)
    y = g.integers(0, 3, size=(500, 1)).astype(np.float32)
    z = g.integers(0, 2, size=(500, 1)).astype(np.float32)
    for k in (1, 4, 8):
        _check_full(lib, ctx, x, y, z, k, f"dup k={k}")
        _check_full(lib, ctx, x, y, None, k, f"dup z-empty k={k}")


@pytest.mark.parametrize("n", [2, 5, 63, 64, 65, 255, 256, 257])
def test_smallest_sizes(lib, ctx, n):
    k = 1
    p = workloads.random_problem(n, n, 1, 1, 1, k)
    _check_full(lib, ctx, p.x, p.y, p.z, k, f"n={n}")


def test_denormals_and_large_magnitudes(lib, ctx):
    g = workloads.rng(5)
    x = (g.standard_normal((400, 1)) * 1e-39).astype(np.float32)  # subnormal FP32 values
    y = (g.standard_normal((400, 1)) * 1e30).astype(np.float32)
    z = (g.standard_normal((400, 1))).astype(np.float32)
    assert np.any((np.abs(x) < np.finfo(np.float32).tiny) & (x != 0))
    _check_full(lib, ctx, x, y, z, 4, "denormal")


@pytest.mark.parametrize("dims_list", [
    [(3, 1, 2), (1, 3, 2), (1, 4, 1), (2, 3, 1), (1, 5, 0), (4, 2, 0)],  # D = 6
    [(4, 1, 4), (1, 6, 2), (3, 3, 3), (1, 8, 0), (2, 2, 5)],              # D = 9; (2, 2, 5) fast
])
def test_generic_same_width_batch(lib, ctx, dims_list):
    """Generic shapes of one column count share one launch (per-width kernel, compile-time
    count loops for a one-column X and selects otherwise); counts exact on every point."""
    import torch
    probs, outs, data = [], [], []
    for i, dims in enumerate(dims_list):
        n = 600 + 97 * i
        pr = workloads.random_problem(1000 + i, n, *dims, 3)
        eps = torch.empty(n, dtype=torch.float32, device="cuda")
        cnt = torch.empty((3, n), dtype=torch.int32, device="cuda")
        probs.append(lib.Problem(soa(pr.x), soa(pr.y), soa(pr.z), 3, eps_out=eps, counts_out=cnt))
        outs.append((eps, cnt))
        data.append(pr)
    res = ctx.cmi_batch(probs).cpu().numpy()
    for i, pr in enumerate(data):
        e, a, b, c = ksg_counts(pr.x, pr.y, pr.z, 3)
        cnt = outs[i][1].cpu().numpy()
        assert np.array_equal(outs[i][0].cpu().numpy(), e), dims_list[i]
        assert np.array_equal(cnt[0], a) and np.array_equal(cnt[1], b) and np.array_equal(cnt[2], c), dims_list[i]
        ref = ksg_cmi_from_counts(pr.n, 3, a, b, c)
        assert abs(res[i] - ref) <= tol(ref), dims_list[i]


def test_surrogate_gather(lib, ctx):
    p, perms, _ = workloads.gaussian_trivariate(seed=0, n_perm=3)
    for q in range(3):
        eps, cnt, _, cmi = _run(lib, ctx, p.x, p.y, p.z, 4, perm=perms[q])
        e, a, b, c = ksg_counts(p.x[perms[q]], p.y, p.z, 4)
        assert np.array_equal(eps, e) and np.array_equal(cnt[0], a) and np.array_equal(cnt[2], c)
        ref = ksg_cmi_from_counts(p.n, 4, a, b, c)
        assert abs(cmi - ref) <= tol(ref)


def test_c0_with_200_surrogates_batch(lib, ctx):
    import torch
    p, perms, _ = workloads.gaussian_trivariate(seed=0, n_perm=200)
    x, y, z = soa(p.x), soa(p.y), soa(p.z)
    dperm = dev(perms)
    probs = [lib.Problem(x, y, z, 4)] + [lib.Problem(x, y, z, 4, perm_x=dperm[q]) for q in range(200)]
    out = ctx.cmi_batch(probs).cpu().numpy()
    for q in [0, 1, 2, 57, 133, 199]:
        xs = p.x if q == 0 else p.x[perms[q - 1]]
        ref = ksg_cmi(xs, p.y, p.z, 4)
        assert abs(out[q] - ref) <= tol(ref), q
    # batch result (a grouped, key-ordered search) == single-call result up to the order of
    # the FP64 sum over the points
    assert abs(out[0] - ctx.cmi(x, y, z, 4)) <= _sum_order_bound(1000)


def test_uneven_batch_sampled(lib, ctx):
    """The 64-problem uneven batch: every problem checked on sampled points and by the count
    inequalities; the smaller problems also in full."""
    import torch
    probs, _ = workloads.uneven_batch(seed=2)
    tens = []
    outs = []
    for pr in probs:
        eps = torch.empty(pr.n, dtype=torch.float32, device="cuda")
        cnt = torch.empty((3, pr.n), dtype=torch.int32, device="cuda")
        tens.append(lib.Problem(soa(pr.x), soa(pr.y), soa(pr.z), pr.k, eps_out=eps, counts_out=cnt))
        outs.append((eps, cnt))
    res = ctx.cmi_batch(tens).cpu().numpy()
    g = workloads.rng(99)
    n_full = 0
    for i, pr in enumerate(probs):
        eps = outs[i][0].cpu().numpy()
        cnt = outs[i][1].cpu().numpy().astype(np.int64)
        assert np.all(cnt[0] <= cnt[2]) and np.all(cnt[1] <= cnt[2]), i
        for q in list(g.choice(pr.n, 6, replace=False)) + [0, pr.n - 1]:
            e, a, b, c = ksg_point_counts(pr.x, pr.y, pr.z, pr.k, int(q))
            assert eps[q] == e and cnt[0][q] == a and cnt[1][q] == b and cnt[2][q] == c, (i, q)
        # the FP64 sum over the device's own counts: exact oracle arithmetic on those counts
        ref_from_counts = ksg_cmi_from_counts(pr.n, pr.k, cnt[0], cnt[1], cnt[2])
        assert abs(res[i] - ref_from_counts) <= tol(ref_from_counts), i
        if pr.n <= 4000 and n_full < 6:
            ref = ksg_cmi(pr.x, pr.y, pr.z, pr.k)
            assert abs(res[i] - ref) <= tol(ref), i
            n_full += 1
    assert n_full >= 3


def test_full_size_n10000_parity(lib, ctx):
    """C1-sized problem (N = 10,000, D = 5) checked in full against the oracle."""
    p = workloads.random_problem(123, 10000, 1, 1, 3, 4)
    _check_full(lib, ctx, p.x, p.y, p.z, 4, "n10000")


def test_errors(lib, ctx):
    import torch
    x = soa(np.zeros((10, 1), np.float32))
    with pytest.raises(lib.KsgError) as e:
        ctx.cmi(x, x, None, 10)
    assert e.value.status == 2
    with pytest.raises(lib.KsgError) as e:
        ctx.cmi(x, x, None, 0)
    assert e.value.status == 1
    bad = np.ones((50, 1), np.float32)
    bad[7] = np.nan
    with pytest.raises(lib.KsgError) as e:
        ctx.cmi(soa(bad), soa(np.ones((50, 1), np.float32)), None, 4)
    assert e.value.status == 3
    big = soa(np.zeros((50, 32), np.float32))  # 33 columns with Y
    with pytest.raises(lib.KsgError) as e:
        ctx.cmi(big, soa(np.zeros((50, 1), np.float32)), None, 4)
    assert e.value.status == 1
    # the context stays usable after errors
    p = workloads.random_problem(1, 100, 1, 1, 1, 4)
    ref = ksg_cmi(p.x, p.y, p.z, 4)
    assert abs(ctx.cmi(soa(p.x), soa(p.y), soa(p.z), 4) - ref) <= tol(ref)


def test_deterministic(lib, ctx):
    p = workloads.random_problem(9, 3000, 1, 1, 4, 4)
    a = ctx.cmi(soa(p.x), soa(p.y), soa(p.z), 4)
    b = ctx.cmi(soa(p.x), soa(p.y), soa(p.z), 4)
    assert a == b


def _sum_order_bound(n):
    """Largest difference between two FP64 sums of the same per-point terms taken in different
    orders (the grouped search visits the rows in key order): each term is H_a + H_b - H_c
    with |.| <= 3 H_n, each order a tree of depth <= 9 within a tile plus a compensated sum
    over tiles, so two results differ by at most 2 * 9 * 2^-53 * 3 H_n (after the 1/n)."""
    h = float(np.sum(1.0 / np.arange(1, n + 1)))
    return 2 * 9 * 2.0 ** -53 * 3 * h


@pytest.mark.parametrize("m,k", [(0, 4), (1, 4), (3, 8), (8, 4), (14, 2)])
def test_grouped_equals_ungrouped_and_oracle(lib, ctx, m, k):
    """Problems sharing Y and Z (the candidates x surrogates of a greedy step) are searched in
    groups; both group sizes give bit-identical estimates (same radii, counts and summation
    order), equal to the single-problem kernel's up to the order of the FP64 sum, and to the
    oracle's."""
    import torch
    g = workloads.rng(600 + m)
    n, n_cand, n_perm = 700, 5, 13  # 5 x 14 = 70 problems: ragged groups of 8 and 16
    p = workloads.random_problem(700 + m, n, 1, 1, m, k)
    cands = g.standard_normal((n_cand, n)).astype(np.float32)
    cands[1] = (cands[1] + p.y[:, 0]).astype(np.float32)  # one dependent candidate
    perms = workloads.permutations(n, n_perm, seed=800 + m)
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
    assert np.max(np.abs(res[0] - res[8])) <= _sum_order_bound(n)
    for idx in (0, 1, 15, 16, 17, 69):
        c, q = divmod(idx, n_perm + 1)
        x = cands[c] if q == 0 else cands[c][perms[q - 1]]
        ref = ksg_cmi(x, p.y, p.z, k)
        assert abs(res[8][idx] - ref) <= tol(ref), idx


def test_many_groups_xcd_order(lib, ctx):
    """Enough groups for the XCD-interleaved work order (with empty slots); still exact."""
    g = workloads.rng(900)
    n, n_cand, n_perm = 300, 40, 15  # 640 problems -> 40 groups of 16 / 80 groups of 8
    p = workloads.random_problem(901, n, 1, 1, 2, 4)
    cands = g.standard_normal((n_cand, n)).astype(np.float32)
    perms = workloads.permutations(n, n_perm, seed=902)
    y, z = soa(p.y), soa(p.z)
    dc, dp = dev(cands), dev(perms)
    probs = [lib.Problem(dc[c], y, z, 4, perm_x=None if q == 0 else dp[q - 1])
             for c in range(n_cand) for q in range(n_perm + 1)]
    ctx.set_option(ctx.OPT_GROUP_SIZE, 0)
    ref_all = ctx.cmi_batch(probs).cpu().numpy()
    got = {}
    for gs in (8, 16):
        ctx.set_option(ctx.OPT_GROUP_SIZE, gs)
        got[gs] = ctx.cmi_batch(probs).cpu().numpy()
    ctx.set_option(ctx.OPT_GROUP_SIZE, -1)
    assert np.array_equal(got[8], got[16])
    assert np.max(np.abs(got[8] - ref_all)) <= _sum_order_bound(n)
    for idx in (0, 333, 639):
        c, q = divmod(idx, n_perm + 1)
        x = cands[c] if q == 0 else cands[c][perms[q - 1]]
        ref = ksg_cmi(x, p.y, p.z, 4)
        assert abs(ref_all[idx] - ref) <= tol(ref)


def _key_window_case(case):
    """(cands [c][n], y [n], z [n][m], k): inputs that stress the grouped kernel's key order
    and window bounds (the key is Z_1, or Y without Z)."""
    g = workloads.rng(1100 + case)
    if case == 0:  # integer grid: heavy ties in the key and in every distance
        p = workloads.random_problem(1200, 333, 1, 1, 2, 4, kind="grid")
        cands = g.integers(0, 4, size=(3, 333)).astype(np.float32)
        return cands, p.y[:, 0], p.z, 4
    if case == 1:  # constant key column: every row lies inside every window
        p = workloads.random_problem(1201, 257, 1, 1, 2, 3)
        z = p.z.copy()
        z[:, 0] = 0.75
        return g.standard_normal((3, 257)).astype(np.float32), p.y[:, 0], z, 3
    if case == 2:  # fewer rows than one wave
        p = workloads.random_problem(1202, 37, 1, 1, 1, 4)
        return g.standard_normal((3, 37)).astype(np.float32), p.y[:, 0], p.z, 4
    if case == 3:  # signed zeros, denormals and large magnitudes in the key
        p = workloads.random_problem(1203, 300, 1, 1, 2, 4)
        z = p.z.astype(np.float32).copy()
        z[::7, 0] = -0.0
        z[1::7, 0] = 0.0
        z[2::7, 0] = np.float32(1e-40) * g.integers(-3, 4, size=z[2::7, 0].shape)
        z[3::11, 0] = np.float32(3e37)
        return g.standard_normal((3, 300)).astype(np.float32), p.y[:, 0], z, 4
    if case == 4:  # key already sorted (time-ordered trend) and one wave past a tile edge
        n = 4 * 256 + 65
        p = workloads.random_problem(1204, n, 1, 1, 2, 4)
        z = p.z.copy()
        z[:, 0] = np.sort(z[:, 0])
        return g.standard_normal((3, n)).astype(np.float32), p.y[:, 0], z, 4
    if case == 5:  # no Z (the key is Y; the count pass scans every row)
        p = workloads.random_problem(1205, 500, 1, 1, 0, 4, kind="grid")
        return g.integers(0, 5, size=(3, 500)).astype(np.float32), p.y[:, 0], None, 4
    # case 6: every row repeated six times in all columns: the unpermuted problems have eps = 0
    # at every row (all radii equal), the surrogates a mix of zero and positive radii
    p = workloads.random_problem(1206, 60, 1, 1, 2, 4)
    rep = np.repeat(np.arange(60), 6)
    cands = np.repeat(g.standard_normal((3, 60)).astype(np.float32), 6, axis=1)
    return cands, p.y[rep, 0], p.z[rep], 4


@pytest.mark.parametrize("case", range(7))
def test_grouped_key_window_edge_cases(lib, ctx, case):
    """Ties, constant and degenerate keys, short and ragged inputs: the key-ordered grouped
    search equals the oracle on every candidate and surrogate."""
    cands, y, z, k = _key_window_case(case)
    n = y.shape[0]
    n_perm = 5
    perms = workloads.permutations(n, n_perm, seed=1300 + case)
    dc, dp = dev(cands), dev(perms)
    yd, zd = soa(y), soa(z)
    probs = [lib.Problem(dc[c], yd, zd, k, perm_x=None if q == 0 else dp[q - 1])
             for c in range(cands.shape[0]) for q in range(n_perm + 1)]
    got = {}
    for gs in (0, 8, 16):
        ctx.set_option(ctx.OPT_GROUP_SIZE, gs)
        got[gs] = ctx.cmi_batch(probs).cpu().numpy()
    ctx.set_option(ctx.OPT_GROUP_SIZE, -1)
    assert np.array_equal(got[8], got[16])
    assert np.max(np.abs(got[8] - got[0])) <= _sum_order_bound(n)
    zz = np.zeros((n, 0), np.float32) if z is None else z
    for idx in range(len(probs)):
        c, q = divmod(idx, n_perm + 1)
        x = cands[c] if q == 0 else cands[c][perms[q - 1]]
        ref = ksg_cmi(x, y, zz, k)
        assert abs(got[8][idx] - ref) <= tol(ref), (case, idx)


def test_autotune_table_and_cache(lib, ctx, tmp_path):
    path = str(tmp_path / "tune.txt")
    a = ctx.autotune(2048, cache_path=path)
    assert all(g in (8, 16) for g in a["k<=4"] + a["k<=8"]) and len(a["k<=4"]) == 15
    assert set(a["tile_q"].values()) <= {64, 128, 256}
    assert sorted(int(d) for d in a["window_min_n"]) == list(range(3, 17))
    assert all(v in (None, 2048, 8192, 32768) for v in a["window_min_n"].values())
    print("autotune", a)
    b = ctx.autotune(2048, cache_path=path)  # served from the cache
    assert a == b
    assert open(path).read().count("\n") == 1
    # the tuned context still gives the oracle's estimates (brute force, windows, groups)
    probs, _ = workloads.uneven_batch(seed=2, n_problems=12, n_lo=2000, n_hi=6000)
    cols = [(soa(p.x), soa(p.y), soa(p.z)) for p in probs]
    got = ctx.cmi_batch([lib.Problem(x, y, z, p.k) for (x, y, z), p in zip(cols, probs)]).cpu().numpy()
    for i in (0, 5, 11):
        ref = ksg_cmi(probs[i].x, probs[i].y, probs[i].z, probs[i].k)
        assert abs(got[i] - ref) <= tol(ref), i


@pytest.mark.parametrize("tq", [64, 128])
@pytest.mark.parametrize("dims", [(1, 1, 2), (2, 1, 3), (2, 2, 9), (3, 2, 14)])
def test_tile_heights_match_oracle(lib, ctx, tq, dims):
    """Brute-force launches with 64- and 128-query tiles: counts and radii as the oracle's, the
    estimate equal to the 256-query tiling up to the order of the FP64 sum."""
    import torch
    n = 613 + 11 * sum(dims)  # ragged last tile at every height
    p = workloads.random_problem(900 + tq + sum(dims), n, *dims, 4)
    ctx.set_option(ctx.OPT_GROUP_SIZE, 0)  # the batch below runs the brute-force kernel
    ctx.set_option(ctx.OPT_TILE_Q, tq)
    try:
        cmi = _check_full(lib, ctx, p.x, p.y, p.z, 4, f"{dims} tq={tq}")
        batch = [lib.Problem(soa(p.x), soa(p.y), soa(p.z), 4)] * 3
        small = ctx.cmi_batch(batch).cpu().numpy()
        ctx.set_option(ctx.OPT_TILE_Q, 256)
        full = float(ctx.cmi_batch(batch).cpu().numpy()[0])
    finally:
        ctx.set_option(ctx.OPT_TILE_Q, 0)
        ctx.set_option(ctx.OPT_GROUP_SIZE, -1)
    assert np.all(np.abs(small - full) <= _sum_order_bound(n)) and abs(cmi - full) <= _sum_order_bound(n)
    with pytest.raises(lib.KsgError):
        ctx.set_option(ctx.OPT_TILE_Q, 32)


def test_device_props(lib):
    """The runtime's figures for the device the roofline is priced on."""
    import torch
    p = lib.device_props(0)
    tp = torch.cuda.get_device_properties(0)
    assert p["cus"] == tp.multi_processor_count
    assert p["arch"].startswith("gfx950")
    assert p["wave_size"] == 64 and p["clock_khz"] > 0 and p["total_mem"] == tp.total_memory
    print("device", p)
    with pytest.raises(lib.KsgError):
        lib.device_props(10 ** 6)


@pytest.mark.parametrize("case", range(5))
def test_window_search_matches_oracle(lib, ctx, case):
    """Single problems searched in key order with windows (N >= 2048, k <= 4, a Z column):
    every estimate equals the oracle's, and the brute-force search's up to the FP64 summation
    order.  Batches of multi-column X share Y and Z (as the omnibus test's do); single problems
    of 1-D X are not grouped and take the same path; grid data put many rows on each key."""
    dims, kind, n_perm, k = [((3, 1, 2), "gaussian", 3, 4), ((1, 4, 3), "gaussian", 2, 3),
                             ((1, 1, 2), "gaussian", 0, 4), ((2, 1, 1), "grid", 2, 4),
                             ((1, 2, 5), "unit12", 1, 1)][case]
    n = 2400 + 97 * case
    p = workloads.random_problem(1400 + case, n, *dims, k, kind=kind)
    perms = workloads.permutations(n, max(n_perm, 1), seed=1500 + case)
    xd, yd, zd = soa(p.x), soa(p.y), soa(p.z)
    dp = dev(perms)
    probs = [lib.Problem(xd, yd, zd, k)] + [lib.Problem(xd, yd, zd, k, perm_x=dp[q]) for q in range(n_perm)]
    got = {}
    for w in (1, 0):  # 2: windows from N = 2048 whatever an earlier autotune found
        ctx.set_option(ctx.OPT_WINDOWS, 2 * w)
        got[w] = ctx.cmi_batch(probs).cpu().numpy()
    ctx.set_option(ctx.OPT_WINDOWS, 1)
    assert np.max(np.abs(got[1] - got[0])) <= _sum_order_bound(n)
    for q in range(n_perm + 1):
        xs = p.x if q == 0 else p.x[perms[q - 1]]
        ref = ksg_cmi(xs, p.y, p.z, k)
        assert abs(got[1][q] - ref) <= tol(ref), (case, q)


def _degenerate_key_case(case):
    """Problems whose key column (Z_1) defeats or stresses the windows."""
    if case == 0:  # every key equal: every row lies in every window (N at the window threshold)
        p = workloads.random_problem(1600, 2048, 2, 1, 2, 4)
        p.z[:, 0] = 0.5
    elif case == 1:  # a few keys far out: windows end at large gaps on both sides
        p = workloads.random_problem(1601, 2300, 1, 2, 2, 4)
        g = workloads.rng(1602)
        rows = g.choice(2300, size=9, replace=False)
        p.z[rows, 0] = np.float32(1e30) * np.sign(g.standard_normal(9)).astype(np.float32)
    elif case == 2:  # signed zeros and denormals among the keys (bit order differs from value order at 0)
        p = workloads.random_problem(1603, 2200, 3, 1, 1, 3, kind="grid")
        g = workloads.rng(1604)
        p.z[:, 0] = np.where(g.random(2200) < 0.5, np.float32(-0.0), np.float32(0.0))
        rows = g.choice(2200, size=40, replace=False)
        p.z[rows, 0] = np.float32(1e-40) * g.integers(-3, 4, size=40).astype(np.float32)
    else:  # wide Z with k = 2
        p = workloads.random_problem(1605, 2500, 2, 2, 10, 2)
    p.z = np.ascontiguousarray(p.z.astype(np.float32))
    return p


@pytest.mark.parametrize("case", range(4))
def test_window_search_degenerate_keys(lib, ctx, case):
    """Key-ordered windows on tied, far-out, signed-zero and denormal keys: estimates equal the
    oracle's and the brute-force search's (FP64 summation order aside); the window path runs
    (its operation count, over the pairs it visits, is at most the brute force's)."""
    p = _degenerate_key_case(case)
    n, (dx, dy, dz) = p.n, p.dims
    perms = workloads.permutations(n, 2, seed=1610 + case)
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
    brute = 3 * n * (n - 1) * (4 * (dx + dy + dz) + 2)
    assert ops[0] == pytest.approx(brute, rel=1e-12)
    assert 0 < ops[1] <= brute * 1.05, (ops[1], brute)
    if case == 0:
        assert ops[1] > 0.9 * brute  # no window can exclude a row
    else:
        assert ops[1] < 0.9 * brute
    assert np.max(np.abs(got[1] - got[0])) <= _sum_order_bound(n)
    for q in range(3):
        xs = p.x if q == 0 else p.x[perms[q - 1]]
        ref = ksg_cmi(xs, p.y, p.z, p.k)
        assert abs(got[1][q] - ref) <= tol(ref), (case, q)


_WINDOW_CASES = [((3, 1, 2), "gaussian", 4), ((1, 4, 3), "gaussian", 3), ((2, 1, 1), "grid", 4),
                 ((1, 2, 5), "unit12", 1)]


@pytest.mark.parametrize("case", range(len(_WINDOW_CASES) + 4))
def test_window_search_per_point_outputs(lib, ctx, case):
    """Per-point outputs on the key-ordered window path: eps, the three counts and the local
    values of every row (written to the problem's own rows through the key order) equal the
    oracle's bit for bit, with X permuted (a surrogate) and X/Y swapped shapes; the window path
    ran (its operation count is below the brute force's, except where every key ties)."""
    if case < len(_WINDOW_CASES):
        dims, kind, k = _WINDOW_CASES[case]
        n = 2300 + 61 * case
        p = workloads.random_problem(1700 + case, n, *dims, k, kind=kind)
        x, y, z = p.x, p.y, p.z
    else:
        p = _degenerate_key_case(case - len(_WINDOW_CASES))
        n, dims, k = p.n, p.dims, p.k
        x, y, z = p.x, p.y, p.z
    perm = workloads.permutations(n, 1, seed=1800 + case)[0]
    ctx.set_option(ctx.OPT_WINDOWS, 2)  # windows from N = 2048 whatever an earlier autotune found
    ctx.set_option(ctx.OPT_TIMING, 1)
    try:
        ctx.take_timing()
        eps, cnt, loc, cmi = _run(lib, ctx, x, y, z, k, perm=perm)
        ops = ctx.take_timing()[2]
    finally:
        ctx.set_option(ctx.OPT_WINDOWS, 1)
        ctx.set_option(ctx.OPT_TIMING, 0)
    xs = x[perm]
    e, a, b, c = ksg_counts(xs, y, z, k)
    assert np.array_equal(eps, e) and np.array_equal(cnt[0], a), case
    assert np.array_equal(cnt[1], b) and np.array_equal(cnt[2], c), case
    ref = ksg_cmi_from_counts(n, k, a, b, c)
    assert abs(cmi - ref) <= tol(ref), (case, cmi, ref)
    assert np.allclose(loc, local_terms(n, k, a, b, c), rtol=0, atol=1e-13), case
    brute = n * (n - 1) * (4 * sum(dims) + 2)
    assert 0 < ops <= brute * 1.05, (ops, brute)
    if case != len(_WINDOW_CASES):  # degenerate case 0: every key equal, no row excluded
        assert ops < 0.9 * brute, (ops, brute)


def test_uneven_batch_windows_match_brute_force(lib, ctx):
    """The 64-problem uneven batch without per-point outputs (so that the problems with k <= 4,
    N >= 2048 and a Z column take the key-ordered window search, in the launch configuration
    that the uneven-batch benchmark times): every estimate equals the brute-force search's up
    to the FP64 summation order, and the smallest problems equal the oracle's."""
    probs, _ = workloads.uneven_batch(seed=2)
    batch = [lib.Problem(soa(p.x), soa(p.y), soa(p.z), p.k) for p in probs]
    got = {}
    try:
        for w in (1, 0):  # 2: windows from N = 2048 whatever an earlier autotune found
            ctx.set_option(ctx.OPT_WINDOWS, 2 * w)
            got[w] = ctx.cmi_batch(batch).cpu().numpy()
    finally:
        ctx.set_option(ctx.OPT_WINDOWS, 1)
    n_win = 0
    for i, p in enumerate(probs):
        assert abs(got[1][i] - got[0][i]) <= _sum_order_bound(p.n), i
        n_win += p.k <= 4 and p.n >= 2048 and p.dims[2] >= 1
    assert n_win >= 20
    for i in sorted(range(len(probs)), key=lambda i: probs[i].n)[:4]:
        p = probs[i]
        ref = ksg_cmi(p.x, p.y, p.z, p.k)
        assert abs(got[1][i] - ref) <= tol(ref), i
