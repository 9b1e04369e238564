"""Pins of the KSG oracle against facts outside the oracle itself (CPU only).

Each test pins one part of the oracle to something the mathematics fixes:
hand-derived worked values, exact rational arithmetic, a library k-d tree,
closed-form Gaussian CMI, invariances of the estimator, and a second,
loop-based implementation.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest
from scipy import special
from scipy.spatial import cKDTree

import workloads
from oracle.harmonic import harmonic, harmonic_exact, harmonic_table
from oracle.ksg import (ksg_cmi, ksg_cmi_exact, ksg_counts, ksg_counts_loops,
                        ksg_point_counts, local_terms)

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _load(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


# ---------------------------------------------------------------- harmonic numbers

def test_harmonic_exact_small():
    h = harmonic_table(400)
    for n in range(0, 400):
        ex = harmonic_exact(n)
        assert h[n] == float(ex), n  # correctly rounded


def test_harmonic_vs_digamma():
    h = harmonic_table(60000)
    for n in [1, 2, 3, 7, 10, 99, 1000, 9999, 10000, 29950, 50000, 59999]:
        ref = special.digamma(n + 1) + np.euler_gamma
        assert abs(h[n] - ref) <= 8 * np.spacing(ref), n


def test_digamma_constants():
    # psi(n) = H_{n-1} - gamma; constants from the closed forms H_3 = 11/6, H_7 = 363/140
    assert harmonic_exact(3) == Fraction(11, 6)
    assert harmonic_exact(7) == Fraction(363, 140)
    assert abs((harmonic(3) - np.euler_gamma) - 1.2561176684318003) < 1e-15
    assert abs((harmonic(7) - np.euler_gamma) - 2.0156414779556098) < 1e-15


# ---------------------------------------------------------------- worked values

def test_worked_example_ties():
    g = _load("ksg_tiny_ties.json")
    x, y, z = (np.array(g[c], np.float32) for c in "xyz")
    eps, nxz, nyz, nz = ksg_counts(x, y, z, g["k"])
    assert eps.tolist() == g["eps"]
    assert nxz.tolist() == g["n_xz"]
    assert nyz.tolist() == g["n_yz"]
    assert nz.tolist() == g["n_z"]
    exact = ksg_cmi_exact(x, y, z, g["k"])
    assert exact == Fraction(g["cmi_num"], g["cmi_den"])
    assert abs(ksg_cmi(x, y, z, g["k"]) - g["cmi_num"] / g["cmi_den"]) < 1e-15


def test_worked_example_z_empty_is_ksg_mi():
    g = _load("ksg_tiny_ties.json")
    ge = g["z_empty"]
    x, y = (np.array(g[c], np.float32) for c in "xy")
    eps, nx, ny, nz = ksg_counts(x, y, None, g["k"])
    assert eps.tolist() == ge["eps"]
    assert nx.tolist() == ge["n_x"] and ny.tolist() == ge["n_y"] and nz.tolist() == ge["n_z"]
    assert ksg_cmi_exact(x, y, None, g["k"]) == Fraction(ge["cmi_num"], ge["cmi_den"])
    # KSG MI algorithm 1: psi(k) + psi(N) - <psi(n_x+1) + psi(n_y+1)>
    n, k = 6, g["k"]
    mi = special.digamma(k) + special.digamma(n) - np.mean(special.digamma(nx + 1) + special.digamma(ny + 1))
    assert abs(ksg_cmi(x, y, None, k) - mi) < 1e-14


def test_local_terms_worked_example():
    """Pointwise values of the worked example (hand fractions in the fixture), with and without
    Z, from the oracle's own counts; their mean is the estimate."""
    g = _load("ksg_tiny_ties.json")
    x, y, z = (np.array(g[c], np.float32) for c in "xyz")
    for zz, ref in ((z, g), (None, g["z_empty"])):
        _, nxz, nyz, nz = ksg_counts(x, y, zz, g["k"])
        loc = local_terms(6, g["k"], nxz, nyz, nz)
        want = [Fraction(v, ref["local_den"]) for v in ref["local_num"]]
        for got, w in zip(loc, want):
            assert abs(got - float(w)) <= 4e-16 * max(1.0, abs(float(w))), (got, w)
        assert sum(want) / 6 == Fraction(ref["cmi_num"], ref["cmi_den"])
        assert abs(math.fsum(loc) / 6 - ksg_cmi(x, y, zz, g["k"])) <= 1e-15


def test_local_terms_mean_is_the_estimate():
    """On random data the pointwise values average to the estimate (summation-order rounding
    only), and each is psi(k) - psi(n_xz+1) - psi(n_yz+1) + psi(n_z+1) with scipy's digamma."""
    for seed, dims, k in ((31, (1, 1, 2), 4), (32, (2, 1, 0), 3), (33, (1, 2, 3), 8)):
        p = workloads.random_problem(seed, 300, *dims, k)
        _, nxz, nyz, nz = ksg_counts(p.x, p.y, p.z, k)
        loc = local_terms(300, k, nxz, nyz, nz)
        assert abs(math.fsum(loc) / 300 - ksg_cmi(p.x, p.y, p.z, k)) <= 1e-14
        ref = special.digamma(k) - special.digamma(nxz + 1) - special.digamma(nyz + 1) + special.digamma(nz + 1)
        assert np.max(np.abs(loc - ref)) <= 1e-12


def test_fp32_discriminator():
    g = _load("fp32_discriminator.json")
    x = np.array(g["x"], np.float32)
    y = np.array(g["y"], np.float32)
    eps, nx, ny, nz = ksg_counts(x, y, None, g["k"])
    assert eps[0] == g["eps0"]
    assert nx[0] == g["n_x0"]
    e2, nx2, _, _ = ksg_counts_loops(x, y, None, g["k"])
    assert e2[0] == g["eps0"] and nx2[0] == g["n_x0"]
    # the same data with exact differences would count the neighbour
    xd = x.astype(np.float64)
    assert abs(xd[1] - xd[0]) == g["eps0"] + 2 and g["n_x0_if_fp64"] == 1


# ---------------------------------------------------------------- two implementations

@pytest.mark.parametrize("kind", ["gaussian", "grid", "unit12"])
def test_loops_equal_numpy(kind):
    cases = 0
    for seed in range(40):
        g = workloads.rng(1000 + seed)
        n = int(g.integers(5, 28))
        dx, dy, dz = int(g.integers(1, 3)), int(g.integers(1, 3)), int(g.integers(0, 3))
        k = int(g.integers(1, min(6, n - 1) + 1))
        p = workloads.random_problem(seed, n, dx, dy, dz, k, kind=kind)
        if kind == "grid" and seed % 4 == 0:  # exact duplicate rows
            p.x[1], p.y[1], p.z[1] = p.x[0], p.y[0], p.z[0]
        a = ksg_counts(p.x, p.y, p.z, k)
        b = ksg_counts_loops(p.x, p.y, p.z, k)
        for u, v in zip(a, b):
            assert np.array_equal(np.asarray(u), np.asarray(v)), (kind, seed)
        cases += 1
    assert cases == 40


def test_fsum_matches_exact_rational():
    for seed in range(12):
        p = workloads.random_problem(seed, 40, 1, 1, seed % 3, 3, kind="grid" if seed % 2 else "gaussian")
        ex = ksg_cmi_exact(p.x, p.y, p.z, 3)
        # only the last two FP64 operations (s / N and H_{k-1} - s / N) round after the exact
        # fsum; their operands are below 2 here, so the error is a few ulp of 2
        assert abs(ksg_cmi(p.x, p.y, p.z, 3) - float(ex)) <= 4 * np.spacing(2.0)


# ---------------------------------------------------------------- library k-d tree

@pytest.mark.parametrize("dims,k", [((1, 1, 1), 4), ((1, 1, 0), 4), ((2, 1, 3), 8), ((1, 2, 5), 4)])
def test_ckdtree_on_unit_interval(dims, k):
    # On [1, 2) every FP32 difference is exact (Sterbenz), so FP64 distances of the tree equal FP32 ones.
    n = 1500
    p = workloads.random_problem(7 + sum(dims), n, *dims, k, kind="unit12")
    eps, nxz, nyz, nz = ksg_counts(p.x, p.y, p.z, k)
    joint = np.concatenate([p.x, p.y, p.z], axis=1).astype(np.float64)
    d, _ = cKDTree(joint).query(joint, k=k + 1, p=np.inf)
    assert np.array_equal(d[:, k].astype(np.float32), eps)
    assert np.all(eps > 0)
    r = np.nextafter(eps.astype(np.float64), 0)

    def counts(cols):
        if cols.shape[1] == 0:
            return np.full(n, n - 1)
        t = cKDTree(cols.astype(np.float64))
        return t.query_ball_point(cols.astype(np.float64), r=r, p=np.inf, return_length=True) - 1

    assert np.array_equal(counts(np.concatenate([p.x, p.z], 1)), nxz)
    assert np.array_equal(counts(np.concatenate([p.y, p.z], 1)), nyz)
    assert np.array_equal(counts(p.z), nz)


# ---------------------------------------------------------------- invariants

def _case(seed=3, n=600, dims=(1, 2, 2), k=4):
    return workloads.random_problem(seed, n, *dims, k)


def test_xy_symmetry_bit_exact():
    p = _case()
    a = ksg_counts(p.x, p.y, p.z, 4)
    b = ksg_counts(p.y, p.x, p.z, 4)
    assert np.array_equal(a[0], b[0])
    assert np.array_equal(a[1], b[2]) and np.array_equal(a[2], b[1]) and np.array_equal(a[3], b[3])
    assert ksg_cmi(p.x, p.y, p.z, 4) == ksg_cmi(p.y, p.x, p.z, 4)


def test_power_of_two_scaling_bit_exact():
    p = _case()
    base = ksg_counts(p.x, p.y, p.z, 4)
    for m in (-3, 5):
        s = np.float32(2.0 ** m)
        sc = ksg_counts(p.x * s, p.y * s, p.z * s, 4)
        assert np.array_equal(sc[0], base[0] * s)
        for u, v in zip(sc[1:], base[1:]):
            assert np.array_equal(u, v)


def test_joint_row_permutation():
    p = _case()
    perm = workloads.rng(9).permutation(p.n)
    a = ksg_counts(p.x, p.y, p.z, 4)
    b = ksg_counts(p.x[perm], p.y[perm], p.z[perm], 4)
    for u, v in zip(a, b):
        assert np.array_equal(np.asarray(u)[perm], v)
    assert ksg_cmi(p.x, p.y, p.z, 4) == ksg_cmi(p.x[perm], p.y[perm], p.z[perm], 4)


def test_count_inequalities_and_neighbour_ranks():
    p = _case(n=400)
    k = 4
    eps, nxz, nyz, nz = ksg_counts(p.x, p.y, p.z, k)
    assert np.all(nxz <= nz) and np.all(nyz <= nz)
    pts = np.concatenate([p.x, p.y, p.z], 1)
    for i in range(0, p.n, 37):
        d = np.max(np.abs(pts - pts[i]), axis=1).astype(np.float32)
        d = np.delete(d, i)
        assert (d < eps[i]).sum() <= k - 1
        assert (d <= eps[i]).sum() >= k


def test_point_counts_match_block_counts():
    p = _case(n=700)
    full = ksg_counts(p.x, p.y, p.z, 4)
    for i in (0, 1, 350, 699):
        e, a, b, c = ksg_point_counts(p.x, p.y, p.z, 4, i)
        assert e == full[0][i] and a == full[1][i] and b == full[2][i] and c == full[3][i]


def test_duplicates_give_zero_radius():
    # k+1 identical points: eps = 0 and no neighbour lies strictly inside a zero radius
    x = np.array([1, 1, 1, 1, 1, 2, 3, 4], np.float32)
    y = np.array([5, 5, 5, 5, 5, 1, 0, 2], np.float32)
    eps, nxz, nyz, nz = ksg_counts(x, y, None, 4)
    assert eps[0] == 0 and nxz[0] == 0 and nyz[0] == 0 and nz[0] == 0
    e2 = ksg_counts_loops(x, y, None, 4)
    for u, v in zip((eps, nxz, nyz, nz), e2):
        assert np.array_equal(u, v)


# ---------------------------------------------------------------- statistical pins

def _gauss_cmi(cov, ix, iy, iz):
    def ld(idx):
        if not idx:
            return 0.0
        return np.linalg.slogdet(cov[np.ix_(idx, idx)])[1]
    return 0.5 * (ld(ix + iz) + ld(iy + iz) - ld(iz) - ld(ix + iy + iz))


def test_gaussian_closed_form():
    _, _, cov = workloads.gaussian_trivariate(seed=0, n_perm=0)
    exact = _gauss_cmi(cov, [0], [1], [2])
    assert abs(exact - 0.188506) < 5e-6
    assert abs(_gauss_cmi(cov, [0], [1], []) - 0.223144) < 5e-6
    est, est_mi = [], []
    for s in range(20):
        p, _, _ = workloads.gaussian_trivariate(seed=100 + s, n_perm=0)
        est.append(ksg_cmi(p.x, p.y, p.z, 4))
        est_mi.append(ksg_cmi(p.x, p.y, None, 4))
    assert abs(np.mean(est) - exact) < 0.02
    assert abs(np.mean(est_mi) - 0.223144) < 0.02


def test_independence_given_z():
    vals = []
    for s in range(10):
        g = workloads.rng(500 + s)
        z = g.standard_normal(1000)
        x = (z + g.standard_normal(1000)).astype(np.float32)
        y = (z + g.standard_normal(1000)).astype(np.float32)
        vals.append(ksg_cmi(x, y, z.astype(np.float32), 4))
    assert abs(np.mean(vals)) < 0.01
    assert np.max(np.abs(vals)) < 0.05
