"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke run.

This module only *draws* data: it holds none of the estimator's arithmetic
(no distances, neighbour counts, digamma sums, statistics or embeddings).
Both the CPU oracle and the HIP path are fed from here, so that they see
byte-identical FP32 inputs and identical permutation tables.

Every generator draws from ``numpy.random.Generator(PCG64(seed))`` in FP64
and rounds once to FP32.  Random numbers that the method itself consumes
(the surrogate row permutations of the max-statistic test) are produced here
and handed to both sides as data.

Workloads (the shapes of the paper's use case: greedy multivariate transfer
entropy with a nearest-neighbour CMI estimator and surrogate tests):

* ``gaussian_trivariate``: one CMI problem I(X;Y|Z), 1-D each, correlated
  Gaussian (corr(X,Y)=0.6, corr(X,Z)=corr(Y,Z)=0.3), N=1000, k=4, plus 200
  row permutations of X.
* ``ar2_network``: a 5-node linear AR(2) network whose node 0 is driven by
  three other nodes at lags 1..3; 10,005 samples, so 10,000 embedded points
  at maximum lag 5 (25 lagged candidates).
* ``uneven_batch``: 64 independent Gaussian CMI problems with log-uniform N
  in [2000, 50000], X/Y dims 1..2, Z dims 0..10, k in {4, 8}.
* ``logistic_network``: a 20-node coupled logistic-map network (r=4, two
  delayed in-edges per node, coupling 0.1..0.3, noise sigma 0.01), 10 trials
  x 3000 samples.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "rng",
    "permutations",
    "gaussian_trivariate",
    "ar2_network",
    "uneven_batch",
    "logistic_network",
    "random_problem",
    "CmiProblemData",
    "NetworkData",
]


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def permutations(n: int, n_perm: int, seed: int) -> np.ndarray:
    """``n_perm`` independent uniform permutations of ``range(n)``, int32 [n_perm][n]."""
    g = rng(seed)
    out = np.empty((n_perm, n), dtype=np.int32)
    for p in range(n_perm):
        out[p] = g.permutation(n).astype(np.int32)
    return out


@dataclasses.dataclass
class CmiProblemData:
    """One I(X;Y|Z) problem: row-major FP32 point arrays [N][d]."""

    x: np.ndarray
    y: np.ndarray
    z: np.ndarray  # shape [N][0] when Z is empty
    k: int

    @property
    def n(self) -> int:
        return self.x.shape[0]

    @property
    def dims(self):
        return (self.x.shape[1], self.y.shape[1], self.z.shape[1])


@dataclasses.dataclass
class NetworkData:
    """Multivariate time series [n_trials][n_vars][T] FP32 with its ground truth."""

    data: np.ndarray
    edges: list  # (source, target, delay)
    params: dict


def _split(pts: np.ndarray, dx: int, dy: int, dz: int):
    pts = np.ascontiguousarray(pts.astype(np.float32))
    x = np.ascontiguousarray(pts[:, :dx])
    y = np.ascontiguousarray(pts[:, dx:dx + dy])
    z = np.ascontiguousarray(pts[:, dx + dy:dx + dy + dz])
    return x, y, z


def gaussian_trivariate(seed: int = 0, n: int = 1000, k: int = 4, n_perm: int = 200,
                        perm_seed: int = 100):
    """Single-problem workload: correlated trivariate Gaussian, with X permutations."""
    cov = np.array([[1.0, 0.6, 0.3], [0.6, 1.0, 0.3], [0.3, 0.3, 1.0]])
    g = rng(seed)
    chol = np.linalg.cholesky(cov)
    pts = g.standard_normal((n, 3)) @ chol.T
    x, y, z = _split(pts, 1, 1, 1)
    perms = permutations(n, n_perm, perm_seed) if n_perm > 0 else np.zeros((0, n), np.int32)
    return CmiProblemData(x, y, z, k), perms, cov


def random_problem(seed: int, n: int, dx: int, dy: int, dz: int, k: int,
                   kind: str = "gaussian"):
    """A generic seeded problem.

    kind = "gaussian": N(0, Sigma) with Sigma a random correlation matrix.
    kind = "grid": small integers (heavy distance ties and duplicates).
    kind = "unit12": uniform in [1, 2) (every FP32 difference is exact there).
    """
    g = rng(seed)
    d = dx + dy + dz
    if kind == "gaussian":
        a = g.standard_normal((d, d))
        s = a @ a.T / d + 0.25 * np.eye(d)
        s = s / np.sqrt(np.outer(np.diag(s), np.diag(s)))
        pts = g.standard_normal((n, d)) @ np.linalg.cholesky(s).T
    elif kind == "grid":
        pts = g.integers(0, 4, size=(n, d)).astype(np.float64)
    elif kind == "unit12":
        pts = 1.0 + g.random((n, d))
    else:
        raise ValueError(kind)
    x, y, z = _split(pts, dx, dy, dz)
    return CmiProblemData(x, y, z, k)


def uneven_batch(seed: int = 2, n_problems: int = 64, n_lo: int = 2000, n_hi: int = 50000):
    """64 independent Gaussian problems of uneven size and dimension."""
    g = rng(seed)
    probs = []
    covs = []
    for _ in range(n_problems):
        n = int(round(math.exp(g.uniform(math.log(n_lo), math.log(n_hi)))))
        dx = int(g.integers(1, 3))
        dy = int(g.integers(1, 3))
        dz = int(g.integers(0, 11))
        k = int(g.choice([4, 8]))
        d = dx + dy + dz
        a = g.standard_normal((d, d))
        s = a @ a.T / d + 0.25 * np.eye(d)
        s = s / np.sqrt(np.outer(np.diag(s), np.diag(s)))
        pts = g.standard_normal((n, d)) @ np.linalg.cholesky(s).T
        x, y, z = _split(pts, dx, dy, dz)
        probs.append(CmiProblemData(x, y, z, k))
        covs.append(s)
    return probs, covs


def ar2_network(seed: int = 1, n_vars: int = 5, T: int = 10005, burn: int = 1000,
                n_trials: int = 1):
    """5-node linear AR(2) network; node 0 is driven by 3 other nodes at lags 1, 2, 3.

    x_i(t) = a_i1 x_i(t-1) - a_i2 x_i(t-2) + eta_i(t),  a ~ U(0.2, 0.5), eta ~ N(0,1)
    x_0(t) += sum_s c_s x_{j_s}(t-s),  s = 1, 2, 3,  c_s ~ U(0.2, 0.5)
    """
    g = rng(seed)
    a1 = g.uniform(0.2, 0.5, n_vars)
    a2 = g.uniform(0.2, 0.5, n_vars)
    drivers = g.choice(np.arange(1, n_vars), size=3, replace=False)
    cs = g.uniform(0.2, 0.5, 3)
    total = burn + T
    data = np.empty((n_trials, n_vars, T), dtype=np.float32)
    for tr in range(n_trials):
        x = np.zeros((n_vars, total))
        eta = g.standard_normal((n_vars, total))
        for t in range(2, total):
            x[:, t] = a1 * x[:, t - 1] - a2 * x[:, t - 2] + eta[:, t]
            for s in range(3):
                if t - (s + 1) >= 0:
                    x[0, t] += cs[s] * x[drivers[s], t - (s + 1)]
        data[tr] = x[:, burn:].astype(np.float32)
    edges = [(int(drivers[s]), 0, s + 1) for s in range(3)]
    params = dict(a1=a1, a2=a2, drivers=drivers, c=cs, target=0)
    return NetworkData(data, edges, params)


def logistic_network(seed: int = 3, n_nodes: int = 20, n_trials: int = 10, T: int = 3000,
                     burn: int = 1000, noise: float = 0.01, max_delay: int = 5):
    """20-node coupled logistic maps, two delayed in-edges per node.

    x_i(t) = frac[(1 - sum_j c_ij) f(x_i(t-1)) + sum_j c_ij f(x_j(t - d_ij)) + noise*eta],
    f(u) = 4u(1-u), c_ij ~ U(0.1, 0.3), d_ij ~ U{1..max_delay}.
    """
    g = rng(seed)
    parents = []
    for i in range(n_nodes):
        others = np.array([j for j in range(n_nodes) if j != i])
        ps = g.choice(others, size=2, replace=False)
        cs = g.uniform(0.1, 0.3, 2)
        ds = g.integers(1, max_delay + 1, 2)
        parents.append([(int(ps[q]), float(cs[q]), int(ds[q])) for q in range(2)])
    total = burn + T
    data = np.empty((n_trials, n_nodes, T), dtype=np.float32)
    for tr in range(n_trials):
        x = np.zeros((n_nodes, total))
        x[:, :max_delay + 1] = g.random((n_nodes, max_delay + 1))
        eta = g.standard_normal((n_nodes, total))
        csum = np.array([sum(c for _, c, _ in parents[i]) for i in range(n_nodes)])
        for t in range(max_delay + 1, total):
            fx = 4.0 * x[:, t - 1] * (1.0 - x[:, t - 1])
            v = (1.0 - csum) * fx
            for i in range(n_nodes):
                for (j, c, d) in parents[i]:
                    u = x[j, t - d]
                    v[i] += c * 4.0 * u * (1.0 - u)
            v = v + noise * eta[:, t]
            x[:, t] = v - np.floor(v)
        data[tr] = x[:, burn:].astype(np.float32)
    edges = [(j, i, d) for i in range(n_nodes) for (j, _, d) in parents[i]]
    return NetworkData(data, edges, dict(parents=parents))


def mlp_init(seed: int, n_params: int = 5378) -> np.ndarray:
    """He-uniform initial FP32 parameters of the 16-64-64-2 threshold network, biases zero.

    Flat layout: W1 [64][16] | b1 [64] | W2 [64][64] | b2 [64] | W3 [2][64] | b3 [2].
    """
    g = rng(seed)
    shapes = [((64, 16), True), ((64,), False), ((64, 64), True), ((64,), False),
              ((2, 64), True), ((2,), False)]
    parts = []
    for shape, is_w in shapes:
        if is_w:
            lim = math.sqrt(6.0 / shape[1])
            parts.append(g.uniform(-lim, lim, size=shape).ravel())
        else:
            parts.append(np.zeros(shape).ravel())
    out = np.concatenate(parts).astype(np.float32)
    assert out.size == n_params
    return out


def redundant_driver_network(seed: int, T: int = 170, n_trials: int = 2) -> np.ndarray:
    """[n_trials][4][T] FP32: variable 3 driven by variable 0 at lag 1 plus its own past at lag
    1; variable 1 is a near-copy of variable 0 (redundant given it); variable 2 is noise."""
    g = rng(seed)
    x = g.standard_normal((n_trials, 4, T))
    x[:, 1] = x[:, 0] + 0.05 * g.standard_normal((n_trials, T))
    for tr in range(n_trials):
        for t in range(1, T):
            x[tr, 3, t] = 0.9 * x[tr, 0, t - 1] + 0.5 * x[tr, 3, t - 1] + 0.3 * g.standard_normal()
    return x.astype(np.float32)


def proxy_driver_network(seed: int, T: int = 200, n_trials: int = 2) -> np.ndarray:
    """[n_trials][4][T] FP32: variable 3 driven by variables 0 and 1 at lag 1; variable 2 is a
    noisy proxy of their sum (informative alone, redundant once both drivers are known)."""
    g = rng(seed)
    x = g.standard_normal((n_trials, 4, T))
    x[:, 2] = x[:, 0] + x[:, 1] + 0.5 * g.standard_normal((n_trials, T))
    for tr in range(n_trials):
        for t in range(1, T):
            x[tr, 3, t] = x[tr, 0, t - 1] + x[tr, 1, t - 1] + 0.3 * g.standard_normal()
    return x.astype(np.float32)
