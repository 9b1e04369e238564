"""KSG algorithm 2 in conditional form, written out from its definition (test infrastructure only).

Kraskov, Stoegbauer & Grassberger (2004) define two nearest-neighbour MI estimators; the paper
names the KSG estimator (Summary, estimator paragraph) without choosing between them.  This
module is the second one, extended to I(X;Y|Z) by the entropy decomposition
I = H(XZ) + H(YZ) - H(Z) - H(XYZ), each entropy taken with the algorithm-2 rectangle
correction (m - 1)/n for a space of m subspaces whose rectangle holds n points.  Readings:

* max norm inside each of the spaces X, Y, Z; every coordinate difference is one
  round-to-nearest-even FP32 subtraction, |.| and max exact (as in algorithm 1);
* the k nearest neighbours of point i: the k smallest (d_ij, j) pairs over j != i in
  lexicographic order, d_ij the joint max-norm distance (ties at the k-th distance are
  broken by the lower index, because here the neighbours' identities matter);
* eps^S_i = max over those k neighbours of d^S_ij, for S in {X, Y, Z};
* counts with <= and a rectangle per space:
  n_xz(i) = #{j != i : d^X_ij <= eps^X_i and d^Z_ij <= eps^Z_i}, n_yz likewise,
  n_z(i) = #{j != i : d^Z_ij <= eps^Z_i} (every count is >= k: the neighbours are inside);
* with Z:  I = psi(k) - 2/k + <psi(n_z) - psi(n_xz) - psi(n_yz) + 1/n_xz + 1/n_yz>
             = H_{k-1} - 2/k + <H_{n_z-1} - H_{n_xz-1} - H_{n_yz-1} + 1/n_xz + 1/n_yz>;
* without Z (algorithm 2 for MI, n_x and n_y counted in X and Y alone):
  I = psi(k) - 1/k + psi(N) - <psi(n_x) + psi(n_y)>
    = H_{k-1} - 1/k + H_{N-1} - <H_{n_x-1} + H_{n_y-1}>;
  the counts array n_z then holds N - 1.

Two forms: ``ksg2_counts`` (NumPy over blocks of queries, stable argsort for the neighbour
set) and ``ksg2_counts_loops`` (pure-Python loops, small N), plus the exact rational value.
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np

from .harmonic import harmonic_exact, harmonic_table
from .ksg import _as_points, _sub_max

__all__ = ["ksg2_counts", "ksg2_cmi", "ksg2_cmi_from_counts", "ksg2_counts_loops", "ksg2_cmi_exact",
           "ksg2_local_terms"]


def ksg2_counts(x, y, z, k: int, block: int = 256):
    """Per point: eps (joint k-th distance, FP32), the three rectangle sides (FP32 [3][N]:
    X, Y, Z) and the counts n_xz, n_yz, n_z (int64; n_z = N - 1 without Z)."""
    x = np.asarray(x, dtype=np.float32)
    n = x.shape[0]
    x, y, z = _as_points(x, n), _as_points(y, n), _as_points(z, n)
    if not (1 <= k < n):
        raise ValueError("need 1 <= k < N")
    has_z = z.shape[1] > 0
    eps = np.empty(n, dtype=np.float32)
    sides = np.empty((3, n), dtype=np.float32)
    nxz = np.empty(n, dtype=np.int64)
    nyz = np.empty(n, dtype=np.int64)
    nz = np.empty(n, dtype=np.int64)
    for i0 in range(0, n, block):
        i1 = min(n, i0 + block)
        rows = np.arange(i0, i1)
        dX = _sub_max(x[i0:i1], x)
        dY = _sub_max(y[i0:i1], y)
        dZ = _sub_max(z[i0:i1], z)
        joint = np.maximum(np.maximum(dX, dY), dZ)
        joint[rows - i0, rows] = np.inf  # j == i is not a neighbour
        knn = np.argsort(joint, axis=1, kind="stable")[:, :k]  # (distance, index) order
        r = np.arange(i1 - i0)[:, None]
        eps[i0:i1] = joint[r[:, 0], knn[:, k - 1]]
        ex = dX[r, knn].max(axis=1)
        ey = dY[r, knn].max(axis=1)
        ez = dZ[r, knn].max(axis=1)
        sides[0, i0:i1], sides[1, i0:i1], sides[2, i0:i1] = ex, ey, ez
        inX = dX <= ex[:, None]
        inY = dY <= ey[:, None]
        inZ = dZ <= ez[:, None]
        for m in (inX, inY, inZ):
            m[rows - i0, rows] = False  # j == i is not counted
        nxz[i0:i1] = (inX & inZ).sum(axis=1)
        nyz[i0:i1] = (inY & inZ).sum(axis=1)
        nz[i0:i1] = inZ.sum(axis=1) if has_z else n - 1
    return eps, sides, nxz, nyz, nz


def _terms(n: int, k: int, nxz, nyz, nz, has_z: bool):
    """The constant C and the per-point FP64 components whose exact sum S gives I = C + S / N."""
    h = harmonic_table(n)
    nxz, nyz, nz = (np.asarray(a, dtype=np.int64) for a in (nxz, nyz, nz))
    if has_z:
        c = h[k - 1] - 2.0 / k
        comps = [h[nz - 1], -h[nxz - 1], -h[nyz - 1], 1.0 / nxz, 1.0 / nyz]
    else:
        c = h[k - 1] - 1.0 / k + h[n - 1]
        comps = [-h[nxz - 1], -h[nyz - 1]]
    return c, comps


def ksg2_cmi_from_counts(n: int, k: int, nxz, nyz, nz, has_z: bool) -> float:
    """C + (1/N) * (exactly rounded sum of the per-point components), C as in the module doc."""
    c, comps = _terms(n, k, nxz, nyz, nz, has_z)
    s = math.fsum(np.concatenate(comps).tolist())
    return float(c + s / n)


def ksg2_local_terms(n: int, k: int, nxz, nyz, nz, has_z: bool) -> np.ndarray:
    """Pointwise values C + (components of point i), FP64; their mean is the estimate."""
    c, comps = _terms(n, k, nxz, nyz, nz, has_z)
    return c + sum(comps)


def ksg2_cmi(x, y, z, k: int) -> float:
    """Estimated I(X;Y|Z) in nats with algorithm 2."""
    x = np.asarray(x, dtype=np.float32)
    n = x.shape[0]
    has_z = _as_points(z, n).shape[1] > 0
    _, _, nxz, nyz, nz = ksg2_counts(x, y, z, k)
    return ksg2_cmi_from_counts(n, k, nxz, nyz, nz, has_z)


def ksg2_counts_loops(x, y, z, k: int):
    """The same per-point quantities by explicit loops over every ordered pair (small N only)."""
    x = np.asarray(x, dtype=np.float32)
    n = x.shape[0]
    x, y, z = _as_points(x, n), _as_points(y, n), _as_points(z, n)
    has_z = z.shape[1] > 0

    def dist(p, i, j):
        d = np.float32(0.0)
        for a in range(p.shape[1]):
            diff = np.float32(p[j, a]) - np.float32(p[i, a])
            d = max(d, abs(diff))
        return d

    eps, sides, nxz, nyz, nz = [], [], [], [], []
    for i in range(n):
        cand = []
        for j in range(n):
            if j != i:
                dx_, dy_, dz_ = dist(x, i, j), dist(y, i, j), dist(z, i, j)
                cand.append((max(dx_, dy_, dz_), j, dx_, dy_, dz_))
        cand.sort(key=lambda t: (t[0], t[1]))
        nb = cand[:k]
        eps.append(nb[-1][0])
        ex = max(t[2] for t in nb)
        ey = max(t[3] for t in nb)
        ez = max(t[4] for t in nb)
        sides.append((ex, ey, ez))
        nxz.append(sum(1 for t in cand if t[2] <= ex and t[4] <= ez))
        nyz.append(sum(1 for t in cand if t[3] <= ey and t[4] <= ez))
        nz.append(sum(1 for t in cand if t[4] <= ez) if has_z else n - 1)
    return (np.array(eps, dtype=np.float32), np.array(sides, dtype=np.float32).T, np.array(nxz),
            np.array(nyz), np.array(nz))


def ksg2_cmi_exact(x, y, z, k: int) -> Fraction:
    """Exact rational estimator value from the loop counts."""
    x = np.asarray(x, dtype=np.float32)
    n = x.shape[0]
    has_z = _as_points(z, n).shape[1] > 0
    _, _, nxz, nyz, nz = ksg2_counts_loops(x, y, z, k)
    H = harmonic_exact
    s = Fraction(0)
    for a, b, c in zip(nxz, nyz, nz):
        a, b, c = int(a), int(b), int(c)
        if has_z:
            s += H(c - 1) - H(a - 1) - H(b - 1) + Fraction(1, a) + Fraction(1, b)
        else:
            s -= H(a - 1) + H(b - 1)
    const = H(k - 1) - Fraction(2, k) if has_z else H(k - 1) - Fraction(1, k) + H(n - 1)
    return const + s / n
