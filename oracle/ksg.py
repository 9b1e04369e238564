"""KSG conditional mutual information, written out from its definition (test infrastructure only).

Estimator: Kraskov, Stoegbauer & Grassberger (2004), algorithm 1 - the
nonlinear nearest-neighbour estimator the paper names for accurate
continuous-valued (C)MI and TE (Summary, estimator paragraph) - in the
conditional form of Frenzel & Pompe (2007).  The paper prints no formula;
the readings taken are:

* max (Chebyshev) norm in every space;
* every coordinate difference is one IEEE round-to-nearest-even FP32
  subtraction fl32(a_j - a_i); |.| and max are exact;
* eps_i = k-th smallest element of the multiset {d_ij : j != i} of joint
  distances (ties need no tie-break: only the value is used);
* n_S(i) = #{j != i : d^S_ij < eps_i} for S in {XZ, YZ, Z} (strict), with
  d^S == 0 when S is empty;
* I = psi(k) - <psi(n_xz+1) + psi(n_yz+1) - psi(n_z+1)>, in nats, not clipped,
  which equals H_{k-1} - (1/N) sum_i [H_{n_xz} + H_{n_yz} - H_{n_z}].

Three forms:

* ``ksg_counts`` / ``ksg_cmi`` (O1): NumPy, one block of query rows at a time,
  the full [B][N] distance matrix per subspace, ``np.partition`` for the k-th
  value, ``math.fsum`` for the FP64 digamma sum.
* ``ksg_counts_loops`` (O2): pure-Python double loop with numpy.float32
  scalar arithmetic, for N <= ~60.
* ``ksg_cmi_exact``: the same counts, exact rational sum (``Fraction``).
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np

from .harmonic import harmonic_exact, harmonic_table

__all__ = [
    "ksg_counts",
    "ksg_cmi",
    "ksg_cmi_from_counts",
    "ksg_counts_loops",
    "ksg_cmi_exact",
    "ksg_point_counts",
    "local_terms",
]


def _as_points(a, n):
    if a is None:
        return np.zeros((n, 0), dtype=np.float32)
    a = np.asarray(a, dtype=np.float32)
    if a.ndim == 1:
        a = a.reshape(n, 1)
    if a.size == 0:
        return np.zeros((n, 0), dtype=np.float32)
    return np.ascontiguousarray(a)


def _sub_max(block: np.ndarray, pts: np.ndarray) -> np.ndarray:
    """max over the columns of |fl32(pts[j, a] - block[b, a])|, shape [B][N] float32.

    Returns zeros when the subspace has no columns (d^{empty} == 0).
    """
    B, N = block.shape[0], pts.shape[0]
    out = np.zeros((B, N), dtype=np.float32)
    for a in range(pts.shape[1]):
        diff = pts[None, :, a] - block[:, None, a]  # float32 - float32 -> float32 (RNE)
        np.maximum(out, np.abs(diff), out=out)
    return out


def ksg_counts(x, y, z, k: int, block: int = 256):
    """Per-point eps_i (FP32) and strict counts n_xz, n_yz, n_z (int64)."""
    x = np.asarray(x, dtype=np.float32)
    n = x.shape[0]
    x, y, z = _as_points(x, n), _as_points(y, n), _as_points(z, n)
    if not (1 <= k < n):
        raise ValueError("need 1 <= k < N")
    eps = np.empty(n, dtype=np.float32)
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
        joint[rows - i0, rows] = np.inf  # exclude j == i
        e = np.partition(joint, k - 1, axis=1)[:, k - 1]
        eps[i0:i1] = e
        dXZ = np.maximum(dX, dZ)
        dYZ = np.maximum(dY, dZ)
        for dist, out in ((dXZ, nxz), (dYZ, nyz), (dZ, nz)):
            dist[rows - i0, rows] = np.inf  # exclude j == i from the counts
            out[i0:i1] = (dist < e[:, None]).sum(axis=1)
    return eps, nxz, nyz, nz


def ksg_cmi_from_counts(n: int, k: int, nxz, nyz, nz) -> float:
    """H_{k-1} - (1/N) sum_i [H_nxz + H_nyz - H_nz] with an exactly rounded (fsum) inner sum."""
    h = harmonic_table(n)
    terms = np.concatenate([h[np.asarray(nxz)], h[np.asarray(nyz)], -h[np.asarray(nz)]])
    s = math.fsum(terms.tolist())
    return float(h[k - 1] - s / n)


def ksg_cmi(x, y, z, k: int) -> float:
    """Estimated I(X;Y|Z) in nats (O1)."""
    x = np.asarray(x, dtype=np.float32)
    n = x.shape[0]
    _, nxz, nyz, nz = ksg_counts(x, y, z, k)
    return ksg_cmi_from_counts(n, k, nxz, nyz, nz)


def local_terms(n: int, k: int, nxz, nyz, nz) -> np.ndarray:
    """Pointwise (local) CMI values psi(k) - psi(n_xz+1) - psi(n_yz+1) + psi(n_z+1), FP64."""
    h = harmonic_table(n)
    return h[k - 1] - (h[np.asarray(nxz)] + h[np.asarray(nyz)] - h[np.asarray(nz)])


def ksg_point_counts(x, y, z, k: int, i: int):
    """eps_i and the three strict counts of one query point i (O(N) memory), for sampled checks."""
    x = np.asarray(x, dtype=np.float32)
    n = x.shape[0]
    x, y, z = _as_points(x, n), _as_points(y, n), _as_points(z, n)
    dX = _sub_max(x[i:i + 1], x)[0]
    dY = _sub_max(y[i:i + 1], y)[0]
    dZ = _sub_max(z[i:i + 1], z)[0]
    joint = np.maximum(np.maximum(dX, dY), dZ)
    joint[i] = np.inf
    e = np.partition(joint, k - 1)[k - 1]
    dXZ = np.maximum(dX, dZ)
    dYZ = np.maximum(dY, dZ)
    dXZ[i] = dYZ[i] = np.inf
    dZ = dZ.copy()
    dZ[i] = np.inf
    return (np.float32(e), int((dXZ < e).sum()), int((dYZ < e).sum()), int((dZ < e).sum()))


def ksg_counts_loops(x, y, z, k: int):
    """O2: the same quantities by explicit loops over every ordered pair (small N only)."""
    x = np.asarray(x, dtype=np.float32)
    n = x.shape[0]
    x, y, z = _as_points(x, n), _as_points(y, n), _as_points(z, n)

    def dist(p, i, j):
        d = np.float32(0.0)
        for a in range(p.shape[1]):
            diff = np.float32(p[j, a]) - np.float32(p[i, a])  # one FP32 subtraction
            d = max(d, abs(diff))
        return d

    eps, nxz, nyz, nz = [], [], [], []
    for i in range(n):
        joint = []
        sub = []
        for j in range(n):
            if j == i:
                continue
            dx_, dy_, dz_ = dist(x, i, j), dist(y, i, j), dist(z, i, j)
            joint.append(max(dx_, dy_, dz_))
            sub.append((max(dx_, dz_), max(dy_, dz_), dz_))
        e = sorted(joint)[k - 1]
        eps.append(e)
        nxz.append(sum(1 for s in sub if s[0] < e))
        nyz.append(sum(1 for s in sub if s[1] < e))
        nz.append(sum(1 for s in sub if s[2] < e))
    return (np.array(eps, dtype=np.float32), np.array(nxz), np.array(nyz), np.array(nz))


def ksg_cmi_exact(x, y, z, k: int) -> Fraction:
    """Exact rational estimator value from the O2 counts."""
    x = np.asarray(x, dtype=np.float32)
    n = x.shape[0]
    _, nxz, nyz, nz = ksg_counts_loops(x, y, z, k)
    s = Fraction(0)
    for a, b, c in zip(nxz, nyz, nz):
        s += harmonic_exact(int(a)) + harmonic_exact(int(b)) - harmonic_exact(int(c))
    return harmonic_exact(k - 1) - s / n
