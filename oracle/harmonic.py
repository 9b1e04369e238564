"""Harmonic numbers H_n = sum_{m=1}^{n} 1/m  (test infrastructure only).

The KSG estimator is written with digamma values psi(n+1) of integer counts.
For integers psi(n+1) = -gamma + H_n, and every digamma term of the CMI sum
enters with a +1/-1 weight whose total is +1 - (1 + 1 - 1) = 0, so gamma
cancels exactly and the estimator is a rational number fixed by the counts:

    I = H_{k-1} - (1/N) sum_i [H_{n_xz(i)} + H_{n_yz(i)} - H_{n_z(i)}].

``harmonic_table`` evaluates H_n to FP64 by mpmath at 120 bits (correctly
rounded in all practical cases); ``harmonic_exact`` returns the exact rational.
"""
from __future__ import annotations

import functools
from fractions import Fraction

import mpmath
import numpy as np


@functools.lru_cache(maxsize=None)
def _table(nmax: int) -> np.ndarray:
    out = np.empty(nmax + 1, dtype=np.float64)
    with mpmath.workprec(120):
        for n in range(nmax + 1):
            out[n] = float(mpmath.harmonic(n)) if n > 0 else 0.0
    out.setflags(write=False)
    return out


def harmonic_table(nmax: int) -> np.ndarray:
    """FP64 array [H_0 .. H_nmax] (read-only, cached; rounded up to a multiple of 4096)."""
    size = max(4096, ((int(nmax) + 4096) // 4096) * 4096)
    return _table(size)[: nmax + 1]


def harmonic(n: int) -> float:
    return float(harmonic_table(int(n))[int(n)])


@functools.lru_cache(maxsize=None)
def harmonic_exact(n: int) -> Fraction:
    """Exact H_n as a Fraction (sum of 1/m)."""
    s = Fraction(0)
    for m in range(1, n + 1):
        s += Fraction(1, m)
    return s
