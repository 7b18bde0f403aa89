"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle
checks.  This module holds no arithmetic of the multigrid method: only random
draws (parameters, right-hand sides, test vectors) and the closed-form
manufactured solution u(x) = x^2 (1-x)^2 used to measure discretisation error.
"""
from __future__ import annotations

import numpy as np


def rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(seed)


def random_vector(m: int, seed: int) -> np.ndarray:
    """N(0,1) entries, FP64."""
    return rng(seed).standard_normal(m)


def random_tpx_arrays(n: int, seed: int, decay: float = 0.0):
    """Random finest-level Toeplitz generators for [A B; C D] with n = N-1
    (A: 2n-1, B: 2n, C: 2n, D: 2n+1 entries, lowest offset first).  With
    decay > 0 entries fall off like exp(-decay*|offset|) around a dominant
    diagonal, which keeps the operator comfortably invertible."""
    g = rng(seed)

    def gen(lo, hi, diag=0.0):
        off = np.arange(lo, hi + 1)
        v = g.standard_normal(len(off))
        if decay > 0:
            v *= np.exp(-decay * np.abs(off))
        v[off == 0] += diag
        return v

    return (gen(-(n - 1), n - 1, 4.0), gen(-(n - 1), n), gen(-n, n - 1),
            gen(-n, n, 4.0))


def u_manufactured(x):
    """u(x) = x^2 (1-x)^2 (zero volume-constraint data on both sides)."""
    x = np.asarray(x, dtype=np.float64)
    return x * x * (1.0 - x) ** 2


def points_block(N: int) -> np.ndarray:
    """Grid points in the paper's unknown order [x_1..x_{N-1}, x_{1/2}..x_{N-1/2}]."""
    v = np.arange(1, N) / N
    w = (np.arange(1, N + 1) - 0.5) / N
    return np.concatenate([v, w])
