"""Oracle, part 2: dense algebraic multigrid (TEST INFRASTRUCTURE ONLY).

Plain dense FP64 transcription of Sec. 3.1 of arXiv 2202.11288 for small N:

* restriction I_k^{k-1} = 1/4 [1 2 1] (stride 2) applied to the block-ordered
  level vector [v; w] of length 2 n_k + 1, prolongation I_{k-1}^k = 2 (I_k^{k-1})^T
  (Sec. 3.1; pinned exactly by Example 1);
* Galerkin coarse operators A_{k-1} = I_k^{k-1} A_k I_{k-1}^k (eq. (block Galerkin));
* damped Jacobi u <- u + omega D^{-1} (b - A u) (eq. (7 Jacobi): S = I - omega D^-1 A
  is its error propagator -- the printed update is read this way);
* the block V-cycle of Algorithm 2 from a zero initial guess, with exactly m2
  post-sweeps, and an exact solve on the coarsest level;
* the stationary outer iteration x <- x + B_K (b - A x) stopped when
  ||r_i||_2 / ||r_0||_2 < tol (Sec. 5).

Level k has 2^k intervals: v-size n_k = 2^k - 1, total 2 n_k + 1.  The
coarsest level is 2^kc intervals (63 unknowns for kc = 5).
"""
from __future__ import annotations

import dataclasses

import numpy as np


def restriction(m_fine: int):
    """R of size ((m_fine-1)/2) x m_fine: row i has 1/4 [1 2 1] at columns
    2i, 2i+1, 2i+2 (0-based), i.e. the matrix printed in Sec. 3.1."""
    assert m_fine % 2 == 1
    mc = (m_fine - 1) // 2
    R = np.zeros((mc, m_fine))
    for i in range(mc):
        R[i, 2 * i] = 0.25
        R[i, 2 * i + 1] = 0.5
        R[i, 2 * i + 2] = 0.25
    return R


def prolongation(m_fine: int):
    """P = 2 R^T (Sec. 3.1)."""
    return 2.0 * restriction(m_fine).T


@dataclasses.dataclass
class DenseHierarchy:
    """Dense operators of every level, finest first."""

    A: list            # A[0] = finest
    R: list            # R[l]: level l -> level l+1 (coarser)
    P: list
    lu_coarsest: tuple  # (LU, piv) from scipy.linalg.lu_factor

    @property
    def nlevels(self):
        return len(self.A)


def build_hierarchy(A_fine, coarsest_log2: int = 5):
    """Galerkin hierarchy A_{k-1} = R A_k P down to 2^coarsest_log2 intervals."""
    import scipy.linalg

    A = [np.asarray(A_fine, dtype=np.float64)]
    R, P = [], []
    m = A[0].shape[0]
    m_coarsest = 2 ** (coarsest_log2 + 1) - 1
    assert m >= m_coarsest
    while m > m_coarsest:
        Rl, Pl = restriction(m), prolongation(m)
        R.append(Rl)
        P.append(Pl)
        A.append(Rl @ A[-1] @ Pl)
        m = A[-1].shape[0]
    return DenseHierarchy(A, R, P, scipy.linalg.lu_factor(A[-1]))


@dataclasses.dataclass(frozen=True)
class Options:
    m1: int = 1
    m2: int = 1
    omega_pre: float = 2.0 / 3.0
    omega_post: float = 2.0 / 3.0
    cycle: int = 1  # coarse-level visits per cycle: 1 = V, 2 = W (Toeplitz-plus-Cross path)


def jacobi(A, u, b, omega):
    """One damped-Jacobi sweep (eq. (7 Jacobi))."""
    return u + omega * (b - A @ u) / np.diag(A)


def vcycle(H: DenseHierarchy, b, opts: Options = Options(), level: int = 0):
    """B_k b of Algorithm 2 (zero initial guess)."""
    import scipy.linalg

    if level == H.nlevels - 1:
        return scipy.linalg.lu_solve(H.lu_coarsest, b)
    A = H.A[level]
    u = np.zeros_like(b)
    for _ in range(opts.m1):
        u = jacobi(A, u, b, opts.omega_pre)
    e = vcycle(H, H.R[level] @ (b - A @ u), opts, level + 1)
    u = u + H.P[level] @ e
    for _ in range(opts.m2):
        u = jacobi(A, u, b, opts.omega_post)
    return u


def solve(H: DenseHierarchy, b, tol=1e-10, max_iter=500, opts: Options = Options(), x0=None):
    """Stationary iteration x <- x + B_K (b - A x) with Sec. 5's stopping rule.

    Returns (x, iterations, history) with history[i] = ||b - A x_i|| / ||r_0||.
    """
    A = H.A[0]
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    r = b - A @ x
    r0 = np.linalg.norm(r)
    hist = [1.0]
    it = 0
    while hist[-1] >= tol and it < max_iter:
        x = x + vcycle(H, r, opts)
        r = b - A @ x
        it += 1
        hist.append(np.linalg.norm(r) / r0)
    return x, it, np.array(hist)


def two_grid_error_operator(A, omega, m1=0, m2=1):
    """E = S^m2 T S^m1 with T = I - P A_c^{-1} R A (Sec. 3.1, T_k) and
    S = I - omega D^{-1} A; Theorem 4.1 bounds ||S T||_A for m1=0, m2=1."""
    m = A.shape[0]
    R, P = restriction(m), prolongation(m)
    Ac = R @ A @ P
    T = np.eye(m) - P @ np.linalg.solve(Ac, R @ A)
    S = np.eye(m) - omega * (A / np.diag(A)[:, None])
    E = T
    for _ in range(m1):
        E = E @ S
    for _ in range(m2):
        E = S @ E
    return E


def energy_norm(E, A):
    """||E||_A = ||A^{1/2} E A^{-1/2}||_2 for SPD A."""
    w, V = np.linalg.eigh(A)
    Ah = (V * np.sqrt(w)) @ V.T
    Aih = (V / np.sqrt(w)) @ V.T
    return np.linalg.norm(Ah @ E @ Aih, 2)
