"""Oracle, part 5: the weakly singular nonlocal model (TEST INFRASTRUCTURE ONLY).

Sec. 2.1 of arXiv 2202.11288: the operator

    L u(x) = int_0^1 (u(x) - u(y)) |x - y|^(-gamma) dy,   0 <= gamma < 1,

on Omega = (0, 1) with Dirichlet data u(0) = u_0, u(1) = u_N, discretised by
the standard piecewise-quadratic collocation (nodes x_i = i h, midpoints
x_{i-1/2}; the interpolant on each mesh cell [x_k, x_{k+1}] through x_k,
x_{k+1/2}, x_{k+1}) at every node and midpoint, unknowns in the block order
[u_1..u_{N-1}, u_{1/2}..u_{N-1/2}].  Written out, row c of the system is

    L_h U (x_c) = u_c int_0^1 |x_c - y|^-gamma dy
                  - sum_cells sum_basis u_basis int_cell |x_c - y|^-gamma l(y) dy,

i.e. A = D - T: D the variable diagonal (x^(1-gamma) + (1-x)^(1-gamma)) /
(1-gamma) (the matrices D_1, D_2 of eq. (3system)), T the product-integration
weights (the Toeplitz blocks M, Q, P, N of eq. (3system)); the weights of the
two boundary nodes move to the right-hand side with u_0, u_N (the vector K).
This is eq. (3system) divided by its factor eta_{h,gamma} = (3-gamma)
(2-gamma)(1-gamma) / h^(1-gamma): A here is the operator in physical units.

Weights: W(a, l) = int_0^1 |a - t|^-gamma l(t) dt for a cell in local
coordinates t (collocation point at local position a, a multiple of 1/2),
l = 1 - 3t + 2t^2 (left node), 4t - 4t^2 (midpoint), 2t^2 - t (right node),
from the closed-form moments of |s|^-gamma s^i, evaluated with mpmath at 50
digits (the differences of large powers at far cells need it).  Times
h^(1-gamma).

Readings: the printed closed forms of m_k, q_k, n_k,
n_0, m_0 and p_k (k >= 1) equal these weights times eta h^(1-gamma); the
printed p_0 and eta_{i/2} (i >= 2, the vector K) do not (the pins show the
product-integration values instead, which reproduce the paper's Table TT03b).
Time stepping (Sec. 5): u_t + L u = f, BDF4 of eq. (bdf4) with tau = h,
u = e^t (1+x)^6, U^0..U^3 exact, error at t = 1.
"""
from __future__ import annotations

import functools
from math import comb

import mpmath as mp
import numpy as np

from . import tpx

L_LEFT = (1, -3, 2)
L_MID = (0, 4, -4)
L_RIGHT = (0, -1, 2)


@functools.lru_cache(maxsize=None)
def cell_weight(gamma: float, a2: int, ell: tuple) -> float:
    """int_0^1 |a - t|^-gamma l(t) dt with a = a2 / 2 (l given by its
    coefficients in t^0, t^1, t^2)."""
    with mp.workdps(50):
        g = mp.mpf(gamma)
        a = mp.mpf(a2) / 2

        def G(i, s):  # antiderivative of |s|^-g s^i, zero at s = 0
            if s == 0:
                return mp.mpf(0)
            sg = 1 if s > 0 else -1
            return sg ** (i + 1) * abs(s) ** (i + 1 - g) / (i + 1 - g)

        tot = mp.mpf(0)
        for j, cj in enumerate(ell):
            if cj == 0:
                continue
            Ij = mp.mpf(0)
            for i in range(j + 1):  # t^j = (s + a)^j, s = t - a
                Ij += comb(j, i) * a ** (j - i) * (G(i, 1 - a) - G(i, -a))
            tot += cj * Ij
        return float(tot)


def node_weight(gamma, s2):
    """Weight of a node basis function at half-step offset s2 from the
    collocation point: its left cell (as right end) and right cell (as left
    end)."""
    return cell_weight(gamma, 2 - s2, L_RIGHT) + cell_weight(gamma, -s2, L_LEFT)


def mid_weight(gamma, s2):
    """Weight of a midpoint basis function at half-step offset s2."""
    return cell_weight(gamma, 1 - s2, L_MID)


def stencils(gamma: float, N: int):
    """(node-row stencil, midpoint-row stencil) as (W, S), W[s2 + S] = -h^(1-gamma)
    * weight of the unknown at offset s2 (S = 2N: every unknown is reached).
    Node rows see nodes at even offsets, midpoint rows at odd ones."""
    h = 1.0 / N
    S = 2 * N
    sc = h ** (1.0 - gamma)
    Wn = np.zeros(2 * S + 1)
    Wm = np.zeros(2 * S + 1)
    for s2 in range(-S, S + 1):
        wn = node_weight(gamma, s2)
        wm = mid_weight(gamma, s2)
        Wn[s2 + S] = -sc * (wn if s2 % 2 == 0 else wm)
        Wm[s2 + S] = -sc * (wm if s2 % 2 == 0 else wn)
    return (Wn, S), (Wm, S)


def positions(N: int):
    """Half-step positions of the unknowns in block order."""
    return np.concatenate([2 * np.arange(1, N), 2 * np.arange(1, N + 1) - 1])


def variable_diagonal(gamma: float, N: int):
    """int_0^1 |x - y|^-gamma dy at the collocation points (block order)."""
    x = positions(N) / (2.0 * N)
    return (x ** (1 - gamma) + (1 - x) ** (1 - gamma)) / (1 - gamma)


def boundary_coupling(gamma: float, N: int):
    """(K0, K1): h^(1-gamma) times the weights of the boundary nodes x = 0 (its
    right cell only) and x = 1 (its left cell only) in each row; L_h U =
    A U - K0 u_0 - K1 u_N."""
    h = 1.0 / N
    c = positions(N)
    sc = h ** (1.0 - gamma)
    K0 = np.array([sc * cell_weight(gamma, int(ci), L_LEFT) for ci in c])
    K1 = np.array([sc * cell_weight(gamma, int(ci) - (2 * N - 2), L_RIGHT) for ci in c])
    return K0, K1


def assemble_dense(gamma: float, N: int):
    """A = D - T (block order), row by row from the weights."""
    (Wn, S), (Wm, _) = stencils(gamma, N)
    c = positions(N)
    A = np.zeros((2 * N - 1, 2 * N - 1))
    for r, cr in enumerate(c):
        W = Wn if cr % 2 == 0 else Wm
        A[r, :] = W[c - cr + S]
    A[np.arange(2 * N - 1), np.arange(2 * N - 1)] += variable_diagonal(gamma, N)
    return A


def level(gamma: float, N: int) -> tpx.TpX:
    """The finest Toeplitz-plus-Cross level with the variable diagonal as its
    band (main diagonal only)."""
    (Wn, Sn), (Wm, Sm) = stencils(gamma, N)
    T = tpx.from_stencils(Wn, Sn, Wm, Sm, N)
    m = 2 * N - 1
    T.band = (np.zeros(m), variable_diagonal(gamma, N), np.zeros(m))
    return T


def L_poly6(gamma: float, x):
    """L (1+y)^6 at x, in closed form: with (1+y)^6 - (1+x)^6 =
    sum_{k>=1} C(6,k) (1+x)^(6-k) (y-x)^k and int_0^1 |y-x|^-gamma (y-x)^k dy
    = ((1-x)^(k+1-gamma) + (-1)^k x^(k+1-gamma)) / (k+1-gamma)."""
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros_like(x)
    for k in range(1, 7):
        out -= comb(6, k) * (1 + x) ** (6 - k) * ((1 - x) ** (k + 1 - gamma)
                                                  + (-1) ** k * x ** (k + 1 - gamma)) / (k + 1 - gamma)
    return out


def exact(t, x):
    return np.exp(t) * (1.0 + x) ** 6


def bdf4_dense(gamma: float, N: int, steps: int = None):
    """u_t + L u = f to t = steps * h (default 1) with BDF4 at tau = h, every
    step by LU of 25/12 I + tau A; returns (U at the end, max error there)."""
    import scipy.linalg
    from .bdf4 import BDF4_LEAD, history_rhs
    steps = N if steps is None else steps
    A = assemble_dense(gamma, N)
    K0, K1 = boundary_coupling(gamma, N)
    x = positions(N) / (2.0 * N)
    tau = 1.0 / N
    lu = scipy.linalg.lu_factor(BDF4_LEAD * np.eye(2 * N - 1) + tau * A)
    U = [exact(k * tau, x) for k in range(4)]
    for k in range(4, steps + 1):
        t = k * tau
        F = exact(t, x) + np.exp(t) * L_poly6(gamma, x)
        src = tau * (F + K0 * exact(t, 0.0) + K1 * exact(t, 1.0))
        U.append(scipy.linalg.lu_solve(lu, history_rhs(U[-1], U[-2], U[-3], U[-4], src)))
        U = U[-4:]
    return U[-1], float(np.abs(U[-1] - exact(steps * tau, x)).max())


def bdf4_tpx(gamma: float, N: int, steps: int, tol: float = 1e-10, coarsest_log2: int = 5,
             max_iter: int = 200, opts: tpx.Options = tpx.Options()):
    """The same steps solved by the V-cycle iteration on the hierarchy of
    25/12 I + tau A (band included), from U^{k-1}; returns (U, iterations)."""
    from .bdf4 import BDF4_LEAD, history_rhs, shifted_tpx
    tau = 1.0 / N
    H = tpx.Hierarchy.build(shifted_tpx(level(gamma, N), BDF4_LEAD, tau), coarsest_log2)
    K0, K1 = boundary_coupling(gamma, N)
    x = positions(N) / (2.0 * N)
    U = [exact(k * tau, x) for k in range(4)]
    its = []
    for k in range(4, steps + 1):
        t = k * tau
        F = exact(t, x) + np.exp(t) * L_poly6(gamma, x)
        src = tau * (F + K0 * exact(t, 0.0) + K1 * exact(t, 1.0))
        Uk, it, _ = tpx.solve(H, history_rhs(U[-1], U[-2], U[-3], U[-4], src), tol=tol,
                              max_iter=max_iter, opts=opts, x0=U[-1])
        its.append(it)
        U.append(Uk)
        U = U[-4:]
    return U[-1], its
