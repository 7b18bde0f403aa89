"""Oracle, part 1: the collocation system (TEST INFRASTRUCTURE ONLY).

Follows Sec. 2.2 of Chen, Cao and Serra-Capizzano (arXiv 2202.11288):

* the volume-constrained problem  -L_delta u = f on (0,1), u = g = 0 on the
  interaction volume, with  -L_delta u(x) = int_{|t|<=delta} gamma(t)
  [u(x) - u(x+t)] dt  (eq. (ccs2.5) and the operator definition above it);
* the piecewise-quadratic Lagrange interpolant u_Q (eq. (ccs2.1)) substituted
  for u, collocated at every node x_i = i h and midpoint x_{i-1/2}
  (eq. (ccs2.6)), h = 1/N;
* the shifted-symmetric variant of Sec. 2.2.2 (eq. (system1)): a midpoint row
  sees the quadratic pieces whose end points are midpoints, so every row has
  the same stencil and the block system is [A B; B^T A^] for the constant
  kernel;
* unknowns ordered U_h = [u_1..u_{N-1}, u_{1/2}..u_{N-1/2}] (Sec. 2.2.1).

Readings where the paper is silent (each also listed in the design doc):

* kernels are normalised so that int gamma(s) s^2 ds = 1: constant
  c = 3/(2 delta^3); "weighted" = c*wl for s < 0 and c*wr for s > 0;
  fractional c |s|^(-1-2 alpha) with c = (1-alpha) delta^(2 alpha - 2),
  0 < alpha < 1/2 (beyond 1/2 the product-integration weights diverge);
* when delta/h is not an integer, the last sub-interval I_{r+1} = [r h, delta]
  (Sec. 2.2) is integrated exactly, so the stencil reaches offset r+1;
  when delta < h the same rule integrates over [0, delta];
* the manufactured solution is u = x^2 (1-x)^2 with zero volume data.

All arithmetic is FP64 NumPy; the moment integrals are evaluated in closed
form (constant kernels) or by closed form / binomial series (fractional
kernel).  Pins: the integer coefficients printed after eq. (system1)
(delta = r h, constant kernel), the row-sum identity of Lemma 4.1, exactness
on quadratics, high-precision quadrature of the fractional weights
(tests/test_oracle_discretize.py).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

CONST, WEIGHTED, FRACTIONAL = "const", "weighted", "fractional"


@dataclasses.dataclass(frozen=True)
class Kernel:
    """Interaction kernel gamma on |s| <= delta (Sec. 2.2; normalisation is a
    reading, see module docstring)."""

    kind: str
    delta: float
    alpha: float = 0.0
    wl: float = 1.0
    wr: float = 1.0

    @property
    def c(self) -> float:
        if self.kind in (CONST, WEIGHTED):
            return 3.0 / (2.0 * self.delta ** 3)
        if self.kind == FRACTIONAL:
            return (1.0 - self.alpha) * self.delta ** (2.0 * self.alpha - 2.0)
        raise ValueError(self.kind)

    @property
    def beta(self) -> float:
        """Exponent of |s| in gamma (0 for the piecewise-constant kernels)."""
        return -1.0 - 2.0 * self.alpha if self.kind == FRACTIONAL else 0.0

    def side_weights(self):
        """(left, right) multipliers: left means s = y - x < 0."""
        if self.kind == WEIGHTED:
            return self.wl, self.wr
        return 1.0, 1.0

    def gamma(self, s):
        """gamma(s) itself (used by the quadrature pins only)."""
        s = np.asarray(s, dtype=np.float64)
        a = np.abs(s)
        base = self.c * (a ** self.beta if self.kind == FRACTIONAL else 1.0)
        side = np.where(s < 0, self.side_weights()[0], self.side_weights()[1])
        return np.where(a <= self.delta, base * side, 0.0)


def cells(kernel: Kernel, N: int):
    """Sub-intervals of [0, delta] in units of h: cell k covers [k h, (k+th_k) h].

    r = floor(delta/h) full cells I_1..I_r and, when delta/h is not an
    integer, the partial cell I_{r+1} = [r h, delta] (Sec. 2.2 index sets).
    Returns (k, theta) arrays.
    """
    R = kernel.delta * N  # exact: N is a power of two
    r = int(math.floor(R))
    th = R - r
    k = np.arange(r + (1 if th > 0 else 0), dtype=np.int64)
    theta = np.ones(len(k))
    if th > 0:
        theta[-1] = th
    return k, theta


def _frac_moments(k, theta, beta):
    """J_j = int_0^theta (k+tau)^beta tau^j dtau, j = 0, 1, 2 (dimensionless).

    k = 0: closed form (J_0 diverges and is never used there).
    theta/k <= 1/2: binomial series of (1 + tau/k)^beta, integrated term by
    term.  Otherwise (k = 1, theta > 1/2): substitution s = 1 + tau and
    closed-form powers.
    """
    k = np.asarray(k, dtype=np.float64)
    theta = np.asarray(theta, dtype=np.float64)
    J = np.full((3, len(k)), np.nan)
    z = k == 0
    for j in (1, 2):
        J[j, z] = theta[z] ** (beta + j + 1) / (beta + j + 1)
    s = (~z) & (theta <= 0.5 * np.maximum(k, 1.0))
    if s.any():
        ks, ts = k[s], theta[s]
        x = ts / ks
        for j in range(3):
            acc = np.zeros(len(ks))
            coef = 1.0  # binom(beta, m)
            xm = np.ones(len(ks))
            for m in range(400):
                term = coef * xm / (j + m + 1)
                acc += term
                if np.all(np.abs(term) <= 1e-19 * np.abs(acc)):
                    break
                coef *= (beta - m) / (m + 1)
                xm = xm * x
            J[j, s] = ks ** beta * ts ** (j + 1) * acc
    o = (~z) & (~s)
    if o.any():
        assert np.all(k[o] == 1.0)
        to = theta[o]
        F = lambda e: np.expm1(e * np.log1p(to)) / e  # ((1+theta)^e - 1)/e
        f1, f2, f3 = F(beta + 1), F(beta + 2), F(beta + 3)
        J[0, o] = f1
        J[1, o] = f2 - f1
        J[2, o] = f3 - 2 * f2 + f1
    return J


def cell_moments(kernel: Kernel, N: int):
    """Physical moments int_{cell} gamma_+(t) tau^j dt for the right side with
    unit side weight, tau = t/h - k the local coordinate of cell k."""
    h = 1.0 / N
    k, theta = cells(kernel, N)
    if kernel.kind == FRACTIONAL:
        J = _frac_moments(k, theta, kernel.beta)
        scale = kernel.c * h ** (kernel.beta + 1.0)
    else:
        J = np.stack([theta ** (j + 1) / (j + 1) for j in range(3)])
        scale = kernel.c * h
    return k, theta, scale * J


def cell_integrals(kernel: Kernel, N: int):
    """Product-integration weights of one cell (eq. (ccs2.1) basis).

    On cell k the interpolant is the quadratic through the values at local
    coordinates tau = 0, 1/2, 1 with Lagrange basis
      l_a = 1 - 3 tau + 2 tau^2, l_b = 4 tau - 4 tau^2, l_c = -tau + 2 tau^2.
    Returns (Ia, Ib, Ic, Idiag): Ix = int gamma l_x over the cell, and Idiag
    the cell's contribution int gamma (1 - l_0) to the own-point coefficient
    (l_0 = l_a on cell 0, 0 elsewhere).  Ia[0] is not defined (NaN).
    """
    k, theta, J = cell_moments(kernel, N)
    J0, J1, J2 = J
    Ia = J0 - 3 * J1 + 2 * J2
    Ib = 4 * J1 - 4 * J2
    Ic = -J1 + 2 * J2
    Idiag = np.where(k == 0, 3 * J1 - 2 * J2, J0)
    Ia = np.where(k == 0, np.nan, Ia)
    return k, Ia, Ib, Ic, Idiag


def stencil(kernel: Kernel, N: int):
    """Row stencil W(s2) in half-grid offsets s2 = 2 (y - x_c)/h.

    W(0) is the own-point coefficient int gamma (1 - l_0); W(s2), s2 != 0, is
    -int gamma l_{s2} summed over the cells that contain that point.  Returns
    (W, S) with W[s2 + S] for s2 in [-S, S].  Under the shifted-symmetric rule
    (eq. (system1)) every row -- node or midpoint -- has this stencil.
    """
    k, Ia, Ib, Ic, Idiag = cell_integrals(kernel, N)
    S = 2 * len(k)
    W = np.zeros(2 * S + 1)
    wl, wr = kernel.side_weights()
    for sign, ws in ((+1, wr), (-1, wl)):
        W[S] += ws * Idiag.sum()
        for kk in k:
            if kk > 0:
                W[S + sign * 2 * kk] -= ws * Ia[kk]
            W[S + sign * (2 * kk + 1)] -= ws * Ib[kk]
            W[S + sign * (2 * kk + 2)] -= ws * Ic[kk]
    return W, S


def block_permutation(N: int):
    """Interleaved positions p (x = p h/2, p = 1..2N-1) in block order
    [v; w] = [u_1..u_{N-1}, u_{1/2}..u_{N-1/2}] (Sec. 2.2.1 ordering)."""
    v = 2 * np.arange(1, N)          # x = i h
    w = 2 * np.arange(1, N + 1) - 1  # x = (j - 1/2) h
    return np.concatenate([v, w])


def points_block(N: int):
    """Collocation points x in block order."""
    return block_permutation(N) / (2.0 * N)


def assemble_dense(kernel: Kernel, N: int):
    """Dense collocation matrix (block order), written out row by row.

    Row x_c:  sum over the cells of [x_c - delta, x_c + delta] of
      int gamma(t) [u(x_c) - u_Q(x_c + t)] dt,
    with u_Q's nodal values at points outside (0,1) set to g = 0 and dropped
    (eq. (ccs2.6) with zero volume data).  O(N r) Python work: tiny N only.
    """
    M = 2 * N - 1
    k, Ia, Ib, Ic, Idiag = cell_integrals(kernel, N)
    wl, wr = kernel.side_weights()
    Aint = np.zeros((M + 1, M + 1))  # 1-based interleaved positions
    for p in range(1, M + 1):
        for sign, ws in ((+1, wr), (-1, wl)):
            for kk in k:
                Aint[p, p] += ws * Idiag[kk]
                for off, I in ((2 * kk, Ia[kk]), (2 * kk + 1, Ib[kk]),
                               (2 * kk + 2, Ic[kk])):
                    if off == 0:
                        continue
                    col = p + sign * off
                    if 1 <= col <= M:
                        Aint[p, col] -= ws * I
    perm = block_permutation(N)
    return Aint[np.ix_(perm, perm)]


def assemble_dense_from_blocks(gA, gB, gC, gD, N: int):
    """Dense [A B; C D] from four Toeplitz generators (eq. (blocksystem)).

    Sizes: A (N-1)x(N-1), B (N-1)xN, C Nx(N-1), D NxN, entries T[i,j] =
    t_{j-i}; each generator is ordered from the lowest offset to the highest
    (A: -(N-2)..N-2, B: -(N-2)..N-1, C: -(N-1)..N-2, D: -(N-1)..N-1).
    """
    n = N - 1

    def toe(g, rows, cols, lo):
        i = np.arange(rows)[:, None]
        j = np.arange(cols)[None, :]
        return np.asarray(g, dtype=np.float64)[j - i - lo]

    A = toe(gA, n, n, -(n - 1))
    B = toe(gB, n, n + 1, -(n - 1))
    C = toe(gC, n + 1, n, -n)
    D = toe(gD, n + 1, n + 1, -n)
    return np.block([[A, B], [C, D]])


# --- manufactured solution u = x^2 (1-x)^2, zero outside (0,1) -------------

def u_exact(x):
    x = np.asarray(x, dtype=np.float64)
    return x * x * (1 - x) ** 2


def _U(y):
    """Antiderivative of u on [0,1]: y^3/3 - y^4/2 + y^5/5."""
    return y ** 3 / 3 - y ** 4 / 2 + y ** 5 / 5


def rhs_manufactured(kernel: Kernel, N: int):
    """b = f(x_c), f = -L_delta u for u = x^2(1-x)^2 extended by zero.

    f(x) = int_{|t|<=delta} gamma(t) (u(x) - u~(x+t)) dt, evaluated in closed
    form: piecewise-constant kernels through the antiderivative of u;
    the fractional kernel through the Taylor expansion of u about x (exact,
    degree 4) on the part of the horizon inside (0,1) and u(x) times the
    kernel mass on the part outside.
    """
    x = points_block(N)
    d = kernel.delta
    c = kernel.c
    wl, wr = kernel.side_weights()
    ux = u_exact(x)
    if kernel.kind in (CONST, WEIGHTED):
        right = ux * d - (_U(np.minimum(x + d, 1.0)) - _U(x))
        left = ux * d - (_U(x) - _U(np.maximum(x - d, 0.0)))
        return c * (wr * right + wl * left)
    b = kernel.beta
    t2 = np.minimum(d, 1.0 - x)   # right end of the inside part
    t1 = np.minimum(d, x)         # |left end| of the inside part
    derivs = [2 * x - 6 * x ** 2 + 4 * x ** 3, 2 - 12 * x + 12 * x ** 2,
              -12 + 24 * x, np.full_like(x, 24.0)]
    f = np.zeros_like(x)
    for p, dp in enumerate(derivs, start=1):
        Mp = (t2 ** (b + p + 1) + (-1) ** p * t1 ** (b + p + 1)) / (b + p + 1)
        f -= dp / math.factorial(p) * Mp
    for a in (1.0 - x, x):  # distance to the boundary on each side
        out = a < d
        f += np.where(out, ux * (d ** (b + 1) - np.where(out, a, d) ** (b + 1)) / (b + 1), 0.0)
    return c * f
