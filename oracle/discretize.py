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
* unknowns ordered U_h = [u_1..u_{N-1}, u_{1/2}..u_{N-1/2}] (Sec. 2.2.1);
* the standard collocation of Sec. 2.2.1 (eq. (nonsym system)): midpoint rows
  see the mesh cells around them, so C and D differ from B^T and A
  (`midpoint_stencil_standard`, constant and weighted kernels), and non-zero
  volume data g carried to the right-hand side through the coupling of the
  interior rows to the exterior points (`assemble_with_exterior`, the content
  of eqs. (rightside1), (rightside2)).

Readings where the paper is silent:

* kernels are normalised so that int gamma(s) s^2 ds = 1: constant
  c = 3/(2 delta^3); "weighted" = c*wl for s < 0 and c*wr for s > 0;
  fractional c |s|^(-1-2 alpha) with c = (1-alpha) delta^(2 alpha - 2),
  0 < alpha < 1/2 (beyond 1/2 the product-integration weights diverge);
* "fractional_near" (an extension, not in the paper): the same kernel for
  0 < alpha < 1, with the piecewise quadratic replaced on |t| <= h/2 by the
  one quadratic through x_c - h/2, x_c, x_c + h/2, so that the linear term
  cancels between the two sides (principal value) and the rest is
  integrable; product integration of the cell pieces beyond h/2;
* when delta/h is not an integer, the last sub-interval I_{r+1} = [r h, delta]
  (Sec. 2.2) is integrated exactly, so the stencil reaches offset r+1;
  when delta < h the same rule integrates over [0, delta];
* manufactured solutions: u = x^2 (1-x)^2 with zero volume data, and
  u = (1+x)^6 with g = u on the interaction volume (the spatial profile of
  the paper's test solution).

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
FRACTIONAL_NEAR = "fractional_near"
FRACTIONAL_KINDS = (FRACTIONAL, FRACTIONAL_NEAR)


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
        if self.kind in FRACTIONAL_KINDS:
            return (1.0 - self.alpha) * self.delta ** (2.0 * self.alpha - 2.0)
        raise ValueError(self.kind)

    @property
    def beta(self) -> float:
        """Exponent of |s| in gamma (0 for the piecewise-constant kernels)."""
        return -1.0 - 2.0 * self.alpha if self.kind in FRACTIONAL_KINDS else 0.0

    def side_weights(self):
        """(left, right) multipliers: left means s = y - x < 0."""
        if self.kind == WEIGHTED:
            return self.wl, self.wr
        return 1.0, 1.0

    def gamma(self, s):
        """gamma(s) itself (used by the quadrature pins only)."""
        s = np.asarray(s, dtype=np.float64)
        a = np.abs(s)
        base = self.c * (a ** self.beta if self.kind in FRACTIONAL_KINDS else 1.0)
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
        e = beta + j + 1
        if e > 0:  # otherwise the moment diverges (alpha >= 1/2, j = 1)
            J[j, z] = theta[z] ** e / e
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
        # ((1+theta)^e - 1)/e, and its limit log(1+theta) at e = 0
        F = lambda e: np.expm1(e * np.log1p(to)) / e if e != 0 else np.log1p(to)
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
    if kernel.kind in FRACTIONAL_KINDS:
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


def _power_integral(a, b, e):
    """int_a^b tau^(e-1) dtau for 0 < a <= b: (b^e - a^e)/e, log(b/a) at e = 0."""
    if e == 0:
        return math.log(b / a)
    return a ** e * math.expm1(e * math.log(b / a)) / e


def near_field_rule(kernel: Kernel, N: int):
    """The fractional_near kernel's rule on cell 0 (one side, unit side
    weight), in physical units:

    * near part, |t| <= rho h with rho = min(1/2, theta_0): the quadratic
      through the half-grid neighbours, u_c + t (u_+ - u_-)/h
      + 2 t^2 (u_+ - 2 u_c + u_-)/h^2; its linear term integrates to zero
      over the two sides, its quadratic term gives -m (u_+ - 2 u_c + u_-)
      for the two sides together, m = (4/h^2) int_0^{rho h} gamma t^2 dt;
    * far part of cell 0, tau in [rho, theta_0]: the cell's own quadratic
      (basis l_a, l_b, l_c as in `cell_integrals`), moments
      F_j = int gamma tau^j over that sub-interval.

    Returns (m, F0, F1, F2); F_j = 0 when theta_0 <= 1/2."""
    h = 1.0 / N
    _, theta = cells(kernel, N)
    th0 = float(theta[0])
    be = kernel.beta
    scale = kernel.c * h ** (be + 1.0)
    rho = min(0.5, th0)
    m = 4.0 * scale * rho ** (be + 3.0) / (be + 3.0)
    if th0 <= 0.5:
        return m, 0.0, 0.0, 0.0
    F = [scale * _power_integral(rho, th0, be + j + 1.0) for j in range(3)]
    return (m, *F)


def stencil_near(kernel: Kernel, N: int):
    """Row stencil W(s2) of the fractional_near kernel (shifted rule, every
    row the same), as (W, S): cell 0 by `near_field_rule`, cells k >= 1 by
    product integration as in `stencil`."""
    k, Ia, Ib, Ic, Idiag = cell_integrals(kernel, N)
    m, F0, F1, F2 = near_field_rule(kernel, N)
    S = 2 * len(k)
    W = np.zeros(2 * S + 1)
    W[S] += 2.0 * m
    W[S - 1] -= m
    W[S + 1] -= m
    for sign in (+1, -1):
        W[S] += 3 * F1 - 2 * F2                     # int gamma (1 - l_a)
        W[S + sign * 1] -= 4 * F1 - 4 * F2          # l_b
        W[S + sign * 2] -= -F1 + 2 * F2             # l_c
        for kk in k[1:]:
            W[S] += Idiag[kk]
            W[S + sign * 2 * kk] -= Ia[kk]
            W[S + sign * (2 * kk + 1)] -= Ib[kk]
            W[S + sign * (2 * kk + 2)] -= Ic[kk]
    return W, S


def stencil(kernel: Kernel, N: int):
    """Row stencil W(s2) in half-grid offsets s2 = 2 (y - x_c)/h.

    W(0) is the own-point coefficient int gamma (1 - l_0); W(s2), s2 != 0, is
    -int gamma l_{s2} summed over the cells that contain that point.  Returns
    (W, S) with W[s2 + S] for s2 in [-S, S].  Under the shifted-symmetric rule
    (eq. (system1)) every row -- node or midpoint -- has this stencil.
    """
    if kernel.kind == FRACTIONAL_NEAR:
        return stencil_near(kernel, N)
    if kernel.kind == FRACTIONAL and not 0.0 < kernel.alpha < 0.5:
        raise ValueError("product integration of the fractional kernel needs 0 < alpha < 1/2 "
                         "(fractional_near covers 0 < alpha < 1)")
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
    if kernel.kind == FRACTIONAL_NEAR:
        return _assemble_dense_near(kernel, N)
    if kernel.kind == FRACTIONAL and not 0.0 < kernel.alpha < 0.5:
        raise ValueError("product integration of the fractional kernel needs 0 < alpha < 1/2")
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


def _assemble_dense_near(kernel: Kernel, N: int):
    """`assemble_dense` for the fractional_near kernel: each row is the near
    part (second difference on the half grid), the far part of cell 0 and
    the cells k >= 1 on both sides, with exterior values dropped."""
    M = 2 * N - 1
    k, Ia, Ib, Ic, Idiag = cell_integrals(kernel, N)
    m, F0, F1, F2 = near_field_rule(kernel, N)
    Aint = np.zeros((M + 1, M + 1))
    for p in range(1, M + 1):
        terms = [(0, 2.0 * m), (-1, -m), (1, -m)]
        for sign in (+1, -1):
            terms += [(0, 3 * F1 - 2 * F2), (sign, -(4 * F1 - 4 * F2)), (2 * sign, -(-F1 + 2 * F2))]
            for kk in k[1:]:
                terms += [(0, Idiag[kk]), (sign * 2 * kk, -Ia[kk]),
                          (sign * (2 * kk + 1), -Ib[kk]), (sign * (2 * kk + 2), -Ic[kk])]
        for off, v in terms:
            col = p + off
            if 1 <= col <= M:
                Aint[p, col] += v
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
        # int_{-t1}^{t2} t^p |t|^b dt; for b + p + 1 <= 0 (p = 1, alpha >= 1/2)
        # the principal value, the same expression (log(t2/t1) at 0)
        e = b + p + 1
        if e == 0:
            Mp = np.log(t2 / t1)
        else:
            Mp = (t2 ** e + (-1) ** p * t1 ** e) / e
        f -= dp / math.factorial(p) * Mp
    for a in (1.0 - x, x):  # distance to the boundary on each side
        out = a < d
        f += np.where(out, ux * (d ** (b + 1) - np.where(out, a, d) ** (b + 1)) / (b + 1), 0.0)
    return c * f


# --- the standard (unshifted) collocation of Sec. 2.2.1 and volume data -------
#
# eq. (ccs2.6) / eq. (nonsym system): every row uses the quadratic pieces of
# the mesh cells [x_m, x_{m+1}] (nodes at the ends, the midpoint inside).  For
# a node row this is the rule of `stencil` above; a midpoint row x_c sees the
# cells [(k - 1/2) h, (k + 1/2) h] around it, the central one holding x_c as
# its midpoint, and the last one cut at the horizon.  The blocks C and D then
# differ from B^T and A; the system is non-symmetric.  Constant and weighted
# kernels.

STANDARD, SHIFTED = "standard", "shifted"


def midpoint_stencil_standard(kernel: Kernel, N: int):
    """Midpoint-row stencil of the standard scheme, W(s2) in half-grid
    offsets (odd s2: nodes, even s2: midpoints), returned as (W, S) with
    W[s2 + S].  Right side t in [0, delta] (units of h, R = delta N): the
    sub-interval [0, min(1/2, R)] of the central cell and the cells
    [k - 1/2, min(k + 1/2, R)], k = 1, 2, ...; cell k's quadratic goes through
    k - 1/2 (node, s2 = 2k - 1), k (midpoint, s2 = 2k), k + 1/2 (node,
    s2 = 2k + 1) with Lagrange basis, in s = tau - k,
      l_- = 2 s^2 - s,  l_0 = 1 - 4 s^2,  l_+ = 2 s^2 + s.
    The left side is the mirror image (weight wl)."""
    if kernel.kind not in (CONST, WEIGHTED):
        raise ValueError("the standard scheme is set up for the constant and weighted kernels")
    h = 1.0 / N
    R = kernel.delta * N
    subs = [(0.0, min(0.5, R), 0)]
    k = 1
    while k - 0.5 < R:
        subs.append((k - 0.5, min(k + 0.5, R), k))
        k += 1
    S = 2 * subs[-1][2] + 1
    W = np.zeros(2 * S + 1)
    wl, wr = kernel.side_weights()
    c = kernel.c * h

    def mom(a, b, j):  # int_a^b s^j ds
        return (b ** (j + 1) - a ** (j + 1)) / (j + 1)

    for a, b, kk in subs:
        sa, sb = a - kk, b - kk
        J0, J1, J2 = (c * mom(sa, sb, j) for j in range(3))
        Im = 2 * J2 - J1      # int gamma l_-
        I0 = J0 - 4 * J2      # int gamma l_0
        Ip = 2 * J2 + J1      # int gamma l_+
        for sign, ws in ((+1, wr), (-1, wl)):
            # mirror: on the left the cell's "-" end is at -(2k - 1), its "+" end at -(2k + 1)
            W[S] += ws * J0
            if kk == 0:
                W[S] -= ws * I0
            else:
                W[S + sign * 2 * kk] -= ws * I0
            W[S + sign * (2 * kk - 1)] -= ws * Im
            W[S + sign * (2 * kk + 1)] -= ws * Ip
    return W, S


def row_stencils(kernel: Kernel, N: int, scheme: str = SHIFTED):
    """(node-row stencil, midpoint-row stencil), each as (W, S)."""
    Wn = stencil(kernel, N)
    if scheme == SHIFTED:
        return Wn, Wn
    return Wn, midpoint_stencil_standard(kernel, N)


def assemble_with_exterior(kernel: Kernel, N: int, scheme: str = SHIFTED):
    """Dense collocation rows over interior AND exterior points.

    Returns (A, E, q_ext): A is the (2N-1)^2 block-ordered matrix of the
    interior unknowns; E (2N-1 x len(q_ext)) couples the interior rows to the
    exterior half-grid positions q_ext (x = q h/2 <= 0 or >= 1, the points of
    N_out the stencils reach), so that eq. (ccs2.6) with volume data g reads
    A U = F - E g(x_ext), the right-hand side of eqs. (rightside1),
    (rightside2).  Written out row by row; tiny N only."""
    (Wn, Sn), (Wm, Sm) = row_stencils(kernel, N, scheme)
    M = 2 * N - 1
    S = max(Sn, Sm)
    q_ext = np.concatenate([np.arange(-S, 1), np.arange(2 * N, 2 * N + S + 1)])
    col_of_ext = {int(q): i for i, q in enumerate(q_ext)}
    Aint = np.zeros((M + 1, M + 1))
    E = np.zeros((M + 1, len(q_ext)))
    for p in range(1, M + 1):
        W, Sw = (Wn, Sn) if p % 2 == 0 else (Wm, Sm)
        for s2 in range(-Sw, Sw + 1):
            w = W[s2 + Sw]
            if w == 0.0:
                continue
            q = p + s2
            if 1 <= q <= M:
                Aint[p, q] += w
            else:
                E[p, col_of_ext[q]] += w
    perm = block_permutation(N)
    return Aint[np.ix_(perm, perm)], E[perm, :], q_ext


# --- manufactured solution with volume data: u = (1 + x)^6, g = u outside -----

def u_poly6(x):
    return (1.0 + np.asarray(x, dtype=np.float64)) ** 6


def f_poly6(kernel: Kernel, x):
    """f = -L_delta u for u = (1+x)^6 on all of R (so g = u on the interaction
    volume), constant / weighted kernel, closed form through the
    antiderivative U = (1+y)^7 / 7."""
    if kernel.kind not in (CONST, WEIGHTED):
        raise ValueError(kernel.kind)
    x = np.asarray(x, dtype=np.float64)
    d = kernel.delta
    wl, wr = kernel.side_weights()
    U = lambda y: (1.0 + y) ** 7 / 7.0
    ux = u_poly6(x)
    right = ux * d - (U(x + d) - U(x))
    left = ux * d - (U(x) - U(x - d))
    return kernel.c * (wr * right + wl * left)


def volume_correction(kernel: Kernel, N: int, g_left, g_right, scheme: str = SHIFTED):
    """E g (block order) from the stencils, row by row over the rows that
    reach the interaction volume only: g_left[k] = g(-k h/2),
    g_right[k] = g(1 + k h/2), k = 0..S (S = the longer stencil's reach).
    The same numbers as `assemble_with_exterior`'s E @ g without forming E."""
    (Wn, Sn), (Wm, Sm) = row_stencils(kernel, N, scheme)
    S = max(Sn, Sm)
    g_left = np.asarray(g_left, dtype=np.float64)
    g_right = np.asarray(g_right, dtype=np.float64)
    M = 2 * N - 1
    out = np.zeros(M + 1)  # interleaved positions 1..M
    for p in range(1, M + 1):
        W, Sw = (Wn, Sn) if p % 2 == 0 else (Wm, Sm)
        acc = 0.0
        # left exterior points q = -k, offset s2 = -k - p, in reach while s2 >= -Sw
        kl = min(S, Sw - p)
        if kl >= 0:
            k = np.arange(kl + 1)
            acc += W[-k - p + Sw] @ g_left[:kl + 1]
        # right exterior points q = 2N + k, offset s2 = 2N + k - p, in reach while s2 <= Sw
        kr = min(S, Sw - 2 * N + p)
        if kr >= 0:
            k = np.arange(kr + 1)
            acc += W[2 * N + k - p + Sw] @ g_right[:kr + 1]
        out[p] = acc
    return out[block_permutation(N)]


def volume_reach(kernel: Kernel, N: int, scheme: str = SHIFTED):
    (Wn, Sn), (Wm, Sm) = row_stencils(kernel, N, scheme)
    return max(Sn, Sm)
