"""Oracle, part 3: Toeplitz-like-plus-Cross levels (TEST INFRASTRUCTURE ONLY).

Sec. 3.2.2 of arXiv 2202.11288 (eq. (split01)): a level of n = 2^k - 1
v-unknowns and n + 1 w-unknowns, w = [w_o; w_bar], is

    A_k = [A 0 B_bar; 0' 0 0'; C_bar 0 D_bar] + [0 p 0; q o zeta; 0 xi 0]

with four n x n Toeplitz blocks (entries T[i, j] = t_{j-i}, the convention of
Lemma 3.1) and the Cross vectors p (column w_o, v rows), q (row w_o, v
columns), xi (column w_o, w_bar rows), zeta (row w_o, w_bar columns) and the
scalar o.  Generators are stored as arrays g[d + n - 1], d = -(n-1)..n-1.

* ``coarsen`` is Lemma 3.1 written in the paper's notation, with N_k read as
  the number of intervals of level k (= n + 1); under that reading the
  formulas equal the dense Galerkin product (pinned in the tests).
* ``matvec`` uses, for each of the four Toeplitz blocks separately, the
  circulant embedding of eq. (ccs3.4) of size L = 2(n+1) and
  C x = ifft(fft(c) .* fft(x)) (Sec. 3.2), plus the O(n) Cross terms.
* ``vcycle``/``solve`` are the same Algorithm 2 / outer loop as in
  ``oracle.dense`` on this representation (FP64, scipy.fft).
* ``pcg`` is conjugate gradients preconditioned by one V-cycle, the Krylov
  acceleration of the outer iteration for the SPD case.  The paper runs the
  stationary iteration only; ``pcg`` is pinned by properties of CG itself
  (finite termination, monotone energy-norm error, the LU solution), not by
  numbers of the paper.
* ``gmres`` is restarted flexible GMRES right-preconditioned by one V-cycle
  per Arnoldi step, the Krylov acceleration for the non-symmetric operators;
  pinned by the minimal-residual property over the Krylov space (brute-force
  least squares on an explicit basis) and by finite termination.
"""
from __future__ import annotations

import dataclasses
import os

import numpy as np
import scipy.fft
import scipy.linalg

from . import discretize as disc
from .dense import Options

WORKERS = os.cpu_count() or 1


@dataclasses.dataclass
class TpX:
    n: int
    a: np.ndarray
    b: np.ndarray
    c: np.ndarray
    d: np.ndarray
    p: np.ndarray
    q: np.ndarray
    xi: np.ndarray
    zeta: np.ndarray
    o: float
    # optional tridiagonal part on the block-ordered vector (sub, main, super;
    # 2n+1 entries each, sub[0] = super[2n] = 0): the variable diagonal of the
    # weakly singular model (eq. (3system)) and its Galerkin images
    band: tuple = None

    @property
    def size(self):
        return 2 * self.n + 1

    def diag(self):
        n = self.n
        d = np.concatenate([np.full(n, self.a[n - 1]), [self.o], np.full(n, self.d[n - 1])])
        return d if self.band is None else d + self.band[1]

    def band_matvec(self, u):
        if self.band is None:
            return 0.0
        s, m, p = self.band
        y = m * u
        y[1:] += s[1:] * u[:-1]
        y[:-1] += p[:-1] * u[1:]
        return y

    def dense(self):
        n = self.n
        M = np.zeros((2 * n + 1, 2 * n + 1))
        M[:n, :n] = toeplitz_dense(self.a, n)
        M[:n, n + 1:] = toeplitz_dense(self.b, n)
        M[n + 1:, :n] = toeplitz_dense(self.c, n)
        M[n + 1:, n + 1:] = toeplitz_dense(self.d, n)
        M[:n, n] = self.p
        M[n, :n] = self.q
        M[n, n] = self.o
        M[n, n + 1:] = self.zeta
        M[n + 1:, n] = self.xi
        if self.band is not None:
            s, m, p = self.band
            k = np.arange(2 * n + 1)
            M[k, k] += m
            M[k[1:], k[1:] - 1] += s[1:]
            M[k[:-1], k[:-1] + 1] += p[:-1]
        return M


def toeplitz_dense(g, n):
    i = np.arange(n)[:, None]
    j = np.arange(n)[None, :]
    return np.asarray(g)[j - i + n - 1]


def from_dense(M):
    """Split a dense level matrix as in eq. (split01) (Toeplitz-ness is not
    checked here; the tests do)."""
    m = M.shape[0]
    n = (m - 1) // 2

    def gen(T):
        return np.concatenate([T[::-1, 0][:-1], T[0, :]])  # offsets -(n-1)..n-1

    return TpX(n, gen(M[:n, :n]), gen(M[:n, n + 1:]), gen(M[n + 1:, :n]),
               gen(M[n + 1:, n + 1:]), M[:n, n].copy(), M[n, :n].copy(),
               M[n + 1:, n].copy(), M[n, n + 1:].copy(), float(M[n, n]))


def from_stencil(kernel: disc.Kernel, N: int, scheme: str = disc.SHIFTED):
    """Finest level from the row stencils W(s2) (half-grid offsets).

    v_i sits at x = (i+1) h, w_o at h/2, w_bar_j at (j + 3/2) h (0-based).
    Node rows (A, B_bar, p) take the node-row stencil: A at even offsets 2d,
    B_bar at 2d+1, p at the offset to w_o.  Midpoint rows (C_bar, D_bar, q,
    xi, zeta, o) take the midpoint-row stencil: C_bar at 2d-1, D_bar at 2d,
    the w_o row and column at the offsets between w_o and each point.  Under
    the shifted-symmetric rule both stencils are the same; under the standard
    rule (eq. (ccs2.6)) the midpoint rows have their own.
    """
    (Wn, Sn), (Wm, Sm) = disc.row_stencils(kernel, N, scheme)
    return from_stencils(Wn, Sn, Wm, Sm, N)


def from_stencils(Wn, Sn, Wm, Sm, N: int):
    """`from_stencil` for given node-row and midpoint-row stencils."""
    n = N - 1

    def at(W, S):
        def Wat(s2):
            s2 = np.asarray(s2)
            out = np.zeros(s2.shape)
            ok = np.abs(s2) <= S
            out[ok] = W[s2[ok] + S]
            return out
        return Wat

    Wn_at, Wm_at = at(Wn, Sn), at(Wm, Sm)
    d = np.arange(-(n - 1), n)
    i = np.arange(n)
    return TpX(n, Wn_at(2 * d), Wn_at(2 * d + 1), Wm_at(2 * d - 1), Wm_at(2 * d),
               Wn_at(-2 * i - 1), Wm_at(2 * i + 1), Wm_at(-2 * i - 2), Wm_at(2 * i + 2),
               float(Wm_at(np.array(0))))


def from_blocks(gA, gB, gC, gD, N: int):
    """Finest level from generators of A, B, C, D (layout as in
    ``discretize.assemble_dense_from_blocks``)."""
    n = N - 1
    gA, gB, gC, gD = (np.asarray(g, dtype=np.float64) for g in (gA, gB, gC, gD))
    # B: offsets -(n-1)..n ; p = B[:,0] -> p_i = beta_{-i}; B_bar offset d -> beta_{d+1}
    bB = lambda off: gB[off + n - 1]
    # C: offsets -n..n-1 ; q_i = C[0,i] = gamma_i; C_bar offset d -> gamma_{d-1}
    cC = lambda off: gC[off + n]
    dD = lambda off: gD[off + n]
    d = np.arange(-(n - 1), n)
    i = np.arange(n)
    return TpX(n, gA.copy(), bB(d + 1), cC(d - 1), dD(d), bB(-i), cC(i),
               dD(-i - 1), dD(i + 1), float(dD(0)))


def coarsen(T: TpX) -> TpX:
    """Lemma 3.1: the Galerkin coarse level, O(n) work.

    Toeplitz generators: 8 g'_i = g_{2i-2} + 4 g_{2i-1} + 6 g_{2i} + 4 g_{2i+1} + g_{2i+2}.
    Cross vectors (1-based i, N_k = n + 1):
      8 p'_i  = (a_{Nk-2i} + 2a_{Nk-2i-1} + a_{Nk-2i-2}) + 2(p_{2i-1} + 2p_{2i} + p_{2i+1})
                + (b_{-2i+2} + 2b_{-2i+1} + b_{-2i})
      8 q'_i  = (a_{-Nk+2i} + 2a_{-Nk+2i+1} + a_{-Nk+2i+2}) + 2(q_{2i-1} + 2q_{2i} + q_{2i+1})
                + (c_{2i-2} + 2c_{2i-1} + c_{2i})
      8 o'    = (a_0 + 2p_{Nk-1} + b_{-Nk+2}) + 2(q_{Nk-1} + 2o + zeta_1)
                + (c_{Nk-2} + 2xi_1 + d_0)
      8 xi'_i = (c_{Nk-2i} + 2c_{Nk-2i-1} + c_{Nk-2i-2}) + 2(xi_{2i-1} + 2xi_{2i} + xi_{2i+1})
                + (d_{-2i+2} + 2d_{-2i+1} + d_{-2i})
      8 zeta'_i = (b_{-Nk+2i} + 2b_{-Nk+2i+1} + b_{-Nk+2i+2}) + 2(zeta_{2i-1} + 2zeta_{2i} + zeta_{2i+1})
                + (d_{2i-2} + 2d_{2i-1} + d_{2i})
    """
    n = T.n
    Nk = n + 1
    nc = (n - 1) // 2
    g = lambda arr: (lambda off: arr[np.asarray(off) + n - 1])
    a, b, c, d = g(T.a), g(T.b), g(T.c), g(T.d)
    v1 = lambda arr: (lambda i: arr[np.asarray(i) - 1])  # 1-based vectors
    p, q, xi, zeta = v1(T.p), v1(T.q), v1(T.xi), v1(T.zeta)

    ic = np.arange(-(nc - 1), nc)

    def toe(t):
        return (t(2 * ic - 2) + 4 * t(2 * ic - 1) + 6 * t(2 * ic) + 4 * t(2 * ic + 1)
                + t(2 * ic + 2)) / 8.0

    i = np.arange(1, nc + 1)
    pc = ((a(Nk - 2 * i) + 2 * a(Nk - 2 * i - 1) + a(Nk - 2 * i - 2))
          + 2 * (p(2 * i - 1) + 2 * p(2 * i) + p(2 * i + 1))
          + (b(-2 * i + 2) + 2 * b(-2 * i + 1) + b(-2 * i))) / 8.0
    qc = ((a(-Nk + 2 * i) + 2 * a(-Nk + 2 * i + 1) + a(-Nk + 2 * i + 2))
          + 2 * (q(2 * i - 1) + 2 * q(2 * i) + q(2 * i + 1))
          + (c(2 * i - 2) + 2 * c(2 * i - 1) + c(2 * i))) / 8.0
    oc = ((a(0) + 2 * p(Nk - 1) + b(-Nk + 2)) + 2 * (q(Nk - 1) + 2 * T.o + zeta(1))
          + (c(Nk - 2) + 2 * xi(1) + d(0))) / 8.0
    xic = ((c(Nk - 2 * i) + 2 * c(Nk - 2 * i - 1) + c(Nk - 2 * i - 2))
           + 2 * (xi(2 * i - 1) + 2 * xi(2 * i) + xi(2 * i + 1))
           + (d(-2 * i + 2) + 2 * d(-2 * i + 1) + d(-2 * i))) / 8.0
    zc = ((b(-Nk + 2 * i) + 2 * b(-Nk + 2 * i + 1) + b(-Nk + 2 * i + 2))
          + 2 * (zeta(2 * i - 1) + 2 * zeta(2 * i) + zeta(2 * i + 1))
          + (d(2 * i - 2) + 2 * d(2 * i - 1) + d(2 * i))) / 8.0
    return TpX(nc, toe(a), toe(b), toe(c), toe(d), pc, qc, xic, zc, float(oc),
               coarsen_band(T.band, n))


def coarsen_band(band, n):
    """Galerkin image R B P of a tridiagonal B (R = 1/4 [1 2 1] stride 2 on the
    block-ordered vector, P = 2 R^T, Sec. 3.1): again tridiagonal, formed with
    sparse products."""
    if band is None:
        return None
    import scipy.sparse as sp
    m = 2 * n + 1
    mc = n
    s, d, p = band
    B = sp.diags([s[1:], d, p[:-1]], [-1, 0, 1], shape=(m, m), format="csr")
    rows = np.repeat(np.arange(mc), 3)
    cols = (2 * np.arange(mc)[:, None] + np.arange(3)[None, :]).ravel()
    vals = np.tile([0.25, 0.5, 0.25], mc)
    R = sp.csr_matrix((vals, (rows, cols)), shape=(mc, m))
    C = (R @ B @ (2.0 * R.T)).tocsr()
    sc = np.concatenate([[0.0], C.diagonal(-1)])
    pc = np.concatenate([C.diagonal(1), [0.0]])
    return (sc, C.diagonal(0).astype(np.float64), pc)


# --- FFT matvec -------------------------------------------------------------

def circulant_spectrum(g, n):
    """rfft of the first column of the L = 2(n+1) circulant that embeds
    T[i, j] = t_{j-i} (eq. (ccs3.4)): c_m = t_{-m}, c_{L-m} = t_m."""
    L = 2 * (n + 1)
    col = np.zeros(L)
    col[:n] = g[n - 1::-1]          # t_0, t_{-1}, ..., t_{-(n-1)}
    if n > 1:
        col[L - (n - 1):] = g[n:][::-1]      # t_{n-1}, ..., t_1
    return scipy.fft.rfft(col, workers=WORKERS)


def toeplitz_apply(spec, x, n):
    """T x through the circulant embedding: ifft(fft(c) .* fft([x; 0]))[:n]."""
    L = 2 * (n + 1)
    X = scipy.fft.rfft(x, n=L, workers=WORKERS)
    return scipy.fft.irfft(spec * X, n=L, workers=WORKERS)[:n]


@dataclasses.dataclass
class Level:
    T: TpX
    sA: np.ndarray
    sB: np.ndarray
    sC: np.ndarray
    sD: np.ndarray
    diag: np.ndarray

    @classmethod
    def build(cls, T: TpX):
        n = T.n
        return cls(T, circulant_spectrum(T.a, n), circulant_spectrum(T.b, n),
                   circulant_spectrum(T.c, n), circulant_spectrum(T.d, n), T.diag())

    def matvec(self, u):
        """A_k u via the Cross splitting (Sec. 3.2.2)."""
        T, n = self.T, self.T.n
        v, wo, wb = u[:n], u[n], u[n + 1:]
        yv = toeplitz_apply(self.sA, v, n) + toeplitz_apply(self.sB, wb, n) + T.p * wo
        yo = T.q @ v + T.o * wo + T.zeta @ wb
        yw = toeplitz_apply(self.sC, v, n) + toeplitz_apply(self.sD, wb, n) + T.xi * wo
        return np.concatenate([yv, [yo], yw]) + T.band_matvec(u)


def from_stencil_rowsum(kernel: disc.Kernel, N: int, scheme: str = disc.SHIFTED):
    """The finest level of `from_stencil` with every array in long double and
    the own-point weight W(0) = int gamma (1 - l_0) of each row stencil taken
    as -sum_{k != 0} W(k), summed in long double: the quadratic basis is a
    partition of unity on every cell (sum_k l_k = 1), so the two are equal
    and an interior row of the matrix sums to zero (Sec. 2.2).  The FP64
    rounding of W(0) (a number of size c h^-2alpha for the fractional
    kernel) alone moves b - A x by eps |W(0)| |x|; this form defines the
    matrix without it, for `residual_extended`.  Pinned: its diagonal equals
    the integral formula's to a few FP64 units of W(0)."""
    ld = np.longdouble
    (Wn, Sn), (Wm, Sm) = disc.row_stencils(kernel, N, scheme)
    Wn = np.asarray(Wn, dtype=ld)
    Wm = np.asarray(Wm, dtype=ld)
    Wn[Sn] = -(Wn[:Sn].sum() + Wn[Sn + 1:].sum())
    Wm[Sm] = -(Wm[:Sm].sum() + Wm[Sm + 1:].sum())
    n = N - 1

    def at(W, S):
        def Wat(s2):
            s2 = np.asarray(s2)
            out = np.zeros(s2.shape, dtype=ld)
            ok = np.abs(s2) <= S
            out[ok] = W[s2[ok] + S]
            return out
        return Wat

    Wn_at, Wm_at = at(Wn, Sn), at(Wm, Sm)
    d = np.arange(-(n - 1), n)
    i = np.arange(n)
    T = TpX(n, Wn_at(2 * d), Wn_at(2 * d + 1), Wm_at(2 * d - 1), Wm_at(2 * d),
            Wn_at(-2 * i - 1), Wm_at(2 * i + 1), Wm_at(-2 * i - 2), Wm_at(2 * i + 2), 0.0)
    T.o = Wm_at(np.array(0))[()]
    return T


def residual_extended(T: TpX, b, x):
    """b - A x for the level T in extended precision (x86 80-bit long
    double, unit roundoff 5.4e-20): the definition of the residual of the
    operator whose FP64 generators and Cross data T holds, evaluated with the
    same circulant embedding as `Level.matvec` (eq. (ccs3.4)) but with every
    step, the spectra included, in long double.  b and x are FP64 (or long
    double) vectors of T.size entries.  Returns the residual as a long
    double array; its norm relative to ||b|| is the stopping rule's measure
    (Sec. 5) free of FP64's evaluation floor eps |A| |x|.  Pinned against
    50-digit exact dense products at tiny N and against the FP64 FFT matvec
    within that matvec's own error at large N."""
    ld = np.longdouble
    n = T.n
    L = 2 * (n + 1)

    def spec(g):
        g = np.asarray(g, dtype=ld)
        col = np.zeros(L, dtype=ld)
        col[:n] = g[n - 1::-1]
        if n > 1:
            col[L - (n - 1):] = g[n:][::-1]
        return scipy.fft.rfft(col)

    def apply(S, X):
        return scipy.fft.irfft(S * X, n=L)[:n]

    x = np.asarray(x, dtype=ld)
    b = np.asarray(b, dtype=ld)
    v, wo, wb = x[:n], x[n], x[n + 1:]
    V = scipy.fft.rfft(v, n=L)
    W = scipy.fft.rfft(wb, n=L)
    p, q, xi, zeta = (np.asarray(a, dtype=ld) for a in (T.p, T.q, T.xi, T.zeta))
    yv = apply(spec(T.a), V) + apply(spec(T.b), W) + p * wo
    yw = apply(spec(T.c), V) + apply(spec(T.d), W) + xi * wo
    yo = np.dot(q, v) + np.longdouble(T.o) * wo + np.dot(zeta, wb)
    y = np.concatenate([yv, [yo], yw])
    if T.band is not None:
        s_, m_, p_ = (np.asarray(a, dtype=ld) for a in T.band)
        y += m_ * x
        y[1:] += s_[1:] * x[:-1]
        y[:-1] += p_[:-1] * x[1:]
    return b - y


def relres_extended(T: TpX, b, x) -> float:
    """||b - A x||_2 / ||b||_2 with the residual from `residual_extended`."""
    r = residual_extended(T, b, x)
    bl = np.asarray(b, dtype=np.longdouble)
    return float(np.sqrt(np.dot(r, r)) / np.sqrt(np.dot(bl, bl)))


def restrict(r):
    """1/4 [1 2 1] stride 2 on the block-ordered vector (Sec. 3.1)."""
    return 0.25 * (r[0:-2:2] + 2.0 * r[1:-1:2] + r[2::2])


def prolong(e):
    """2 R^T e (Sec. 3.1)."""
    m = 2 * len(e) + 1
    u = np.zeros(m)
    u[0:-2:2] += 0.5 * e
    u[1:-1:2] += e
    u[2::2] += 0.5 * e
    return u


@dataclasses.dataclass
class Hierarchy:
    levels: list
    lu: tuple

    @classmethod
    def build(cls, T_fine: TpX, coarsest_log2: int = 5):
        Ts = [T_fine]
        while Ts[-1].n > 2 ** coarsest_log2 - 1:
            Ts.append(coarsen(Ts[-1]))
        assert Ts[-1].n == 2 ** coarsest_log2 - 1, "N must be 2^K with K >= coarsest_log2"
        levels = [Level.build(T) for T in Ts[:-1]]
        coarsest = Ts[-1]
        return cls(levels + [coarsest], scipy.linalg.lu_factor(coarsest.dense()))

    @property
    def finest(self):
        return self.levels[0]

    def matvec(self, u):
        return self.levels[0].matvec(u)


def vcycle(H: Hierarchy, b, opts: Options = Options(), level: int = 0, x0=None):
    """Algorithm 2 on Toeplitz-plus-Cross levels (same steps as oracle.dense.vcycle).

    opts.cycle = 2 gives the W-cycle: the correction of every level above the
    coarsest is computed by two cycles on the next level, the second starting
    from the first's result (the same right-hand side); the level above the
    coarsest visits the exact solve once.  x0 is the level's initial guess
    (zero when None)."""
    if level == len(H.levels) - 1:
        return scipy.linalg.lu_solve(H.lu, b)
    L = H.levels[level]
    u = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    for _ in range(opts.m1):
        u = u + opts.omega_pre * (b - L.matvec(u)) / L.diag
    rc = restrict(b - L.matvec(u))
    visits = 1 if level + 2 == len(H.levels) else opts.cycle
    e = None
    for _ in range(visits):
        e = vcycle(H, rc, opts, level + 1, e)
    u = u + prolong(e)
    for _ in range(opts.m2):
        u = u + opts.omega_post * (b - L.matvec(u)) / L.diag
    return u


def solve(H: Hierarchy, b, tol=1e-10, max_iter=500, opts: Options = Options(), x0=None):
    """Outer stationary iteration with Sec. 5's stopping rule; returns
    (x, iterations, history)."""
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    r = b - H.matvec(x)
    r0 = np.linalg.norm(r)
    hist = [1.0]
    it = 0
    while hist[-1] >= tol and it < max_iter:
        x = x + vcycle(H, r, opts)
        r = b - H.matvec(x)
        it += 1
        hist.append(np.linalg.norm(r) / r0)
    return x, it, np.array(hist)


def pcg(H: Hierarchy, b, tol=1e-10, max_iter=500, opts: Options = Options(), x0=None,
        precond=None, callback=None):
    """Conjugate gradients for the SPD case, preconditioned by one V-cycle
    (the Krylov acceleration of the V-cycle iteration; the paper's method is
    the stationary iteration of `solve`).  Steps, in this order, per
    iteration: q = A p, alpha = <r, z> / <p, q>, x += alpha p, r -= alpha q,
    stop test on ||r|| / ||r_0||, z = B r, beta in the Polak-Ribiere form
    <z_new, r_new - r_old> / <z_old, r_old> (equal to the Fletcher-Reeves
    ratio for an exactly symmetric preconditioner, and robust when the
    preconditioner is applied in lower precision), p = z + beta p.
    The stopping rule of Sec. 5 is on b - A x; the recurrence's r drifts
    from it on ill-conditioned problems, so when ||r|| passes the test the
    true residual is formed and decides: below tol the solve ends, otherwise
    CG restarts from it (p = z = B r); a true residual not below 0.9 times the
    previous one ends the solve (the FP64 evaluation floor of b - A x).  `precond` replaces the V-cycle (used
    by the pins with the identity); `callback(x)` sees every iterate.
    Returns (x, iterations, history); a history entry that passed the test
    is replaced by the true residual."""
    B = precond if precond is not None else (lambda r: vcycle(H, r, opts))
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    r = b - H.matvec(x)
    r0 = np.linalg.norm(r)
    hist = [1.0]
    if r0 == 0.0:
        return x, 0, np.array(hist)
    it = 0
    restart = True
    prev_true = None
    while it < max_iter:
        if restart:
            z = B(r)
            p = z.copy()
            rz = float(r @ z)
            restart = False
        q = H.matvec(p)
        alpha = rz / float(p @ q)
        x = x + alpha * p
        if callback is not None:
            callback(x)
        r_old = r
        r = r - alpha * q
        it += 1
        hist.append(np.linalg.norm(r) / r0)
        if hist[-1] < tol:
            r = b - H.matvec(x)
            hist[-1] = np.linalg.norm(r) / r0
            if hist[-1] < tol or (prev_true is not None and hist[-1] >= 0.9 * prev_true):
                break
            prev_true = hist[-1]
            restart = True
            continue
        z = B(r)
        rz_new = float(r @ z)
        beta = (rz_new - float(r_old @ z)) / rz
        rz = rz_new
        p = z + beta * p
    return x, it, np.array(hist)


def gmres(H: Hierarchy, b, tol=1e-10, max_iter=500, restart=30, opts: Options = Options(),
          x0=None, precond=None):
    """Restarted flexible GMRES, right-preconditioned (Saad's FGMRES): per
    Arnoldi step j, z_j = B v_j (one V-cycle), w = A z_j, modified Gram-Schmidt
    against v_0..v_j, v_{j+1} = w / h_{j+1,j}; Givens rotations keep the
    Hessenberg matrix triangular and give the residual norm |g_{j+1}| of the
    minimiser over span(z_0..z_j) without forming it.  A cycle ends when that
    estimate is below tol * ||r_0||, after `restart` steps, at max_iter or on
    breakdown (h_{j+1,j} = 0); then x += Z y with y from the triangular
    system, the true residual b - A x is formed, and the solve stops if its
    norm is below tol * ||r_0|| (else the next cycle starts from it).
    Iterations count Arnoldi steps (V-cycles).  The history holds the
    estimates, the last entry of each cycle replaced by the true value.
    Returns (x, iterations, history)."""
    B = precond if precond is not None else (lambda r: vcycle(H, r, opts))
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    r = b - H.matvec(x)
    r0 = np.linalg.norm(r)
    hist = [1.0]
    if r0 == 0.0:
        return x, 0, np.array(hist)
    it = 0
    while True:
        beta = np.linalg.norm(r)
        V = [r / beta]
        Z = []
        Hm = np.zeros((restart + 1, restart))
        g = np.zeros(restart + 1)
        g[0] = beta
        cs, sn = np.zeros(restart), np.zeros(restart)
        k = 0
        for j in range(restart):
            z = B(V[j])
            Z.append(z)
            w = H.matvec(z)
            for i in range(j + 1):
                Hm[i, j] = float(w @ V[i])
                w = w - Hm[i, j] * V[i]
            hn = np.linalg.norm(w)
            Hm[j + 1, j] = hn
            for i in range(j):
                a, c = Hm[i, j], Hm[i + 1, j]
                Hm[i, j] = cs[i] * a + sn[i] * c
                Hm[i + 1, j] = -sn[i] * a + cs[i] * c
            d = np.hypot(Hm[j, j], Hm[j + 1, j])
            cs[j], sn[j] = Hm[j, j] / d, Hm[j + 1, j] / d
            Hm[j, j], Hm[j + 1, j] = d, 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            it += 1
            k = j + 1
            hist.append(abs(g[j + 1]) / r0)
            if hn == 0.0 or hist[-1] < tol or it >= max_iter:
                break
            V.append(w / hn)
        y = scipy.linalg.solve_triangular(Hm[:k, :k], g[:k])
        x = x + np.column_stack(Z) @ y
        r = b - H.matvec(x)
        hist[-1] = np.linalg.norm(r) / r0
        if hist[-1] < tol or it >= max_iter:
            break
    return x, it, np.array(hist)
