"""Pins of the oracle's extended-precision residual (tpx.residual_extended,
CPU only): against an exact 50-digit dense product at tiny N, against the
FP64 FFT evaluation within that evaluation's own error at larger N, and its
error far below FP64's floor where that floor exceeds 1e-10."""
import mpmath
import numpy as np
import pytest

import synthetic
from oracle import discretize as D
from oracle import tpx


def _random_tpx(n, seed):
    g = synthetic.rng(seed)
    gen = lambda: g.standard_normal(2 * n - 1)
    vec = lambda: g.standard_normal(n)
    return tpx.TpX(n, gen(), gen(), gen(), gen(), vec(), vec(), vec(), vec(), float(g.standard_normal()))


def _exact_residual(M, b, x):
    """b - M x with 50-digit sums of the FP64 entries (exact to 1e-50)."""
    mpmath.mp.dps = 50
    out = []
    for i in range(M.shape[0]):
        acc = mpmath.mpf(b[i])
        for j in range(M.shape[1]):
            acc -= mpmath.mpf(M[i, j]) * mpmath.mpf(x[j])
        out.append(acc)
    return out


@pytest.mark.parametrize("n,kind", [(7, "random"), (15, "random"), (31, "frac"), (63, "weighted")])
def test_extended_residual_equals_exact_dense(n, kind):
    """At tiny N the extended residual equals the exact residual of the dense
    level matrix (50-digit mpmath sums of the same FP64 entries) to a few
    units of long double roundoff times the entries' scale; a transposed
    block (B and C swapped) is caught."""
    N = n + 1
    if kind == "random":
        T = _random_tpx(n, seed=n)
    elif kind == "frac":
        T = tpx.from_stencil(D.Kernel(D.FRACTIONAL, 0.1, alpha=0.4), N)
    else:
        T = tpx.from_stencil(D.Kernel(D.WEIGHTED, 0.25, wl=1.2, wr=0.8), N)
    M = T.dense()
    x = synthetic.random_vector(2 * n + 1, seed=100 + n)
    b = M @ x + 1e-3 * synthetic.random_vector(2 * n + 1, seed=200 + n)
    ex = _exact_residual(M, b, x)
    r = tpx.residual_extended(T, b, x)
    scale = float(np.abs(M).sum(axis=1).max() * np.abs(x).max())
    err = max(abs(float(mpmath.mpf(str(r[i])) - ex[i])) for i in range(len(ex))) / scale
    assert err < 1e-17, err
    if kind != "frac":  # non-symmetric levels: swapping B and C changes A
        Tw = tpx.TpX(T.n, T.a, T.c, T.b, T.d, T.p, T.q, T.xi, T.zeta, T.o)
        rw = tpx.residual_extended(Tw, b, x)
        errw = max(abs(float(mpmath.mpf(str(rw[i])) - ex[i])) for i in range(len(ex))) / scale
        assert errw > 1e-3


@pytest.mark.parametrize("kern,N", [(D.Kernel(D.CONST, 0.25), 2 ** 12), (D.Kernel(D.WEIGHTED, 0.05, wl=1.2, wr=0.8), 2 ** 13),
                                    (D.Kernel(D.FRACTIONAL, 0.1, alpha=0.4), 2 ** 14)], ids=lambda k: getattr(k, "kind", k))
def test_extended_residual_within_fp64_error(kern, N):
    """The FP64 FFT evaluation differs from the extended one by no more than
    FP64's error bound for it, c eps_64 log2 L |G|_inf |x|_2 (|G|_inf the
    largest spectrum value), and the two agree to 5e-14 of |b| for the
    constant and weighted kernels (1.1e-15 and 1.0e-14 measured)."""
    T = tpx.from_stencil(kern, N)
    Lv = tpx.Level.build(T)
    x = D.u_exact(D.points_block(N)) + 1e-3 * synthetic.random_vector(2 * N - 1, seed=1)
    b = D.rhs_manufactured(kern, N)
    r64 = b - Lv.matvec(x)
    rex = tpx.residual_extended(T, b, x).astype(np.float64)
    G = max(np.abs(s).max() for s in (Lv.sA, Lv.sB, Lv.sC, Lv.sD))
    bound = 8 * np.finfo(float).eps * np.log2(2 * N) * G * np.linalg.norm(x)
    assert np.linalg.norm(r64 - rex) <= bound
    if kern.kind != D.FRACTIONAL:
        assert np.linalg.norm(r64 - rex) <= 5e-14 * np.linalg.norm(b)


def test_extended_residual_below_fp64_floor():
    """Fractional kernel (alpha = 0.4) at N = 2^16: the FP64 FFT evaluation of
    b - A x for the smooth x = u is off by about 1e-10 |b| (eps |A| |x|);
    the extended evaluation is consistent with itself to long double
    accuracy (eps_ld |A| |x| ~ 5e-14 |b| here): evaluating with x split as
    x1 + x2 (linearity) changes it by less than 1e-12 |b|, a thousandth of
    the FP64 evaluation's error."""
    kern, N = D.Kernel(D.FRACTIONAL, 0.1, alpha=0.4), 2 ** 16
    T = tpx.from_stencil(kern, N)
    x = D.u_exact(D.points_block(N))
    b = D.rhs_manufactured(kern, N)
    nb = np.linalg.norm(b)
    rex = tpx.residual_extended(T, b, x)
    r64 = b - tpx.Level.build(T).matvec(x)
    gap64 = np.linalg.norm(r64 - rex.astype(np.float64))
    assert gap64 > 1e-11 * nb
    x1 = np.round(x, 6)
    x2 = x - x1
    z = np.zeros_like(b)
    lin = rex - (tpx.residual_extended(T, b, x1) + tpx.residual_extended(T, z, x2))
    d = float(np.sqrt(np.dot(lin, lin)))
    assert d < 1e-12 * nb and d < 1e-3 * gap64


@pytest.mark.parametrize("kern", [D.Kernel(D.FRACTIONAL, 0.1, alpha=0.4), D.Kernel(D.CONST, 0.05),
                                  D.Kernel(D.WEIGHTED, 0.05, wl=1.2, wr=0.8),
                                  D.Kernel(D.FRACTIONAL, 0.013, alpha=0.2)], ids=lambda k: k.kind)
def test_rowsum_diagonal_equals_integral_diagonal(kern):
    """from_stencil_rowsum: the own-point weight -sum_{k != 0} W(k) (partition
    of unity) equals the integral formula's int gamma (1 - l_0) to a few FP64
    units of it, every other entry is the FP64 level's exactly, and interior
    rows of the matrix sum to zero to long double accuracy."""
    for N in (2 ** 8, 2 ** 12, 2 ** 15):
        T = tpx.from_stencil(kern, N)
        Tr = tpx.from_stencil_rowsum(kern, N)
        n = N - 1
        for g, gr in ((T.a, Tr.a), (T.d, Tr.d)):
            assert abs(float(gr[n - 1]) - g[n - 1]) <= 16 * np.spacing(abs(g[n - 1]))
            off = np.r_[0:n - 1, n:2 * n - 1]
            np.testing.assert_array_equal(gr[off].astype(np.float64), g[off])
        for g, gr in ((T.b, Tr.b), (T.c, Tr.c), (T.p, Tr.p), (T.xi, Tr.xi)):
            np.testing.assert_array_equal(gr.astype(np.float64), g)
        assert abs(float(Tr.o) - T.o) <= 16 * np.spacing(abs(T.o))
        # a node row in the middle of the interval: its whole stencil is inside
        M = np.zeros(2 * n + 1, dtype=np.longdouble)
        i = n // 2
        row = np.concatenate([Tr.a[n - 1 - i:2 * n - 1 - i], [Tr.p[i]], Tr.b[n - 1 - i:2 * n - 1 - i]])
        tot = float(row.sum())
        assert abs(tot) <= 64 * np.finfo(np.longdouble).eps * float(np.abs(row).sum()), tot


def test_rowsum_level_exact_dense():
    """The extended residual of the row-sum level equals the exact 50-digit
    residual of that level's long double entries (tiny N)."""
    n, N = 31, 32
    Tr = tpx.from_stencil_rowsum(D.Kernel(D.FRACTIONAL, 0.1, alpha=0.4), N)
    mpmath.mp.dps = 50
    Md = tpx.TpX(n, *(np.asarray(getattr(Tr, f), dtype=np.float64) for f in
                      ("a", "b", "c", "d", "p", "q", "xi", "zeta")), float(Tr.o)).dense()
    x = synthetic.random_vector(2 * n + 1, seed=3)
    b = Md @ x
    r = tpx.residual_extended(Tr, b, x)
    # exact residual of the long double matrix: entries as mpmath numbers
    def ent(i, j):
        if i < n and j < n:
            return Tr.a[j - i + n - 1]
        if i < n and j == n:
            return Tr.p[i]
        if i < n:
            return Tr.b[(j - n - 1) - i + n - 1]
        if i == n and j < n:
            return Tr.q[j]
        if i == n and j == n:
            return Tr.o
        if i == n:
            return Tr.zeta[j - n - 1]
        if j < n:
            return Tr.c[j - (i - n - 1) + n - 1]
        if j == n:
            return Tr.xi[i - n - 1]
        return Tr.d[(j - n - 1) - (i - n - 1) + n - 1]
    scale = float(np.abs(Md).sum(axis=1).max() * np.abs(x).max())
    for i in range(2 * n + 1):
        acc = mpmath.mpf(b[i])
        for j in range(2 * n + 1):
            acc -= mpmath.mpf(str(ent(i, j))) * mpmath.mpf(x[j])
        assert abs(float(mpmath.mpf(str(r[i])) - acc)) <= 1e-17 * scale, i
