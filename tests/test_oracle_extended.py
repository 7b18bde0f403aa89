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
