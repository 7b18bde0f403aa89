"""Pins of the oracle's collocation system against what the paper and the
mathematics fix (CPU only)."""
import math

import mpmath
import numpy as np
import pytest

from oracle import discretize as D

H_KINDS = [
    D.Kernel(D.CONST, 0.25),
    D.Kernel(D.CONST, 0.05),
    D.Kernel(D.WEIGHTED, 0.1, wl=1.2, wr=0.8),
    D.Kernel(D.WEIGHTED, 0.05, wl=1.2, wr=0.8),
    D.Kernel(D.FRACTIONAL, 0.1, alpha=0.4),
    D.Kernel(D.FRACTIONAL, 0.13, alpha=0.2),
]


@pytest.mark.parametrize("N,r", [(16, 1), (16, 2), (32, 5), (64, 8), (128, 32), (256, 9)])
def test_printed_integer_coefficients(N, r):
    """Sec. 2.2.2 (coefficients after eq. (system1)), delta = r h, constant
    kernel: in units of c h / 6 the stencil is a_0 = 12r-2, a_m = -2
    (1 <= m <= r-1), a_r = -1, a_{m+1/2} = -4 (0 <= m <= r-1)."""
    k = D.Kernel(D.CONST, r / N)
    W, S = D.stencil(k, N)
    unit = k.c * (1.0 / N) / 6.0
    got = W / unit
    want = np.zeros_like(got)
    want[S] = 12 * r - 2
    for m in range(1, r + 1):
        want[S + 2 * m] = want[S - 2 * m] = -1.0 if m == r else -2.0
    for m in range(r):
        want[S + 2 * m + 1] = want[S - 2 * m - 1] = -4.0
    assert S == 2 * r
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-12 * (12 * r))


@pytest.mark.parametrize("kern", H_KINDS, ids=lambda k: f"{k.kind}-{k.delta}")
def test_row_sum_identity(kern):
    """Lemma 4.1: a_0 + 2 sum a_m + 2 sum a_{m+1/2} = 0 (constants are in
    the kernel of -L_delta; holds for every kernel)."""
    for N in (32, 64, 128):
        W, _ = D.stencil(kern, N)
        assert abs(W.sum()) <= 1e-12 * np.abs(W).sum()


@pytest.mark.parametrize("kern", H_KINDS, ids=lambda k: f"{k.kind}-{k.delta}")
def test_exact_on_quadratics(kern):
    """u_Q = u for quadratics (eq. (ccs2.1)), so on rows whose horizon stays in
    (0,1): A 1 = 0, A x = -m1, A x^2 = -2 x m1 - m2, m_j = int gamma s^j ds;
    m2 = 1 by the normalisation, m1 = c (wr - wl) delta^2 / 2."""
    N = 64
    h = 1.0 / N
    A = D.assemble_dense(kern, N)
    x = D.points_block(N)
    inside = (x - kern.delta > 1.5 * h) & (x + kern.delta < 1 - 1.5 * h)
    assert inside.sum() > 10
    wl, wr = kern.side_weights()
    m1 = kern.c * (wr - wl) * kern.delta ** 2 / 2 if kern.kind != D.FRACTIONAL else 0.0
    scale = np.abs(A).sum(axis=1).max()
    np.testing.assert_allclose((A @ np.ones_like(x))[inside], 0.0, atol=1e-13 * scale)
    np.testing.assert_allclose((A @ x)[inside], -m1, atol=1e-13 * scale)
    np.testing.assert_allclose((A @ x ** 2)[inside], -2 * x[inside] * m1 - 1.0,
                               atol=1e-12 * scale)


@pytest.mark.parametrize("alpha,delta,N", [(0.4, 0.1, 64), (0.2, 0.13, 64),
                                           (0.45, 0.3, 16), (0.3, 0.02, 2048)])
def test_fractional_moments_vs_quadrature(alpha, delta, N):
    """Cell moments int_0^theta (k+tau)^beta tau^j dtau against 30-digit
    tanh-sinh quadrature (independent of the closed form / series); on the
    singular cell k = 0 the substitution tau = theta s^10 removes the endpoint
    singularity before quadrature."""
    k = D.Kernel(D.FRACTIONAL, delta, alpha=alpha)
    kk, theta = D.cells(k, N)
    J = D._frac_moments(kk, theta, k.beta)
    mpmath.mp.dps = 30
    picks = sorted(set([0, 1, 2, 3, len(kk) // 2, len(kk) - 2, len(kk) - 1]) & set(range(len(kk))))
    for i in picks:
        for j in (0, 1, 2):
            if kk[i] == 0 and j == 0:
                continue
            ki, th, be = int(kk[i]), mpmath.mpf(float(theta[i])), mpmath.mpf(k.beta)
            m = 10 if ki == 0 else 1  # t = th s^m smooths the t^(beta+j) endpoint
            ref = mpmath.quad(lambda s: (ki + th * s ** m) ** be * (th * s ** m) ** j
                              * th * m * s ** (m - 1), [0, 1])
            assert abs(J[j, i] - float(ref)) <= 2e-15 * abs(float(ref)), (i, j)


@pytest.mark.parametrize("kern", [H_KINDS[0], H_KINDS[1], H_KINDS[4]],
                         ids=lambda k: f"{k.kind}-{k.delta}")
def test_symmetric_positive_definite(kern):
    """Lemma 4.2: the shifted-symmetric system is SPD (constant kernel); the
    fractional kernel gives a symmetric matrix, SPD as checked numerically."""
    for N in (32, 128):
        A = D.assemble_dense(kern, N)
        np.testing.assert_allclose(A, A.T, rtol=0, atol=1e-14 * np.abs(A).max())
        assert np.linalg.eigvalsh(A).min() > 0


def test_constant_kernel_m_matrix_and_jacobi_bound():
    """Lemma 4.1 (nonpositive off-diagonals, positive diagonal) and Lemma 4.6:
    lambda_max(D^-1 A) in [1, 2] for the constant kernel with delta = r h (the
    paper's setting; a partial last cell makes a few off-diagonals positive)."""
    for delta, N in ((0.25, 32), (0.25, 128), (0.3125, 32), (0.0625, 128), (1 / 32, 32)):
        if True:
            A = D.assemble_dense(D.Kernel(D.CONST, delta), N)
            off = A - np.diag(np.diag(A))
            assert off.max() <= 1e-15 * A.max()
            dinv = 1.0 / np.sqrt(np.diag(A))
            lam = np.linalg.eigvalsh(dinv[:, None] * A * dinv[None, :]).max()
            assert 1.0 <= lam <= 2.0


def _f_quadrature(kern, x):
    """f(x) = int gamma(t)(u(x) - u~(x+t)) dt by 30-digit mpmath quadrature.

    Where x + t stays in (0,1), u(x) - u(x+t) is written as the polynomial
    -sum_p c_p t^p with c_p from mpmath.taylor (exact for the quartic u), so the
    integrand has no cancellation near t = 0; pieces that end at t = 0 are
    mapped by t = t_end s^10 to smooth the |t|^beta singularity.  Where
    x + t leaves (0,1) the integrand is gamma(t) u(x).
    """
    mpmath.mp.dps = 30
    x = mpmath.mpf(float(x))
    u = lambda y: y * y * (1 - y) ** 2
    cp = mpmath.taylor(u, x, 4)
    wl, wr = kern.side_weights()
    d = mpmath.mpf(kern.delta)
    be = mpmath.mpf(kern.beta)
    c = mpmath.mpf(kern.c)

    def g(t):
        base = c * (abs(t) ** be if kern.kind == D.FRACTIONAL else 1)
        return base * (wl if t < 0 else wr)

    inside = lambda t: -g(t) * sum(cp[p] * t ** p for p in range(1, 5))
    outside = lambda t: g(t) * u(x)
    total = mpmath.mpf(0)
    for sign in (1, -1):
        edge = (1 - x) if sign > 0 else x      # distance to the boundary
        b_in = min(edge, d)
        m = 10
        total += mpmath.quad(lambda s: inside(sign * b_in * s ** m) * b_in * m * s ** (m - 1), [0, 1])
        if edge < d:
            total += mpmath.quad(lambda t: outside(sign * t), [edge, d])
    return float(total)


@pytest.mark.parametrize("kern", H_KINDS, ids=lambda k: f"{k.kind}-{k.delta}")
def test_manufactured_rhs_vs_quadrature(kern):
    N = 32
    f = D.rhs_manufactured(kern, N)
    x = D.points_block(N)
    for i in (0, 3, N - 2, N - 1, N + 5, 2 * N - 2, N // 2):
        ref = _f_quadrature(kern, float(x[i]))
        assert abs(f[i] - ref) <= 1e-11 * max(1.0, abs(ref)), (i, f[i], ref)


def test_manufactured_error_falls_fourth_order():
    """delta fixed: the collocation error of u = x^2(1-x)^2 falls about like
    h^4 (Table TT01 reports rates near 4 for delta = 1/4)."""
    errs = []
    for N in (32, 64, 128, 256):
        k = D.Kernel(D.CONST, 0.25)
        U = np.linalg.solve(D.assemble_dense(k, N), D.rhs_manufactured(k, N))
        errs.append(np.abs(U - D.u_exact(D.points_block(N))).max())
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(3)]
    assert all(3.5 < r < 4.5 for r in rates), (errs, rates)


@pytest.mark.parametrize("kern", [D.Kernel(D.CONST, 0.05), D.Kernel(D.FRACTIONAL, 0.1, alpha=0.4),
                                  D.Kernel(D.WEIGHTED, 0.05, wl=1.2, wr=0.8)],
                         ids=lambda k: k.kind)
def test_partial_interval_convergence(kern):
    """delta/h not an integer: with the partial cell [r h, delta] integrated
    the error keeps falling as N grows (no O(1) floor)."""
    errs = []
    for N in (64, 128, 256, 512):
        U = np.linalg.solve(D.assemble_dense(kern, N), D.rhs_manufactured(kern, N))
        errs.append(np.abs(U - D.u_exact(D.points_block(N))).max())
    assert errs[-1] < errs[0] / 20, errs
    assert all(errs[i + 1] < errs[i] for i in range(3)), errs


def test_delta_below_h():
    """delta < h: the horizon is a fraction of the first cell; the rules above
    still hold (row sums, quadratics)."""
    N = 16
    k = D.Kernel(D.CONST, 0.4 / N)
    W, S = D.stencil(k, N)
    assert S == 2 and abs(W.sum()) < 1e-12 * np.abs(W).sum()
    m2 = sum(W[s + S] * (-(s / (2 * N)) ** 2) for s in range(-S, S + 1))
    assert abs(m2 - 1.0) < 1e-12


# --- the fractional_near kernel (an extension for 0 < alpha < 1, not in the
# paper): symmetric quadratic on |t| <= h/2, product integration beyond ------

H_NEAR = [
    D.Kernel(D.FRACTIONAL_NEAR, 0.1, alpha=0.3),
    D.Kernel(D.FRACTIONAL_NEAR, 0.1, alpha=0.5),
    D.Kernel(D.FRACTIONAL_NEAR, 0.13, alpha=0.7),
    D.Kernel(D.FRACTIONAL_NEAR, 0.05, alpha=0.9),
]
NEAR_IDS = lambda k: f"a{k.alpha}-d{k.delta}"


@pytest.mark.parametrize("kern", H_NEAR, ids=NEAR_IDS)
def test_near_rule_row_sum_and_quadratics(kern):
    """Both pieces of the rule reproduce quadratics, so on rows whose horizon
    stays in (0,1): A 1 = 0, A x = 0 (symmetric kernel), A x^2 = -int gamma
    s^2 = -1; and the stencil's row sum is zero."""
    for N in (32, 64, 128):
        W, _ = D.stencil(kern, N)
        assert abs(W.sum()) <= 1e-12 * np.abs(W).sum()
    N = 64
    h = 1.0 / N
    A = D.assemble_dense(kern, N)
    x = D.points_block(N)
    inside = (x - kern.delta > 1.5 * h) & (x + kern.delta < 1 - 1.5 * h)
    assert inside.sum() > 10
    scale = np.abs(A).sum(axis=1).max()
    np.testing.assert_allclose((A @ np.ones_like(x))[inside], 0.0, atol=1e-13 * scale)
    np.testing.assert_allclose((A @ x)[inside], 0.0, atol=1e-13 * scale)
    np.testing.assert_allclose((A @ x ** 2)[inside], -1.0, atol=1e-12 * scale)


@pytest.mark.parametrize("kern", H_NEAR, ids=NEAR_IDS)
def test_near_rule_pieces_vs_quadrature(kern):
    """The near weight m = (4/h^2) int_0^{h/2} gamma t^2 dt and the far
    moments of cell 0, int_{h/2}^{h} gamma (t/h)^j dt, against 30-digit
    quadrature of their definitions (t = (h/2) s^10 smooths the t^(beta+2)
    endpoint of the first)."""
    mpmath.mp.dps = 30
    N = 64
    h = mpmath.mpf(1) / N
    c, be = mpmath.mpf(kern.c), mpmath.mpf(kern.beta)
    m, F0, F1, F2 = D.near_field_rule(kern, N)
    e = h / 2
    ref_m = 4 / h ** 2 * mpmath.quad(
        lambda s: c * (e * s ** 10) ** (be + 2) * e * 10 * s ** 9, [0, 1])
    assert abs(m - float(ref_m)) <= 1e-14 * abs(float(ref_m))
    for j, F in enumerate((F0, F1, F2)):
        ref = mpmath.quad(lambda t: c * t ** be * (t / h) ** j, [h / 2, h])
        assert abs(F - float(ref)) <= 1e-14 * abs(float(ref)), j


@pytest.mark.parametrize("kern", H_NEAR, ids=NEAR_IDS)
def test_near_rule_symmetric_positive_definite(kern):
    for N in (32, 128):
        A = D.assemble_dense(kern, N)
        np.testing.assert_allclose(A, A.T, rtol=0, atol=1e-14 * np.abs(A).max())
        assert np.linalg.eigvalsh(A).min() > 0


def _f_quadrature_pv(kern, x):
    """f(x) = p.v. int gamma(t)(u(x) - u~(x+t)) dt by 30-digit quadrature,
    for a symmetric kernel with |t|^beta, beta <= -2 allowed: on [-a, a]
    (a = the shorter inside reach) the odd Taylor terms of u(x) - u(x+t)
    cancel, leaving 2 sum over even p of c_p int_0^a gamma t^p (t = a s^10
    smooths its endpoint); the rest of the longer side and the outside parts
    are regular."""
    mpmath.mp.dps = 30
    x = mpmath.mpf(float(x))
    u = lambda y: y * y * (1 - y) ** 2
    cp = mpmath.taylor(u, x, 4)
    d, be, c = mpmath.mpf(kern.delta), mpmath.mpf(kern.beta), mpmath.mpf(kern.c)
    g = lambda t: c * abs(t) ** be
    poly = lambda t: sum(cp[p] * t ** p for p in range(1, 5))
    r_in, l_in = min(1 - x, d), min(x, d)
    a = min(r_in, l_in)
    even = lambda t: g(t) * (cp[2] * t ** 2 + cp[4] * t ** 4)
    total = -2 * mpmath.quad(lambda s: even(a * s ** 10) * a * 10 * s ** 9, [0, 1])
    if r_in > a:
        total += mpmath.quad(lambda t: -g(t) * poly(t), [a, r_in])
    if l_in > a:
        total += mpmath.quad(lambda t: -g(t) * poly(-t), [a, l_in])
    for edge in (1 - x, x):
        if edge < d:
            total += mpmath.quad(lambda t: g(t) * u(x), [edge, d])
    return float(total)


@pytest.mark.parametrize("kern", H_NEAR, ids=NEAR_IDS)
def test_near_manufactured_rhs_vs_quadrature(kern):
    N = 32
    f = D.rhs_manufactured(kern, N)
    x = D.points_block(N)
    for i in (0, 3, N - 2, N - 1, N + 5, 2 * N - 2, N // 2):
        ref = _f_quadrature_pv(kern, float(x[i]))
        assert abs(f[i] - ref) <= 1e-10 * max(1.0, abs(ref)), (i, f[i], ref)


@pytest.mark.parametrize("alpha", [0.7, 0.9])
def test_near_manufactured_error_falls(alpha):
    """The collocation error of u = x^2(1-x)^2 falls at least like h^2 (the
    near quadratic is exact to O(h^3) on |t| <= h/2)."""
    k = D.Kernel(D.FRACTIONAL_NEAR, 0.1, alpha=alpha)
    errs = []
    for N in (32, 64, 128, 256):
        U = np.linalg.solve(D.assemble_dense(k, N), D.rhs_manufactured(k, N))
        errs.append(np.abs(U - D.u_exact(D.points_block(N))).max())
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(3)]
    assert all(r > 1.8 for r in rates), (errs, rates)


def test_near_rule_delta_below_half_h():
    """delta < h/2: the near quadratic covers the whole horizon (no far
    part); the row sum vanishes and the second moment is still 1."""
    N = 16
    k = D.Kernel(D.FRACTIONAL_NEAR, 0.4 / N, alpha=0.7)
    W, S = D.stencil(k, N)
    assert S == 2 and W[0] == 0.0 and W[-1] == 0.0
    assert abs(W.sum()) < 1e-12 * np.abs(W).sum()
    m2 = sum(W[s + S] * (-(s / (2 * N)) ** 2) for s in range(-S, S + 1))
    assert abs(m2 - 1.0) < 1e-12


def test_product_integration_refuses_alpha_from_one_half():
    """The plain fractional rule's weights diverge from alpha = 1/2 on; the
    oracle refuses it (as the library returns AMG_EINVAL) instead of
    producing non-finite weights."""
    for a in (0.5, 0.7):
        with pytest.raises(ValueError):
            D.stencil(D.Kernel(D.FRACTIONAL, 0.1, alpha=a), 32)
        with pytest.raises(ValueError):
            D.assemble_dense(D.Kernel(D.FRACTIONAL, 0.1, alpha=a), 32)
    W, _ = D.stencil(D.Kernel(D.FRACTIONAL_NEAR, 0.1, alpha=0.7), 32)
    assert np.all(np.isfinite(W))
