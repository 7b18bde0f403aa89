"""Pins of the oracle's standard (unshifted) collocation and of volume data
(Sec. 2.2.1, eq. (ccs2.6), eq. (nonsym system), eqs. (rightside1),
(rightside2)).  CPU only."""
import numpy as np
import pytest

from oracle import discretize as D
from oracle import tpx


@pytest.mark.parametrize("r", [2, 3, 5, 8])
def test_standard_midpoint_rows_printed_integers(r):
    """delta = r h, constant kernel: the midpoint-row coefficients in units of
    c h / 6 are the integers printed after eq. (nonsym system):
    d_0 = 12 r - 4, d_m = -4 (1 <= m <= r-1), d_r = -2 (midpoints at offset
    m h); c_m = -2 (0 <= m <= r-2), c_{r-1} = -9/4, c_r = 1/4 (nodes at offset
    (m + 1/2) h), the same on both sides; nothing beyond."""
    N = 64
    k = D.Kernel(D.CONST, r / N)
    W, S = D.midpoint_stencil_standard(k, N)
    w = W / (k.c / N / 6.0)
    d = [12 * r - 4] + [-4] * (r - 1) + [-2]
    c = [-2] * (r - 1) + [-9 / 4, 1 / 4]
    for m in range(r + 1):
        assert w[S + 2 * m] == pytest.approx(d[m], abs=1e-10)
        assert w[S - 2 * m] == pytest.approx(d[m], abs=1e-10)
        assert w[S + 2 * m + 1] == pytest.approx(c[m], abs=1e-10)
        assert w[S - 2 * m - 1] == pytest.approx(c[m], abs=1e-10)
    assert np.all(w[: S - 2 * r - 1] == 0) and np.all(w[S + 2 * r + 2:] == 0)


@pytest.mark.parametrize("scheme", [D.STANDARD, D.SHIFTED])
@pytest.mark.parametrize("kern", [D.Kernel(D.CONST, 0.1), D.Kernel(D.CONST, 0.25),
                                  D.Kernel(D.WEIGHTED, 0.1, wl=1.2, wr=0.8),
                                  D.Kernel(D.CONST, 0.01)], ids=lambda k: f"{k.kind}-{k.delta}")
def test_exact_on_quadratics_with_volume_data(scheme, kern):
    """u_Q = u for quadratics, so with the exterior points carried as volume
    data, A u + E g = -L_delta u exactly on every row: 0 for u = 1, -m1 for
    u = x, -2 x m1 - m2 for u = x^2 (m_j = int gamma t^j)."""
    N = 32
    A, E, q = D.assemble_with_exterior(kern, N, scheme)
    x = D.points_block(N)
    xe = q / (2.0 * N)
    wl, wr = kern.side_weights()
    d = kern.delta
    m1 = kern.c * (wr - wl) * d ** 2 / 2
    m2 = kern.c * (wr + wl) * d ** 3 / 3
    for u, f in ((lambda t: np.ones_like(t), lambda t: np.zeros_like(t)),
                 (lambda t: t, lambda t: -m1 * np.ones_like(t)),
                 (lambda t: t * t, lambda t: -2 * t * m1 - m2)):
        lhs = A @ u(x) + E @ u(xe)
        assert np.abs(lhs - f(x)).max() <= 1e-11 * max(1.0, np.abs(A).max())


def test_volume_data_fourth_order():
    """Manufactured u = (1+x)^6 with g = u on the interaction volume (non-zero
    volume data): the discrete solution of A U = f - E g converges to u at
    fourth order for both schemes (the paper's truncation-error order for a
    fixed horizon)."""
    for scheme, kern in ((D.STANDARD, D.Kernel(D.CONST, 0.25)), (D.SHIFTED, D.Kernel(D.CONST, 0.25)),
                         (D.STANDARD, D.Kernel(D.WEIGHTED, 0.1, wl=1.2, wr=0.8))):
        errs = []
        for N in (16, 32, 64, 128):
            A, E, q = D.assemble_with_exterior(kern, N, scheme)
            x = D.points_block(N)
            U = np.linalg.solve(A, D.f_poly6(kern, x) - E @ D.u_poly6(q / (2.0 * N)))
            errs.append(np.abs(U - D.u_poly6(x)).max())
        rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
        assert rates.mean() > 3.6 and errs[-1] < 5e-7, (scheme, kern.kind, errs)


def test_standard_tpx_level_and_vcycle():
    """The Toeplitz-plus-Cross finest level built from the two stencils equals
    the dense standard-scheme matrix (non-symmetric), and the stationary
    V-cycle iteration solves it (the paper's non-symmetric experiments)."""
    kern = D.Kernel(D.CONST, 0.25)
    N = 128
    A, E, q = D.assemble_with_exterior(kern, N, D.STANDARD)
    T = tpx.from_stencil(kern, N, D.STANDARD)
    assert np.array_equal(T.dense(), A)
    assert np.abs(A - A.T).max() > 0.1
    H = tpx.Hierarchy.build(T, 5)
    b = D.f_poly6(kern, D.points_block(N)) - E @ D.u_poly6(q / (2.0 * N))
    x, it, hist = tpx.solve(H, b, tol=1e-10, max_iter=100)
    assert hist[-1] < 1e-10 and it <= 15
    assert np.abs(x - np.linalg.solve(A, b)).max() <= 1e-8 * np.abs(x).max()


@pytest.mark.parametrize("scheme", [D.STANDARD, D.SHIFTED])
def test_volume_correction_rows_equal_dense_exterior(scheme):
    """The row-by-row volume correction equals the dense exterior block times
    g (same stencils, two ways of summing)."""
    kern = D.Kernel(D.WEIGHTED, 0.1, wl=1.2, wr=0.8)
    N = 64
    A, E, q = D.assemble_with_exterior(kern, N, scheme)
    S = D.volume_reach(kern, N, scheme)
    gl = D.u_poly6(-np.arange(S + 1) / (2.0 * N))
    gr = D.u_poly6(1.0 + np.arange(S + 1) / (2.0 * N))
    ge = D.u_poly6(q / (2.0 * N))
    np.testing.assert_allclose(D.volume_correction(kern, N, gl, gr, scheme), E @ ge,
                               rtol=1e-13, atol=1e-12 * np.abs(E).max())
