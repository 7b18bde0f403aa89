"""Pins of the oracle's multigrid (dense and Toeplitz-plus-Cross) against the
paper's worked example, its theorem and plain linear algebra (CPU only)."""
import os

import numpy as np
import pytest
import scipy.linalg

import synthetic
from oracle import dense, discretize as D, tpx

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_example1_exact():
    """Example 1 (Sec. 3.2.2): A = I_7, D = I_8, B, C all ones.  The printed
    coarse matrix (times 8) equals R A P for the plain 1/4[1 2 1] restriction on
    the block-ordered vector, and Lemma 3.1's recurrences reproduce it."""
    M = np.block([[np.eye(7), np.ones((7, 8))], [np.ones((8, 7)), np.eye(8)]])
    G = np.loadtxt(os.path.join(GOLDEN, "example1_coarse_times8.txt"))
    R, P = dense.restriction(15), dense.prolongation(15)
    np.testing.assert_array_equal(8 * R @ M @ P, G)
    np.testing.assert_array_equal(8 * tpx.coarsen(tpx.from_dense(M)).dense(), G)


def _random_tpx(n, seed):
    g = synthetic.rng(seed)
    gen = lambda: g.standard_normal(2 * n - 1)
    vec = lambda: g.standard_normal(n)
    return tpx.TpX(n, gen(), gen(), gen(), gen(), vec(), vec(), vec(), vec(), float(g.standard_normal()))


@pytest.mark.parametrize("n", [7, 15, 63, 255])
def test_lemma31_equals_dense_galerkin(n):
    """Lemma 3.1 (N_k = number of intervals) equals R A P for a general
    non-symmetric Toeplitz-plus-Cross level, and the coarse blocks are
    Toeplitz again."""
    T = _random_tpx(n, seed=n)
    M = T.dense()
    Mc = dense.restriction(2 * n + 1) @ M @ dense.prolongation(2 * n + 1)
    Tc = tpx.coarsen(T)
    np.testing.assert_allclose(Tc.dense(), Mc, rtol=0, atol=1e-13 * np.abs(Mc).max())
    nc = Tc.n
    for blk in (Mc[:nc, :nc], Mc[:nc, nc + 1:], Mc[nc + 1:, :nc], Mc[nc + 1:, nc + 1:]):
        for d in range(-(nc - 1), nc):
            diag = np.diagonal(blk, d)
            assert np.ptp(diag) <= 1e-13 * np.abs(Mc).max()


@pytest.mark.parametrize("k", range(3, 12))
def test_fft_matvec_equals_dense(k):
    """Circulant embedding (eq. (ccs3.4)) + Cross terms equals the dense
    product, sizes 2^k - 1 up to k = 11."""
    n = 2 ** k - 1
    T = _random_tpx(n, seed=100 + k)
    u = synthetic.random_vector(2 * n + 1, seed=k)
    y = tpx.Level.build(T).matvec(u)
    yd = T.dense() @ u
    assert np.abs(y - yd).max() <= 1e-13 * np.abs(yd).max() * max(1, k / 4)


def test_finest_from_blocks_matches_dense_blocks():
    N = 64
    gA, gB, gC, gD = synthetic.random_tpx_arrays(N - 1, seed=3)
    M = D.assemble_dense_from_blocks(gA, gB, gC, gD, N)
    np.testing.assert_array_equal(tpx.from_blocks(gA, gB, gC, gD, N).dense(), M)


@pytest.mark.parametrize("kern", [D.Kernel(D.CONST, 0.25), D.Kernel(D.WEIGHTED, 0.05, wl=1.2, wr=0.8),
                                  D.Kernel(D.FRACTIONAL, 0.1, alpha=0.4)], ids=lambda k: k.kind)
def test_stencil_levels_match_dense(kern):
    """Finest TpX from the stencil equals the dense assembly; every Galerkin
    level from Lemma 3.1 equals the dense R A P."""
    N = 256
    A = D.assemble_dense(kern, N)
    H = dense.build_hierarchy(A, 5)
    Ht = tpx.Hierarchy.build(tpx.from_stencil(kern, N), 5)
    for l in range(H.nlevels - 1):
        Tl = Ht.levels[l].T
        np.testing.assert_allclose(Tl.dense(), H.A[l], rtol=0, atol=1e-13 * np.abs(H.A[l]).max())
    np.testing.assert_allclose(Ht.levels[-1].dense(), H.A[-1], rtol=0,
                               atol=1e-13 * np.abs(H.A[-1]).max())


@pytest.mark.parametrize("omega", [0.5, 2.0 / 3.0, 1.0])
def test_two_grid_bound_theorem41(omega):
    """Theorem 4.1: ||S_K T_K||_A <= sqrt(47/48) for the SPD system, omega in
    (0, 1]; the factor also does not grow with N."""
    bound = np.sqrt(47.0 / 48.0)
    rhos = []
    for N in (16, 32, 64, 128):
        A = D.assemble_dense(D.Kernel(D.CONST, 0.25), N)
        rhos.append(dense.energy_norm(dense.two_grid_error_operator(A, omega), A))
    assert max(rhos) <= bound
    assert all(rhos[i + 1] <= rhos[i] + 0.02 for i in range(len(rhos) - 1)), rhos


def test_vcycle_converges_to_direct_solution():
    """The stationary V-cycle iteration converges to the LU solution
    (brute force, tiny N) and contracts at a rate flat in N."""
    its = []
    for N in (128, 256, 512):
        k = D.Kernel(D.CONST, 0.05)
        A = D.assemble_dense(k, N)
        b = synthetic.random_vector(2 * N - 1, seed=N)
        H = dense.build_hierarchy(A, 5)
        x, it, hist = dense.solve(H, b, tol=1e-12)
        xs = scipy.linalg.solve(A, b)
        assert np.abs(x - xs).max() <= 1e-9 * np.abs(xs).max()
        assert hist[-1] < 1e-12
        its.append(it)
    assert max(its) - min(its) <= 2, its


@pytest.mark.parametrize("kern", [D.Kernel(D.CONST, 0.25), D.Kernel(D.WEIGHTED, 0.05, wl=1.2, wr=0.8),
                                  D.Kernel(D.FRACTIONAL, 0.1, alpha=0.4)], ids=lambda k: k.kind)
def test_tpx_vcycle_equals_dense_vcycle(kern):
    """The O8 path (FFT matvecs, Lemma 3.1 levels) computes the same iterates
    as the dense O2-O7 path."""
    N = 256
    A = D.assemble_dense(kern, N)
    H = dense.build_hierarchy(A, 5)
    Ht = tpx.Hierarchy.build(tpx.from_stencil(kern, N), 5)
    b = D.rhs_manufactured(kern, N)
    e1 = dense.vcycle(H, b)
    e2 = tpx.vcycle(Ht, b)
    # the two coarsest matrices (dense R A P vs Lemma 3.1) differ by rounding;
    # the exact coarsest solve amplifies that by its condition number, which
    # for the fractional kernel is ~2e4 here (it tracks the finest level's)
    kap = np.linalg.cond(H.A[-1])
    assert np.abs(e1 - e2).max() <= max(1e-13, 64 * np.finfo(float).eps * kap) * np.abs(e1).max()
    x1, i1, h1 = dense.solve(H, b, tol=1e-10, max_iter=200)
    x2, i2, h2 = tpx.solve(Ht, b, tol=1e-10, max_iter=200)
    assert i1 == i2
    # histories agree down to the rounding floor of forming b - A x (~1e-13 of ||r_0||)
    np.testing.assert_allclose(h1, h2, rtol=1e-6, atol=1e-12)


def test_two_grid_config_c1():
    """N = 2^7, delta = 1/4, constant kernel, two-grid (coarse level of 2^6
    intervals solved exactly), omega = 2/3, m1 = m2 = 1, tol 1e-10: converges,
    and the discrete solution is within 1e-9 of u = x^2 (1-x)^2."""
    N = 128
    k = D.Kernel(D.CONST, 0.25)
    A = D.assemble_dense(k, N)
    b = D.rhs_manufactured(k, N)
    H = dense.build_hierarchy(A, 6)
    assert H.nlevels == 2
    x, it, hist = dense.solve(H, b, tol=1e-10)
    assert hist[-1] < 1e-10 and it <= 12
    assert np.abs(x - D.u_exact(D.points_block(N))).max() < 1e-9


def test_pcg_identity_preconditioner_terminates():
    """Plain CG (identity preconditioner) on a small SPD system terminates in
    at most m = 2N - 1 steps in exact arithmetic; in FP64 the residual falls
    below 1e-10 within m + 5 steps and the result is the LU solution.  A
    wrong sign, index or beta formula breaks finite termination."""
    N = 16
    k = D.Kernel(D.CONST, 0.25)
    A = D.assemble_dense(k, N)
    H = tpx.Hierarchy.build(tpx.from_stencil(k, N), 2)
    b = synthetic.random_vector(2 * N - 1, seed=3)
    x, it, hist = tpx.pcg(H, b, tol=1e-10, max_iter=200, precond=lambda r: r.copy())
    assert hist[-1] < 1e-10 and it <= (2 * N - 1) + 5, (it, hist[-1])
    xs = scipy.linalg.solve(A, b)
    assert np.abs(x - xs).max() <= 1e-8 * np.abs(xs).max()


@pytest.mark.parametrize("kern", [D.Kernel(D.CONST, 0.05), D.Kernel(D.FRACTIONAL, 0.1, alpha=0.4)],
                         ids=lambda k: k.kind)
def test_pcg_energy_error_decreases(kern):
    """V-cycle-preconditioned CG (symmetric V-cycle: m1 = m2, equal damping,
    P = 2 R^T) minimises the energy norm of the error over growing Krylov
    spaces, so ||x_k - x*||_A never increases; it reaches the LU solution and
    needs no more iterations than the stationary V-cycle iteration."""
    N = 256
    A = D.assemble_dense(kern, N)
    H = tpx.Hierarchy.build(tpx.from_stencil(kern, N), 5)
    b = D.rhs_manufactured(kern, N)
    xs = scipy.linalg.solve(A, b)
    errs = []

    def energy(x):
        e = x - xs
        errs.append(float(np.sqrt(e @ (A @ e))))

    x, it, hist = tpx.pcg(H, b, tol=1e-10, max_iter=100, callback=energy)
    assert hist[-1] < 1e-10
    e0 = float(np.sqrt(xs @ (A @ xs)))
    assert all(errs[i + 1] <= errs[i] * (1 + 1e-6) + 1e-12 * e0 for i in range(len(errs) - 1)), errs
    assert np.abs(x - xs).max() <= 1e-7 * np.abs(xs).max()
    _, it_stat, _ = tpx.solve(H, b, tol=1e-10, max_iter=500)
    assert it <= it_stat, (it, it_stat)


def test_w_cycle_pins():
    """W-cycle (opts.cycle = 2): with two levels it is the V-cycle (the
    coarsest is solved exactly once); it is a fixed linear map (B(r1 + r2) =
    B r1 + B r2) whose error propagator I - B A contracts more than the
    V-cycle's; for the fractional kernel (alpha = 0.4) the stationary
    W-iteration count stays flat in N while the V-iteration's grows."""
    k = D.Kernel(D.FRACTIONAL, 0.1, alpha=0.4)
    W = tpx.Options(cycle=2)
    N = 64
    H2 = tpx.Hierarchy.build(tpx.from_stencil(k, N), 5)
    r = synthetic.random_vector(2 * N - 1, seed=1)
    np.testing.assert_array_equal(tpx.vcycle(H2, r, W), tpx.vcycle(H2, r))
    H = tpx.Hierarchy.build(tpx.from_stencil(k, N), 2)
    r2 = synthetic.random_vector(2 * N - 1, seed=2)
    lin = tpx.vcycle(H, r + r2, W) - tpx.vcycle(H, r, W) - tpx.vcycle(H, r2, W)
    assert np.abs(lin).max() <= 1e-10 * np.abs(tpx.vcycle(H, r, W)).max()
    A = H.levels[0].T.dense()
    m = A.shape[0]
    BW = np.column_stack([tpx.vcycle(H, e, W) for e in np.eye(m)])
    BV = np.column_stack([tpx.vcycle(H, e) for e in np.eye(m)])
    rho = lambda Bm: max(abs(np.linalg.eigvals(np.eye(m) - Bm @ A)))
    assert rho(BW) < rho(BV) < 1
    its = {}
    for N in (256, 1024, 4096):
        HN = tpx.Hierarchy.build(tpx.from_stencil(k, N), 5)
        b = synthetic.random_vector(2 * N - 1, seed=N)
        its[N] = (tpx.solve(HN, b, tol=1e-10, max_iter=600, opts=W)[1],
                  tpx.solve(HN, b, tol=1e-10, max_iter=600)[1])
    w = [v[0] for v in its.values()]
    v = [v[1] for v in its.values()]
    assert max(w) - min(w) <= 5 and v[-1] > 2 * v[0] and w[-1] < v[-1], its
