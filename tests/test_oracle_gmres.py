"""Pins of the oracle's restarted flexible GMRES (V-cycle right
preconditioner): the minimal-residual property against brute-force least
squares over an explicit Krylov basis, finite termination, restarts, and the
LU solution of the non-symmetric systems."""
from __future__ import annotations

import numpy as np
import pytest
import scipy.linalg

import synthetic
from oracle import discretize as D
from oracle import tpx

KERNELS = [(D.Kernel(D.WEIGHTED, 0.25, wl=1.2, wr=0.8), D.SHIFTED),
           (D.Kernel(D.CONST, 0.25), D.STANDARD)]
IDS = ["weighted-shifted", "const-standard"]


@pytest.mark.parametrize("kern,scheme", KERNELS, ids=IDS)
@pytest.mark.parametrize("k", [1, 2, 3, 5])
def test_one_cycle_minimises_residual_over_krylov_space(kern, scheme, k):
    """One cycle of k steps from x0 returns x0 + B c with c minimising
    ||r0 - A B c|| over K_k(A B, r0) (B the V-cycle, a fixed linear map in
    FP64): brute force on the explicit basis [r0, (AB) r0, ...] by least
    squares gives the same residual norm."""
    N = 32
    H = tpx.Hierarchy.build(tpx.from_stencil(kern, N, scheme), 3)
    A = H.levels[0].T.dense()
    b = synthetic.random_vector(2 * N - 1, seed=7)
    x0 = synthetic.random_vector(2 * N - 1, seed=8)
    x, it, hist = tpx.gmres(H, b, tol=1e-30, max_iter=k, restart=k, x0=x0)
    assert it == k
    Bop = lambda v: tpx.vcycle(H, v)
    r0 = b - A @ x0
    K = [r0 / np.linalg.norm(r0)]
    for _ in range(k - 1):
        v = A @ Bop(K[-1])
        K.append(v / np.linalg.norm(v))
    BK = np.column_stack([Bop(v) for v in K])
    c, *_ = np.linalg.lstsq(A @ BK, r0, rcond=None)
    best = np.linalg.norm(r0 - A @ BK @ c)
    got = np.linalg.norm(b - A @ x)
    assert abs(got - best) <= 1e-9 * np.linalg.norm(r0), (got, best)
    assert abs(hist[-1] - got / np.linalg.norm(r0)) <= 1e-12


@pytest.mark.parametrize("kern,scheme", KERNELS, ids=IDS)
def test_identity_preconditioner_terminates(kern, scheme):
    """Unpreconditioned GMRES without restarts terminates in at most m = 2N-1
    steps; in FP64 it reaches 1e-10 within m steps, at the LU solution."""
    N = 16
    H = tpx.Hierarchy.build(tpx.from_stencil(kern, N, scheme), 2)
    A = H.levels[0].T.dense()
    b = synthetic.random_vector(2 * N - 1, seed=3)
    m = 2 * N - 1
    x, it, hist = tpx.gmres(H, b, tol=1e-10, max_iter=200, restart=m, precond=lambda r: r.copy())
    assert hist[-1] < 1e-10 and it <= m, (it, hist[-1])
    xs = scipy.linalg.solve(A, b)
    assert np.abs(x - xs).max() <= 1e-8 * np.abs(xs).max()
    # estimates never increase within a cycle
    assert all(hist[i + 1] <= hist[i] * (1 + 1e-12) for i in range(len(hist) - 2))


@pytest.mark.parametrize("kern,scheme", KERNELS, ids=IDS)
def test_restarted_gmres_solves(kern, scheme):
    """With the V-cycle and short restarts: the true residual ends below tol,
    the solution is the LU one, and no more V-cycles are needed than by the
    stationary iteration."""
    N = 256
    H = tpx.Hierarchy.build(tpx.from_stencil(kern, N, scheme), 5)
    A = H.levels[0].T.dense()
    b = synthetic.random_vector(2 * N - 1, seed=11)
    xs = scipy.linalg.solve(A, b)
    for m in (3, 30):
        x, it, hist = tpx.gmres(H, b, tol=1e-10, max_iter=200, restart=m)
        assert np.linalg.norm(b - A @ x) / np.linalg.norm(b) < 1e-10
        assert abs(hist[-1] - np.linalg.norm(b - A @ x) / np.linalg.norm(b)) < 1e-13
        assert np.abs(x - xs).max() <= 1e-8 * np.abs(xs).max()
        _, it_stat, _ = tpx.solve(H, b, tol=1e-10, max_iter=500)
        assert it <= it_stat, (m, it, it_stat)
