"""Pin of the oracle's cycle step structure (CPU only).

Algorithm 2 from a zero guess is a linear map r -> B_k r.  Its error
propagator I - B_k A_k has a closed matrix form built only from the
definitions of Sec. 3.1: the damped-Jacobi error propagator
S = I - omega D^-1 A (eq. (7 Jacobi)), the restriction R, the prolongation
P = 2 R^T and the Galerkin coarse matrix R A P (eq. (block Galerkin)):

    I - B_k A_k = S_post^m2 (I - P B_{k-1} R A_k) S_pre^m1,
    B_{k-1} = (I - E_{k-1}^gamma) A_{k-1}^-1,   E_{k-1} = I - B_{k-1}' A_{k-1},

with gamma = 1 for the V-cycle and B_coarsest = A_coarsest^-1 (the exact
solve).  For two levels this is the two-grid operator S_post^m2 T S_pre^m1
with T = I - P A_c^-1 R A (T_k of Sec. 3.1).  gamma = 2 is the W-cycle (two
coarse cycles, the second from the first's result; the level above the
coarsest solves exactly once).

The tests form B column by column from the oracle's recursive cycle functions
(``dense.vcycle`` and ``tpx.vcycle``) applied to unit vectors and compare
I - B A with the matrix form entry by entry.  A cycle with one post-sweep too
few (the paper's printed loop bound), or with the two damping factors
swapped, is planted in the oracle's own function to show that the check sees
it.
"""
import numpy as np
import pytest

from oracle import dense, discretize as D, tpx

KERNELS = [D.Kernel(D.CONST, 0.25), D.Kernel(D.WEIGHTED, 0.05, wl=1.2, wr=0.8),
           D.Kernel(D.FRACTIONAL, 0.1, alpha=0.4)]
SWEEPS = [(1, 1, 2.0 / 3.0, 2.0 / 3.0), (2, 1, 1.0, 0.5), (1, 3, 0.8, 0.6)]


def error_propagator(As, level, m1, m2, w_pre, w_post, gamma=1):
    """I - B_level A_level from the matrix definitions (see module docstring).
    As[l] are the dense level matrices, finest first; As[-1] is solved
    exactly."""
    A = As[level]
    m = A.shape[0]
    I = np.eye(m)
    if level == len(As) - 1:
        return np.zeros((m, m))
    R = dense.restriction(m)
    P = 2.0 * R.T
    Dinv = 1.0 / np.diag(A)
    S_pre = I - w_pre * Dinv[:, None] * A
    S_post = I - w_post * Dinv[:, None] * A
    Ac = As[level + 1]
    Ec = error_propagator(As, level + 1, m1, m2, w_pre, w_post, gamma)
    visits = 1 if level + 2 == len(As) else gamma
    Bc = (np.eye(Ac.shape[0]) - np.linalg.matrix_power(Ec, visits)) @ np.linalg.inv(Ac)
    E = I - P @ Bc @ R @ A
    return np.linalg.matrix_power(S_post, m2) @ E @ np.linalg.matrix_power(S_pre, m1)


def columns(f, m):
    return np.column_stack([f(e) for e in np.eye(m)])


def _dense_levels(kern, N, coarsest_log2):
    H = dense.build_hierarchy(D.assemble_dense(kern, N), coarsest_log2)
    return H, H.A


def _tpx_levels(kern, N, coarsest_log2):
    H = tpx.Hierarchy.build(tpx.from_stencil(kern, N), coarsest_log2)
    As = [L.T.dense() for L in H.levels[:-1]] + [H.levels[-1].dense()]
    return H, As


def _gap(E_cycle, E_form):
    # relative to the propagator's largest entry (a few 1e-3 for these cycles)
    return np.abs(E_cycle - E_form).max() / np.abs(E_form).max()


def _tol(As):
    # the rounding of B (which carries A_coarsest^-1) measured here stays
    # below 3e-12 of the propagator's largest entry for every case; planted
    # mistakes move it by more than 0.3
    return 1e-10


@pytest.mark.parametrize("kern", KERNELS, ids=lambda k: k.kind)
@pytest.mark.parametrize("sweeps", SWEEPS, ids=lambda s: "m%d%d_w%.2g_%.2g" % s)
@pytest.mark.parametrize("N,kc", [(64, 5), (128, 6), (128, 5), (128, 4)],
                         ids=["2lev64", "2lev128", "3lev128", "4lev128"])
def test_dense_vcycle_error_propagator(kern, sweeps, N, kc):
    """dense.vcycle: I - B A equals S_post^m2 (I - P B_c R A) S_pre^m1
    recursively (two levels: S_post^m2 T S_pre^m1)."""
    m1, m2, wp, wq = sweeps
    H, As = _dense_levels(kern, N, kc)
    m = As[0].shape[0]
    opts = dense.Options(m1=m1, m2=m2, omega_pre=wp, omega_post=wq)
    B = columns(lambda e: dense.vcycle(H, e, opts), m)
    E_form = error_propagator(As, 0, m1, m2, wp, wq)
    assert _gap(np.eye(m) - B @ As[0], E_form) <= _tol(As)


@pytest.mark.parametrize("kern", KERNELS, ids=lambda k: k.kind)
@pytest.mark.parametrize("sweeps", SWEEPS, ids=lambda s: "m%d%d_w%.2g_%.2g" % s)
@pytest.mark.parametrize("N,kc", [(64, 5), (128, 5), (128, 4)], ids=["2lev64", "3lev128", "4lev128"])
def test_tpx_vcycle_error_propagator(kern, sweeps, N, kc):
    """tpx.vcycle (FFT matvecs, Lemma 3.1 levels) has the same error
    propagator, formed from its own level matrices."""
    m1, m2, wp, wq = sweeps
    H, As = _tpx_levels(kern, N, kc)
    m = As[0].shape[0]
    opts = tpx.Options(m1=m1, m2=m2, omega_pre=wp, omega_post=wq)
    B = columns(lambda e: tpx.vcycle(H, e, opts), m)
    assert _gap(np.eye(m) - B @ As[0], error_propagator(As, 0, m1, m2, wp, wq)) <= _tol(As)


@pytest.mark.parametrize("kern", KERNELS[:1] + KERNELS[2:], ids=lambda k: k.kind)
def test_tpx_wcycle_error_propagator(kern):
    """tpx.vcycle with cycle = 2 (W-cycle) on four levels: gamma = 2 coarse
    cycles per level, one exact solve at the level above the coarsest."""
    H, As = _tpx_levels(kern, 128, 4)
    m = As[0].shape[0]
    opts = tpx.Options(m1=1, m2=2, omega_pre=0.8, omega_post=0.6, cycle=2)
    B = columns(lambda e: tpx.vcycle(H, e, opts), m)
    E = np.eye(m) - B @ As[0]
    assert _gap(E, error_propagator(As, 0, 1, 2, 0.8, 0.6, gamma=2)) <= _tol(As)
    # and it is not the V-cycle's propagator
    assert _gap(E, error_propagator(As, 0, 1, 2, 0.8, 0.6, gamma=1)) > 1e-2


def test_two_grid_operator_matches_cycle():
    """The two-grid operator on which Theorem 4.1's bound is tested
    (dense.two_grid_error_operator) is the error propagator of the oracle's
    own two-level cycle with m1 = 0 pre-sweeps."""
    kern = D.Kernel(D.CONST, 0.25)
    for omega in (0.5, 2.0 / 3.0, 1.0):
        H, As = _dense_levels(kern, 64, 5)
        m = As[0].shape[0]
        opts = dense.Options(m1=0, m2=1, omega_pre=omega, omega_post=omega)
        B = columns(lambda e: dense.vcycle(H, e, opts), m)
        E2 = dense.two_grid_error_operator(As[0], omega, m1=0, m2=1)
        assert _gap(np.eye(m) - B @ As[0], E2) <= _tol(As)


@pytest.mark.parametrize("planted", ["one_post_sweep_short", "damping_swapped"])
def test_planted_cycle_mistakes_fail(planted):
    """Mistakes planted in the oracle's cycle (one post-sweep too few, as the
    printed loop bound reads; pre- and post-damping swapped) are caught: the
    cycle's propagator is then far from the matrix form."""
    kern = D.Kernel(D.CONST, 0.25)
    m1, m2, wp, wq = 2, 1, 1.0, 0.5
    for N, kc, (H, As) in ((64, 5, _dense_levels(kern, 64, 5)), (128, 5, _tpx_levels(kern, 128, 5))):
        m = As[0].shape[0]
        if planted == "one_post_sweep_short":
            bad = dict(m1=m1, m2=m2 - 1, omega_pre=wp, omega_post=wq)
        else:
            bad = dict(m1=m1, m2=m2, omega_pre=wq, omega_post=wp)
        if isinstance(H, dense.DenseHierarchy):
            B = columns(lambda e: dense.vcycle(H, e, dense.Options(**bad)), m)
        else:
            B = columns(lambda e: tpx.vcycle(H, e, tpx.Options(**bad)), m)
        gap = _gap(np.eye(m) - B @ As[0], error_propagator(As, 0, m1, m2, wp, wq))
        assert gap > 0.3, (planted, N, gap)
