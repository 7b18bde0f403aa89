"""Oracle, part 4: BDF4 time stepping (TEST INFRASTRUCTURE ONLY).

Sec. 5 of arXiv 2202.11288, eq. (bdf4), for the time-dependent peridynamic
model (ccs2.4): u_t - L_delta u = f on (0, 1), u = g on the interaction
volume, u(x, 0) = u_0.  With A the collocation matrix of -L_delta (this
package's sign: SPD for the constant kernel under the shifted rule) and E its
coupling to the exterior points, the fourth-order backward differentiation
formula at step tau reads

    (25/12 I + tau A) U^k = 4 U^{k-1} - 3 U^{k-2} + 4/3 U^{k-3} - 1/4 U^{k-4}
                            + tau (F^k - E g^k).

The paper writes the operator as 25/12 I - tau A with A standing for the
discretisation of L_delta itself; the two agree.

Readings, all pinned by the error columns of the paper's Tables TT01 and TT02
(tests/golden/bdf4_tables.json):

* kernel constant 3 delta^-3 (the constant kernel of Sec. 2.2), i.e. `scale`
  = 2 times this package's normalised constant 3 / (2 delta^3);
* exact solution u = e^t (1 + x)^6 (Sec. 5), so F = u_t + scale * (-L u) and
  g = u on the interaction volume;
* tau = h = 1/N, U^0..U^3 taken from the exact solution, the error is the
  maximum over the collocation points at t = 1;
* delta = sqrt(h): the horizon is r h with r = floor(delta / h) (the paper's
  r of Sec. 2.2), kernel constant 3 (r h)^-3.

``run_dense`` solves each step by LU of the dense matrix (small N);
``shifted_tpx`` and ``run_tpx`` give the same steps on Toeplitz-plus-Cross
levels with the stationary V-cycle iteration (for parity at larger N).
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.linalg

from . import discretize as disc
from . import tpx

BDF4 = (4.0, -3.0, 4.0 / 3.0, -0.25)   # coefficients of U^{k-1}..U^{k-4}
BDF4_LEAD = 25.0 / 12.0                # coefficient of U^k


def paper_scale(kernel: disc.Kernel) -> float:
    """Ratio of the paper's constant 3 delta^-3 to this package's normalised
    constant kernel (the factor multiplying A and E)."""
    assert kernel.kind == disc.CONST
    return 3.0 / kernel.delta ** 3 / kernel.c


def paper_delta_sqrt_h(N: int) -> float:
    """The horizon the delta = sqrt(h) columns use: r h, r = floor(sqrt(N))."""
    return float(np.floor(np.sqrt(N))) / N


def exact(t, x):
    return np.exp(t) * (1.0 + x) ** 6


def forcing(kernel: disc.Kernel, scale: float, t: float, x):
    """F(x, t) = u_t - L u for u = e^t (1 + x)^6 with the kernel times scale:
    e^t ((1+x)^6 + scale * f_6(x)), f_6 = -L (1+x)^6 under the normalised kernel."""
    return np.exp(t) * ((1.0 + x) ** 6 + scale * disc.f_poly6(kernel, x))


def history_rhs(U1, U2, U3, U4, src=None):
    """4 U^{k-1} - 3 U^{k-2} + 4/3 U^{k-3} - 1/4 U^{k-4} + src."""
    b = BDF4[0] * U1 + BDF4[1] * U2 + BDF4[2] * U3 + BDF4[3] * U4
    return b if src is None else b + src


def source(kernel: disc.Kernel, N: int, scheme: str, scale: float, tau: float, t: float):
    """tau (F^k - E g^k) with E g from the row sums of the volume correction."""
    x = disc.points_block(N)
    S = disc.volume_reach(kernel, N, scheme)
    k = np.arange(S + 1) / (2.0 * N)
    Eg = disc.volume_correction(kernel, N, exact(t, -k), exact(t, 1.0 + k), scheme)
    return tau * (forcing(kernel, scale, t, x) - scale * Eg)


@dataclasses.dataclass
class Run:
    U: np.ndarray          # U^N (t = 1)
    error: float           # max |U^N - u(., 1)|
    iters: list            # iterations per step (iterative runs)


def run_dense(kernel: disc.Kernel, N: int, scheme: str = disc.SHIFTED, scale: float = None,
              steps: int = None) -> Run:
    """BDF4 with tau = h = 1/N over `steps` steps (default N, to t = 1),
    every step solved by LU of the dense matrix 25/12 I + tau * scale * A."""
    scale = paper_scale(kernel) if scale is None else scale
    steps = N if steps is None else steps
    A, E, q = disc.assemble_with_exterior(kernel, N, scheme)
    x = disc.points_block(N)
    xe = q / (2.0 * N)
    tau = 1.0 / N
    lu = scipy.linalg.lu_factor(BDF4_LEAD * np.eye(len(x)) + tau * scale * A)
    U = [exact(k * tau, x) for k in range(4)]
    for k in range(4, steps + 1):
        t = k * tau
        src = tau * (forcing(kernel, scale, t, x) - scale * (E @ exact(t, xe)))
        U.append(scipy.linalg.lu_solve(lu, history_rhs(U[-1], U[-2], U[-3], U[-4], src)))
        U = U[-4:]
    t_end = steps * tau
    return Run(U[-1], float(np.abs(U[-1] - exact(t_end, x)).max()), [])


def shifted_tpx(T: tpx.TpX, shift: float, scale: float) -> tpx.TpX:
    """shift I + scale T on the Toeplitz-plus-Cross representation: every
    generator, Cross entry and band entry times scale, shift on the diagonal
    entries (offset 0 of A and D_bar, and o)."""
    n = T.n
    a, d = scale * T.a, scale * T.d
    a[n - 1] += shift
    d[n - 1] += shift
    band = None if T.band is None else tuple(scale * v for v in T.band)
    return tpx.TpX(n, a, scale * T.b, scale * T.c, d, scale * T.p, scale * T.q, scale * T.xi,
                   scale * T.zeta, scale * T.o + shift, band)


def run_tpx(kernel: disc.Kernel, N: int, scheme: str = disc.SHIFTED, scale: float = None,
            steps: int = None, tol: float = 1e-12, opts: tpx.Options = tpx.Options(),
            coarsest_log2: int = 5, max_iter: int = 200) -> Run:
    """The same steps solved by the stationary V-cycle iteration on the
    hierarchy of 25/12 I + tau * scale * A, from the initial guess U^{k-1}."""
    scale = paper_scale(kernel) if scale is None else scale
    steps = N if steps is None else steps
    tau = 1.0 / N
    H = tpx.Hierarchy.build(shifted_tpx(tpx.from_stencil(kernel, N, scheme), BDF4_LEAD,
                                        tau * scale), coarsest_log2)
    x = disc.points_block(N)
    U = [exact(k * tau, x) for k in range(4)]
    its = []
    for k in range(4, steps + 1):
        b = history_rhs(U[-1], U[-2], U[-3], U[-4], source(kernel, N, scheme, scale, tau, k * tau))
        Uk, it, _ = tpx.solve(H, b, tol=tol, max_iter=max_iter, opts=opts, x0=U[-1])
        its.append(it)
        U.append(Uk)
        U = U[-4:]
    t_end = steps * tau
    return Run(U[-1], float(np.abs(U[-1] - exact(t_end, x)).max()), its)
