"""BDF4 time stepping (Sec. 5, eq. (bdf4)) on the HIP path through the C ABI:
the paper's printed errors (Tables TT01, TT02) from GPU solves, and step-by-
step parity with the oracle's iterative run at larger N.

Every test prints the case it runs (flushed) before touching the GPU."""
import json
import os
import sys

import numpy as np
import pytest

from oracle import bdf4
from oracle import discretize as D

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU-only machines
    pytest.skip("needs a GPU", allow_module_level=True)
from paper_2202_11288_amd import binding as B  # noqa: E402

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "bdf4_tables.json")))
SCHEMES = {"shifted": (B.AMG_SCHEME_SHIFTED, D.SHIFTED), "standard": (B.AMG_SCHEME_STANDARD, D.STANDARD)}


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(device="cuda", dtype=torch.float64)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def gpu_run(scheme_name, N, delta, steps=None, tol=1e-13, precision=B.AMG_FP64, coarsest=None,
            **opts):
    """BDF4 with tau = h through amg_bdf4_step; the source tau (F - s E g) is
    formed on the host with the library's volume correction (amg_volume_rhs)
    and the manufactured forcing.  Returns (U at the last step, iterations)."""
    bs, osch = SCHEMES[scheme_name]
    kern = B.kernel(B.AMG_K_CONST, scheme=bs)
    okern = D.Kernel(D.CONST, delta)
    s = bdf4.paper_scale(okern)
    tau = 1.0 / N
    steps = N if steps is None else steps
    cl = coarsest if coarsest is not None else min(5, int(np.log2(N)) - 1)
    h = B.amg_setup(kern, delta, N, B.amg_default_opts(shift=bdf4.BDF4_LEAD, scale=tau * s,
                                                      precision=precision, coarsest_log2=cl,
                                                      max_iter=100, **opts))
    try:
        x = D.points_block(N)
        S = B.amg_volume_reach(kern, delta, N)
        k = np.arange(S + 1) / (2.0 * N)
        bufs = [dev(bdf4.exact(j * tau, x)) for j in range(4)]  # U^0..U^3
        its = []
        for step in range(4, steps + 1):
            t = step * tau
            # src = tau (F - s E g): amg_volume_rhs subtracts E g from its input
            Fs = bdf4.forcing(okern, s, t, x) / s
            src = tau * s * B.amg_volume_rhs(kern, delta, N, bdf4.exact(t, -k), bdf4.exact(t, 1.0 + k), Fs)
            hist = [bufs[-1], bufs[-2], bufs[-3], bufs[-4]]
            out = bufs[-4]  # U^{k-4} is overwritten by U^k (b is formed first)
            st, it, rel = B.amg_bdf4_step(h, hist, dev(src), out, tol)
            its.append(it)
            bufs = [bufs[-3], bufs[-2], bufs[-1], out]
        return host(bufs[-1]), its
    finally:
        B.amg_destroy(h)


PAPER = [(tab, col, i) for tab in ("TT01", "TT02") for col in ("delta=1/4", "delta=sqrt(h)")
         for i in (0, 1, 2)]


@pytest.mark.parametrize("tab,col,i", PAPER, ids=[f"{t}-{c}-N{GOLDEN['N'][i]}" for t, c, i in PAPER])
def test_gpu_bdf4_reproduces_paper_errors(tab, col, i):
    """The whole time loop on the GPU (FP64, tol 1e-13 per step, the paper's
    smoother (omega_pre, omega_post) = (1, 1/2), coarsest 2^3) gives the
    paper's printed max-norm error at t = 1 to its printed digits."""
    N = GOLDEN["N"][i]
    delta = 0.25 if col == "delta=1/4" else bdf4.paper_delta_sqrt_h(N)
    scheme = GOLDEN["tables"][tab]["scheme"]
    say("bdf4 paper", tab, col, N)
    U, its = gpu_run(scheme, N, delta, coarsest=3, omega_pre=1.0, omega_post=0.5)
    err = np.abs(U - bdf4.exact(1.0, D.points_block(N))).max()
    printed = GOLDEN["tables"][tab][col]["error"][i]
    say("error", err, "printed", printed, "mean iters", np.mean(its))
    unit = 10.0 ** (np.floor(np.log10(printed)) - 4)
    assert abs(err - printed) <= 1.5 * unit


@pytest.mark.parametrize("scheme,N,prec", [("shifted", 4096, B.AMG_FP64), ("standard", 4096, B.AMG_FP64),
                                           ("shifted", 16384, B.AMG_MIXED)])
def test_gpu_bdf4_matches_oracle_steps(scheme, N, prec):
    """Steps 4..15 at a size with four-step FFT levels: the solution after
    the last step agrees with the oracle's V-cycle run of the same steps, with
    the same iteration counts in FP64.  tol 1e-10 per step: the residual of
    the initial guess U^{k-1} is only O(tau) of b, so the FP64 rounding floor
    of b - A x sits near 1e-11 of it at this N; two runs within tol of the
    step solutions differ by about cond(M) tol |r_0| / |b| <= 1e-10 relative."""
    say("bdf4 oracle parity", scheme, N, prec)
    steps = 15
    U, its = gpu_run(scheme, N, 0.25, steps=steps, tol=1e-10, precision=prec)
    r = bdf4.run_tpx(D.Kernel(D.CONST, 0.25), N, SCHEMES[scheme][1], steps=steps, tol=1e-10)
    err = np.abs(U - r.U).max() / np.abs(r.U).max()
    say("rel diff", err, "gpu iters", its, "oracle iters", r.iters)
    assert err <= 1e-9
    if prec == B.AMG_FP64:
        assert all(abs(a - b) <= 1 for a, b in zip(its, r.iters))
    else:
        assert max(its) <= 2 * max(r.iters) + 3
