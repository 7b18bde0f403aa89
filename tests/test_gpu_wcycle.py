"""W-cycles (opts.cycle = 2) on the HIP path, through the C ABI, against the
oracle's W-cycle.

Every test prints the case it runs (flushed) before touching the GPU."""
import sys

import numpy as np
import pytest

import synthetic
from oracle import discretize as D
from oracle import tpx
from oracle import weakly_singular as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU-only machines
    pytest.skip("needs a GPU", allow_module_level=True)
from paper_2202_11288_amd import binding as B  # noqa: E402

WOPTS = tpx.Options(cycle=2)
FRAC = (B.kernel(B.AMG_K_FRACTIONAL, alpha=0.4), D.Kernel(D.FRACTIONAL, 0.1, alpha=0.4), 0.1)
WEIGHTED = (B.kernel(B.AMG_K_WEIGHTED, wl=1.2, wr=0.8), D.Kernel(D.WEIGHTED, 0.05, wl=1.2, wr=0.8), 0.05)


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def dev(x, dt=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(x)).to(device="cuda", dtype=dt)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("case,N,prec", [(FRAC, 512, B.AMG_FP64), (FRAC, 4096, B.AMG_FP64),
                                         (WEIGHTED, 16384, B.AMG_FP64), (FRAC, 16384, B.AMG_MIXED)])
def test_wcycle_matches_oracle(case, N, prec):
    """One W-cycle from zero, twice (the second replays the captured graph
    when there are two or more four-step levels)."""
    kern, okern, delta = case
    say("wcycle", okern.kind, N, prec)
    h = B.amg_setup(kern, delta, N, B.amg_default_opts(cycle=2, precision=prec))
    try:
        H = tpx.Hierarchy.build(tpx.from_stencil(okern, N), 5)
        r = synthetic.random_vector(2 * N - 1, seed=N)
        eo = tpx.vcycle(H, r, WOPTS)
        dt = torch.float32 if prec == B.AMG_MIXED else torch.float64
        kap = np.linalg.cond(H.levels[-1].dense())
        # FP32 cycles: rounding amplified by the coarsest level's conditioning
        tol = (max(1e-13, 64 * np.finfo(float).eps * kap) if prec == B.AMG_FP64
               else max(1e-5, 16 * float(np.finfo(np.float32).eps) * kap))
        for rep in range(3):
            e = torch.empty(2 * N - 1, device="cuda", dtype=dt)
            B.amg_vcycle(h, dev(r, dt), e)
            err = np.abs(host(e) - eo).max() / np.abs(eo).max()
            say("rep", rep, "err", err, "tol", tol)
            assert err < tol
    finally:
        B.amg_destroy(h)


def test_wcycle_weakly_singular():
    """The band levels in the W-cycle's small-level program."""
    g, N = 0.5, 4096
    say("wcycle weakly singular", N)
    h = B.amg_setup(B.kernel(B.AMG_K_WEAKLY_SINGULAR, gamma=g), 0.0, N, B.amg_default_opts(cycle=2))
    try:
        H = tpx.Hierarchy.build(W.level(g, N), 5)
        r = synthetic.random_vector(2 * N - 1, seed=3)
        e = torch.empty(2 * N - 1, device="cuda", dtype=torch.float64)
        B.amg_vcycle(h, dev(r), e)
        eo = tpx.vcycle(H, r, WOPTS)
        err = np.abs(host(e) - eo).max() / np.abs(eo).max()
        say("err", err)
        assert err < 1e-12
    finally:
        B.amg_destroy(h)


def test_w_iteration_flat_in_n():
    """Stationary iteration with W-cycles for the fractional kernel: the same
    iteration count as the oracle's at each N (+-1), flat in N, and fewer than
    with V-cycles at the largest N."""
    kern, okern, delta = FRAC
    its = {}
    for N in (1024, 4096):
        say("w iteration", N)
        b = synthetic.random_vector(2 * N - 1, seed=N + 1)
        h = B.amg_setup(kern, delta, N, B.amg_default_opts(cycle=2, max_iter=400))
        try:
            x = torch.zeros(2 * N - 1, device="cuda", dtype=torch.float64)
            st, it, rel = B.amg_solve(h, dev(b), x, 1e-10)
        finally:
            B.amg_destroy(h)
        H = tpx.Hierarchy.build(tpx.from_stencil(okern, N), 5)
        _, ito, _ = tpx.solve(H, b, tol=1e-10, max_iter=400, opts=WOPTS)
        hv = B.amg_setup(kern, delta, N, B.amg_default_opts(max_iter=600))
        try:
            xv = torch.zeros(2 * N - 1, device="cuda", dtype=torch.float64)
            _, itv, _ = B.amg_solve(hv, dev(b), xv, 1e-10)
        finally:
            B.amg_destroy(hv)
        say("N", N, "W", it, "oracle W", ito, "V", itv)
        assert abs(it - ito) <= 1
        its[N] = (it, itv)
    assert abs(its[4096][0] - its[1024][0]) <= 5
    assert its[4096][0] < its[4096][1]
