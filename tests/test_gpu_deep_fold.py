"""AMG_FLAG_DEEP_FOLD: the V-cycle below the four-step levels applied as one
dense product formed at setup.  It is the same linear map as the
small-level kernel's cycle up to rounding: V-cycle outputs agree to FP64
rounding (FP64 form) and FP32 rounding (mixed form), solves converge in the
same iteration count to the oracle's residual, the batched rounds reproduce
the solo solves bit for bit, and the W-cycle ignores the flag.

Every test prints the case it runs (flushed) before touching the GPU."""
import sys

import numpy as np
import pytest

import synthetic
from oracle import discretize as D
from oracle import tpx

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU-only machines
    pytest.skip("needs a GPU", allow_module_level=True)
from paper_2202_11288_amd import binding as B  # noqa: E402


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


CASES = [(B.kernel(B.AMG_K_CONST), D.Kernel(D.CONST, 0.25), 0.25, "const"),
         (B.kernel(B.AMG_K_WEIGHTED, wl=1.2, wr=0.8), D.Kernel(D.WEIGHTED, 0.1, wl=1.2, wr=0.8), 0.1,
          "weighted")]


@pytest.mark.parametrize("N", [2 ** 12, 2 ** 14, 2 ** 17])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("case", CASES, ids=lambda c: c[3])
def test_deep_fold_same_vcycle(case, prec, N):
    kern, _, delta, name = case
    P = B.AMG_FP64 if prec == "fp64" else B.AMG_MIXED
    say("deep fold vcycle", name, prec, N)
    hs = [B.amg_setup(kern, delta, N, B.amg_default_opts(precision=P, flags=f))
          for f in (0, B.AMG_FLAG_DEEP_FOLD)]
    try:
        dt = torch.float64 if P == B.AMG_FP64 else torch.float32
        r = torch.from_numpy(synthetic.random_vector(2 * N - 1, seed=N)).cuda().to(dt)
        es = []
        for h in hs:
            e = torch.zeros_like(r)
            B.amg_vcycle(h, r, e)
            es.append(e.double().cpu().numpy())
        rel = np.linalg.norm(es[1] - es[0]) / np.linalg.norm(es[0])
        say("relative difference", rel)
        assert rel < (1e-13 if P == B.AMG_FP64 else 2e-6)
    finally:
        for h in hs:
            B.amg_destroy(h)


@pytest.mark.parametrize("case", CASES, ids=lambda c: c[3])
def test_deep_fold_solve_matches_oracle(case):
    kern, okern, delta, name = case
    N = 2 ** 13
    say("deep fold solve", name, N)
    b = B.amg_manufactured_rhs(kern, delta, N)
    res = {}
    for f in (0, B.AMG_FLAG_DEEP_FOLD):
        h = B.amg_setup(kern, delta, N, B.amg_default_opts(precision=B.AMG_MIXED, flags=f))
        try:
            x = torch.zeros(2 * N - 1, device="cuda", dtype=torch.float64)
            st, it, rel = B.amg_solve(h, torch.from_numpy(b).cuda(), x, 1e-10)
            res[f] = (st, it, x.cpu().numpy())
        finally:
            B.amg_destroy(h)
    assert res[0][0] == res[B.AMG_FLAG_DEEP_FOLD][0] == B.AMG_OK
    assert abs(res[0][1] - res[B.AMG_FLAG_DEEP_FOLD][1]) <= 1
    T = tpx.from_stencil(okern, N)
    xd = res[B.AMG_FLAG_DEEP_FOLD][2]
    relo = np.linalg.norm(b - tpx.Level.build(T).matvec(xd)) / np.linalg.norm(b)
    say("iterations", res[0][1], res[B.AMG_FLAG_DEEP_FOLD][1], "oracle relres", relo)
    assert relo < 1.01e-10


def test_deep_fold_batch_bitwise():
    """Deep-fold and plain handles of several sizes solved together: each
    result equals its own solo solve bit for bit."""
    g = synthetic.rng(9)
    specs = [(2 ** 12, B.AMG_FLAG_DEEP_FOLD), (2 ** 14, B.AMG_FLAG_DEEP_FOLD), (2 ** 14, 0),
             (2 ** 16, B.AMG_FLAG_DEEP_FOLD), (2 ** 11, B.AMG_FLAG_DEEP_FOLD)]
    say("deep fold batch", specs)
    hs, bs, xs = [], [], []
    try:
        for N, f in specs:
            hs.append(B.amg_setup(B.kernel(B.AMG_K_CONST), float(g.uniform(0.05, 0.3)), N,
                                  B.amg_default_opts(precision=B.AMG_MIXED, flags=f)))
            bs.append(torch.from_numpy(g.standard_normal(2 * N - 1)).cuda())
            xs.append(torch.zeros_like(bs[-1]))
        B.amg_solve_batch(hs, bs, xs, [1e-10] * len(hs))
        for h, b, x in zip(hs, bs, xs):
            u = torch.zeros_like(b)
            B.amg_solve(h, b, u, 1e-10)
            assert torch.equal(u, x)
    finally:
        for h in hs:
            B.amg_destroy(h)


def test_deep_fold_ignored_by_wcycle():
    N = 2 ** 13
    say("deep fold with W-cycle", N)
    k = B.kernel(B.AMG_K_CONST)
    hs = [B.amg_setup(k, 0.25, N, B.amg_default_opts(cycle=2, flags=f))
          for f in (0, B.AMG_FLAG_DEEP_FOLD)]
    try:
        r = torch.from_numpy(synthetic.random_vector(2 * N - 1, seed=1)).cuda()
        es = []
        for h in hs:
            e = torch.zeros_like(r)
            B.amg_vcycle(h, r, e)
            es.append(e)
        assert torch.equal(es[0], es[1])
    finally:
        for h in hs:
            B.amg_destroy(h)
