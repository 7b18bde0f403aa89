"""Restarted flexible GMRES with the V-cycle as right preconditioner
(inner = AMG_INNER_GMRES) on the HIP path, through the C ABI, against the
oracle's GMRES.

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

CASES = {
    "weighted-0.05": (B.kernel(B.AMG_K_WEIGHTED, wl=1.2, wr=0.8),
                      D.Kernel(D.WEIGHTED, 0.05, wl=1.2, wr=0.8), 0.05, D.SHIFTED),
    "standard-const-0.25": (B.kernel(B.AMG_K_CONST, scheme=B.AMG_SCHEME_STANDARD),
                            D.Kernel(D.CONST, 0.25), 0.25, D.STANDARD),
    "const-0.25": (B.kernel(B.AMG_K_CONST), D.Kernel(D.CONST, 0.25), 0.25, D.SHIFTED),
}


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(device="cuda", dtype=torch.float64)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def hier(name, N, coarsest=5):
    _, okern, _, scheme = CASES[name]
    return tpx.Hierarchy.build(tpx.from_stencil(okern, N, scheme), coarsest)


def kappa(H):
    return np.linalg.cond(H.levels[-1].dense())


@pytest.mark.parametrize("name,N,restart", [("weighted-0.05", 32768, 30),
                                            ("standard-const-0.25", 16384, 30),
                                            ("const-0.25", 16384, 30),
                                            ("weighted-0.05", 4096, 3),
                                            ("standard-const-0.25", 2048, 2)])
def test_gmres_matches_oracle(name, N, restart):
    """FP64: the same iteration count (+-1) and residual history as the
    oracle's GMRES (classical Gram-Schmidt twice vs modified Gram-Schmidt:
    equal to rounding); the oracle's residual of the GPU solution below tol;
    solutions within 4 kappa tol.  Short restarts exercise the update/restart
    round."""
    kern, okern, delta, _ = CASES[name]
    say("gmres", name, N, restart)
    tol = 1e-10
    b = synthetic.random_vector(2 * N - 1, seed=N + restart)
    h = B.amg_setup(kern, delta, N, B.amg_default_opts(inner=B.AMG_INNER_GMRES, restart=restart,
                                                      max_iter=300))
    try:
        x = torch.zeros(2 * N - 1, device="cuda", dtype=torch.float64)
        st, it, rel = B.amg_solve(h, dev(b), x, tol)
        hist = B.amg_residual_history(h)
    finally:
        B.amg_destroy(h)
    H = hier(name, N)
    xo, ito, histo = tpx.gmres(H, b, tol=tol, max_iter=300, restart=restart)
    xg = host(x)
    relo = np.linalg.norm(b - H.matvec(xg)) / np.linalg.norm(b)
    say("iters", it, "oracle", ito, "rel", rel, "oracle rel of gpu x", relo)
    assert abs(it - ito) <= 1
    assert relo < 1.01 * tol
    assert abs(rel - relo) < 1e-12
    k = min(len(hist), len(histo)) - 1
    np.testing.assert_allclose(hist[:k], histo[:k], rtol=1e-6, atol=1e-13)
    assert np.abs(xg - xo).max() <= max(1e-12, 4 * kappa(H) * tol) * np.abs(xo).max()


def test_gmres_mixed_precision():
    """FP32 V-cycle as the (flexible) preconditioner, FP64 Arnoldi and
    residual: reaches the FP64 tolerance, close to the FP64 oracle's solution,
    with at most a few more V-cycles; fewer than the stationary iteration."""
    name, N = "weighted-0.05", 65536
    kern, okern, delta, _ = CASES[name]
    say("gmres mixed", name, N)
    tol = 1e-10
    b = B.amg_manufactured_rhs(kern, delta, N)
    h = B.amg_setup(kern, delta, N, B.amg_default_opts(inner=B.AMG_INNER_GMRES,
                                                      precision=B.AMG_MIXED))
    try:
        x = torch.zeros(2 * N - 1, device="cuda", dtype=torch.float64)
        st, it, rel = B.amg_solve(h, dev(b), x, tol)
    finally:
        B.amg_destroy(h)
    hs = B.amg_setup(kern, delta, N, B.amg_default_opts(precision=B.AMG_MIXED))
    try:
        xs = torch.zeros(2 * N - 1, device="cuda", dtype=torch.float64)
        _, it_stat, _ = B.amg_solve(hs, dev(b), xs, tol)
    finally:
        B.amg_destroy(hs)
    H = hier(name, N)
    xo, ito, _ = tpx.gmres(H, b, tol=1e-12, max_iter=300)
    xg = host(x)
    relo = np.linalg.norm(b - H.matvec(xg)) / np.linalg.norm(b)
    say("mixed iters", it, "stationary", it_stat, "fp64 oracle", ito, "rel", relo)
    assert relo < 1.01 * tol
    assert np.abs(xg - xo).max() <= 4 * kappa(H) * tol * np.abs(xo).max()
    assert it <= it_stat


def test_gmres_batch_matches_solo():
    """amg_solve_batch with GMRES handles (different N, kernels, restart,
    precision): bitwise the solo solves."""
    say("gmres batch")
    cases = [("weighted-0.05", 4096, 30, B.AMG_FP64), ("standard-const-0.25", 8192, 5, B.AMG_MIXED),
             ("const-0.25", 2048, 30, B.AMG_FP64)]
    hs, bs, xs, solo = [], [], [], []
    try:
        for name, N, R, prec in cases:
            kern, _, delta, _ = CASES[name]
            h = B.amg_setup(kern, delta, N, B.amg_default_opts(inner=B.AMG_INNER_GMRES, restart=R,
                                                              precision=prec))
            hs.append(h)
            bs.append(dev(synthetic.random_vector(2 * N - 1, seed=N)))
            x1 = torch.zeros_like(bs[-1])
            B.amg_solve(h, bs[-1], x1, 1e-10)
            solo.append(x1)
            xs.append(torch.zeros_like(bs[-1]))
        st, its, rels = B.amg_solve_batch(hs, bs, xs, [1e-10] * len(hs))
        for x, x1 in zip(xs, solo):
            assert torch.equal(x, x1)
    finally:
        for h in hs:
            B.amg_destroy(h)
