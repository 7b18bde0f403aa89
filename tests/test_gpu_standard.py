"""The standard (non-symmetric) collocation of eq. (ccs2.6) with non-zero
volume data on the HIP path, through the C ABI, against the CPU FP64 oracle.

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

STD = B.AMG_SCHEME_STANDARD
CASES = {
    "const-0.25": (B.kernel(B.AMG_K_CONST, scheme=STD), D.Kernel(D.CONST, 0.25), 0.25),
    "weighted-0.05": (B.kernel(B.AMG_K_WEIGHTED, wl=1.2, wr=0.8, scheme=STD),
                      D.Kernel(D.WEIGHTED, 0.05, wl=1.2, wr=0.8), 0.05),
    "const-0.0371": (B.kernel(B.AMG_K_CONST, scheme=STD), D.Kernel(D.CONST, 0.0371), 0.0371),
}


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(device="cuda", dtype=torch.float64)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def oracle_hier(name, N, coarsest=5):
    return tpx.Hierarchy.build(tpx.from_stencil(CASES[name][1], N, D.STANDARD), coarsest)


def kappa_tol(H):
    """Rounding of two equally valid hierarchies, amplified by the exact
    coarsest solve (64 eps kappa of the coarsest matrix)."""
    return 64 * np.finfo(float).eps * np.linalg.cond(H.levels[-1].dense())


@pytest.mark.parametrize("name,N", [("const-0.25", 16384), ("weighted-0.05", 32768),
                                    ("const-0.0371", 4096)])
def test_standard_matvec_and_vcycle(name, N):
    """A x and one V-cycle (Algorithm 2) on the non-symmetric finest level."""
    kern, okern, delta = CASES[name]
    say("standard matvec/vcycle", name, N)
    h = B.amg_setup(kern, delta, N)
    try:
        H = oracle_hier(name, N)
        r = synthetic.random_vector(2 * N - 1, seed=N + 3)
        y = torch.empty(2 * N - 1, device="cuda", dtype=torch.float64)
        B.amg_matvec(h, dev(r), y)
        yo = H.matvec(r)
        err = np.abs(host(y) - yo).max() / np.abs(yo).max()
        say("matvec err", err)
        assert err < 1e-13
        e = torch.empty(2 * N - 1, device="cuda", dtype=torch.float64)
        B.amg_vcycle(h, dev(r), e)
        eo = tpx.vcycle(H, r)
        err = np.abs(host(e) - eo).max() / np.abs(eo).max()
        say("vcycle err", err)
        assert err < max(1e-13, kappa_tol(H))
    finally:
        B.amg_destroy(h)


def _volume_rhs_pair(name, N):
    """(library b, oracle b) for u = (1+x)^6 with g = u on the interaction
    volume: f - E g, the library's E g from amg_volume_rhs, the oracle's
    from its row sums."""
    kern, okern, delta = CASES[name]
    S = B.amg_volume_reach(kern, delta, N)
    k = np.arange(S + 1) / (2.0 * N)
    gl, gr = D.u_poly6(-k), D.u_poly6(1.0 + k)
    f = D.f_poly6(okern, D.points_block(N))
    b_lib = B.amg_volume_rhs(kern, delta, N, gl, gr, f.copy())
    b_or = f - D.volume_correction(okern, N, gl, gr, D.STANDARD)
    return b_lib, b_or


@pytest.mark.parametrize("prec", [B.AMG_FP64, B.AMG_MIXED])
@pytest.mark.parametrize("name,N", [("const-0.25", 16384), ("weighted-0.05", 4096),
                                    ("const-0.0371", 4096)])
def test_standard_volume_data_solve(name, N, prec):
    """Solve A U = f - E g (tol 1e-10): the iteration count of the oracle's
    stationary V-cycle iteration (FP64), the oracle's residual of the GPU
    solution below tol, the solution within 4 kappa tol of the oracle's, and
    close to the manufactured u = (1+x)^6 itself (the volume data carried
    through)."""
    kern, okern, delta = CASES[name]
    say("standard volume solve", name, N, "prec", prec)
    tol = 1e-10
    b_lib, b_or = _volume_rhs_pair(name, N)
    np.testing.assert_allclose(b_lib, b_or, rtol=0, atol=1e-12 * np.abs(b_or).max())
    h = B.amg_setup(kern, delta, N, B.amg_default_opts(precision=prec, max_iter=200))
    try:
        x = torch.zeros(2 * N - 1, device="cuda", dtype=torch.float64)
        st, it, rel = B.amg_solve(h, dev(b_lib), x, tol)
        assert st == B.AMG_OK
        H = oracle_hier(name, N)
        xo, ito, histo = tpx.solve(H, b_or, tol=tol, max_iter=200)
        xg = host(x)
        relo = np.linalg.norm(b_or - H.matvec(xg)) / np.linalg.norm(b_or)
        say("iters", it, "oracle", ito, "rel", rel, "oracle rel", relo)
        assert relo < 1.01 * tol + kappa_tol(H)
        if prec == B.AMG_FP64:
            assert abs(it - ito) <= 1
        else:
            assert it <= 2 * ito + 5
        kap = np.linalg.cond(H.levels[-1].dense())
        assert np.abs(xg - xo).max() <= max(1e-12, 4 * kap * tol) * np.abs(xo).max()
        # u itself: the discretisation error is O(h^4) (below 1e-13 here), the
        # rest is the solver's tolerance times the finest level's conditioning;
        # dropping the volume data would leave an O(1) error
        u = D.u_poly6(D.points_block(N))
        assert np.abs(xg - u).max() <= 1e-6 * np.abs(u).max()
    finally:
        B.amg_destroy(h)


def test_standard_pcg_refused_and_batch():
    """Conjugate gradients needs symmetry: the standard scheme is refused;
    a batch of standard-scheme solves equals the solo solves."""
    kern, okern, delta = CASES["weighted-0.05"]
    with pytest.raises(B.AmgError):
        B.amg_setup(kern, delta, 1024, B.amg_default_opts(inner=B.AMG_INNER_PCG))
    N = 4096
    say("standard batch", N)
    b_lib, _ = _volume_rhs_pair("weighted-0.05", N)
    hs = [B.amg_setup(kern, delta, N) for _ in range(2)]
    try:
        bs = [dev(b_lib), dev(b_lib * 0.5)]
        xs = [torch.zeros(2 * N - 1, device="cuda", dtype=torch.float64) for _ in range(2)]
        B.amg_solve_batch(hs, bs, xs, [1e-10, 1e-10])
        for hh, bb, xx in zip(hs, bs, xs):
            x1 = torch.zeros_like(xx)
            B.amg_solve(hh, bb, x1, 1e-10)
            assert torch.equal(x1, xx)
    finally:
        for hh in hs:
            B.amg_destroy(hh)
