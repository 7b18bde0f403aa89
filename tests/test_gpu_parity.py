"""Parity of the HIP path (through the C ABI) with the CPU FP64 oracle.

Every test prints the case it runs (flushed) before touching the GPU."""
import sys

import numpy as np
import pytest

import synthetic
from oracle import dense
from oracle import discretize as D
from oracle import tpx

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU-only machines
    pytest.skip("needs a GPU", allow_module_level=True)
from paper_2202_11288_amd import binding as B  # noqa: E402

CONST25 = ("const-0.25", B.kernel(B.AMG_K_CONST), D.Kernel(D.CONST, 0.25), 0.25)
CONST05 = ("const-0.05", B.kernel(B.AMG_K_CONST), D.Kernel(D.CONST, 0.05), 0.05)
WEIGHT05 = ("weighted-0.05", B.kernel(B.AMG_K_WEIGHTED, wl=1.2, wr=0.8),
            D.Kernel(D.WEIGHTED, 0.05, wl=1.2, wr=0.8), 0.05)
FRAC04 = ("frac-0.4", B.kernel(B.AMG_K_FRACTIONAL, alpha=0.4),
          D.Kernel(D.FRACTIONAL, 0.1, alpha=0.4), 0.1)
# the near-field rule (an extension for 0 < alpha < 1, not in the paper)
NEAR07 = ("near-0.7", B.kernel(B.AMG_K_FRACTIONAL_NEAR, alpha=0.7),
          D.Kernel(D.FRACTIONAL_NEAR, 0.1, alpha=0.7), 0.1)
NEAR09 = ("near-0.9", B.kernel(B.AMG_K_FRACTIONAL_NEAR, alpha=0.9),
          D.Kernel(D.FRACTIONAL_NEAR, 0.05, alpha=0.9), 0.05)


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def dev(x, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(x)).to(device="cuda", dtype=dtype)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


_oracle_cache = {}


def oracle_hier(case, N, coarsest=5):
    key = (case[0], N, coarsest)
    if key not in _oracle_cache:
        _oracle_cache.clear()
        _oracle_cache[key] = tpx.Hierarchy.build(tpx.from_stencil(case[2], N), coarsest)
    return _oracle_cache[key]


def kappa_tol(H):
    """Tolerance for comparing V-cycle outputs and solutions computed from two
    equally valid hierarchies: their coarsest matrices (C++ recurrences vs the
    oracle's Lemma 3.1) differ by rounding, and the exact coarsest solve
    amplifies that by the condition number of the coarsest matrix, which for
    the Galerkin levels tracks that of the finest one.  64 eps kappa."""
    return 64 * np.finfo(float).eps * np.linalg.cond(H.levels[-1].dense())


def oracle_level_matvec(H, l, x):
    if l < len(H.levels) - 1:
        return H.levels[l].matvec(x)
    return H.levels[-1].dense() @ x


@pytest.mark.parametrize("case,N", [
    (CONST25, 64), (CONST25, 1024), (CONST25, 8192), (CONST25, 16384), (CONST25, 65536),
    (CONST05, 32768), (WEIGHT05, 256), (WEIGHT05, 16384), (FRAC04, 1024), (FRAC04, 32768),
    (NEAR07, 16384), (NEAR09, 1024),
])
def test_level_matvec_every_level(case, N):
    """y = A_l x on every level (tail levels: one-workgroup FFT in LDS;
    larger ones: three-pass four-step FFT) against the oracle's FFT matvec
    (itself pinned to dense products).  FFT rounding ~ eps log2 L."""
    say("level_matvec", case[0], N)
    h = B.amg_setup(case[1], case[3], N)
    try:
        H = oracle_hier(case, N)
        for l in range(B.amg_num_levels(h)):
            m = B.amg_level_size(h, l)
            x = synthetic.random_vector(m, seed=1000 + l)
            y = torch.empty(m, device="cuda", dtype=torch.float64)
            B.amg_level_matvec(h, l, dev(x), y)
            yr = oracle_level_matvec(H, l, x)
            err = np.abs(host(y) - yr).max() / np.abs(yr).max()
            assert err < 1e-13, (l, m, err)
    finally:
        B.amg_destroy(h)


@pytest.mark.parametrize("N", [512, 16384, 2 ** 20, 2 ** 21, 2 ** 22])
def test_matvec_general_blocks(N):
    """Caller-supplied non-symmetric blocks (AMG_K_GENERATORS): the general
    two-complex-spectra path against dense (small N) / oracle FFT (large N;
    2^20 runs the full-tile four-step kernels with register first/last passes,
    2^20 and 2^21 the wide column tiles of the largest levels, 2^22 rows of
    4096 points)."""
    say("general_blocks", N)
    gA, gB, gC, gD = synthetic.random_tpx_arrays(N - 1, seed=N, decay=0.001)
    gen = np.ascontiguousarray(np.concatenate([gA, gB, gC, gD]))
    h = B.amg_setup(B.kernel(B.AMG_K_GENERATORS, gen=gen), 0.0, N)
    try:
        T0 = tpx.from_blocks(gA, gB, gC, gD, N)
        x = synthetic.random_vector(2 * N - 1, seed=5)
        y = torch.empty(2 * N - 1, device="cuda", dtype=torch.float64)
        B.amg_matvec(h, dev(x), y)
        yr = (D.assemble_dense_from_blocks(gA, gB, gC, gD, N) @ x if N <= 1024
              else tpx.Level.build(T0).matvec(x))
        err = np.abs(host(y) - yr).max() / np.abs(yr).max()
        assert err < 1e-13, err
        # coarse levels of the general path
        Ts = [T0]
        for l in range(1, B.amg_num_levels(h)):
            Ts.append(tpx.coarsen(Ts[-1]))
            m = B.amg_level_size(h, l)
            x = synthetic.random_vector(m, seed=l)
            y = torch.empty(m, device="cuda", dtype=torch.float64)
            B.amg_level_matvec(h, l, dev(x), y)
            yr = Ts[-1].dense() @ x if m < 2000 else tpx.Level.build(Ts[-1]).matvec(x)
            err = np.abs(host(y) - yr).max() / np.abs(yr).max()
            assert err < 1e-13, (l, err)
    finally:
        B.amg_destroy(h)


@pytest.mark.parametrize("case,N", [(CONST25, 1024), (CONST25, 16384), (WEIGHT05, 32768),
                                    (FRAC04, 16384), (CONST05, 128), (NEAR07, 16384)])
def test_vcycle_matches_oracle(case, N):
    """One V-cycle (Algorithm 2) from zero: same algorithm, so outputs agree
    to rounding amplified by the conditioning (see kappa_tol)."""
    say("vcycle", case[0], N)
    h = B.amg_setup(case[1], case[3], N)
    try:
        H = oracle_hier(case, N)
        r = synthetic.random_vector(2 * N - 1, seed=N + 7)
        e = torch.empty(2 * N - 1, device="cuda", dtype=torch.float64)
        B.amg_vcycle(h, dev(r), e)
        er = tpx.vcycle(H, r)
        err = np.abs(host(e) - er).max() / np.abs(er).max()
        tol = max(1e-13, kappa_tol(H))
        say("vcycle err", err, "tol", tol)
        assert err < tol, (err, tol)
    finally:
        B.amg_destroy(h)


@pytest.mark.parametrize("case,N,coarsest", [
    (CONST25, 128, 6),      # two-grid, 2^7 intervals
    (CONST25, 16384, 5), (CONST05, 16384, 5), (WEIGHT05, 32768, 5), (FRAC04, 4096, 5),
])
def test_solve_matches_oracle(case, N, coarsest):
    """Outer iteration (Sec. 5 stopping rule, tol 1e-10, manufactured RHS):
    same iteration count and residual history as the oracle; the oracle's
    residual of the GPU solution is below tol."""
    say("solve", case[0], N, coarsest)
    tol = 1e-10
    h = B.amg_setup(case[1], case[3], N, B.amg_default_opts(coarsest_log2=coarsest, max_iter=400))
    try:
        b = B.amg_manufactured_rhs(case[1], case[3], N)
        x = torch.zeros(2 * N - 1, device="cuda", dtype=torch.float64)
        st, it, rel = B.amg_solve(h, dev(b), x, tol)
        hist = B.amg_residual_history(h)
        H = oracle_hier(case, N, coarsest)
        xo, ito, histo = tpx.solve(H, b, tol=tol, max_iter=400)
        assert abs(it - ito) <= 1, (it, ito)
        k = min(len(hist), len(histo))
        # each history entry is formed to ~eps kappa |r_0| (see kappa_tol)
        np.testing.assert_allclose(hist[:k], histo[:k], rtol=1e-5, atol=max(1e-12, kappa_tol(H) / 16))
        xg = host(x)
        relo = np.linalg.norm(b - H.matvec(xg)) / np.linalg.norm(b)
        # forming b - A x loses ~eps |A| |x| / |b| <= eps kappa
        assert relo < 1.01 * tol + kappa_tol(H), relo
        assert abs(rel - relo) < 1e-12 + kappa_tol(H)
        # two solutions with relative residual < tol differ by <= 2 kappa tol
        kap = np.linalg.cond(H.levels[-1].dense())
        assert np.abs(xg - xo).max() <= max(1e-12, 4 * kap * tol) * np.abs(xo).max()
    finally:
        B.amg_destroy(h)


@pytest.mark.parametrize("case,N", [(CONST25, 16384), (WEIGHT05, 32768), (CONST05, 4096)])
def test_mixed_precision_refinement(case, N):
    """FP32 V-cycle inside FP64 refinement reaches the same FP64 tolerance; the
    solution agrees with the FP64 oracle's to ~cond * tol."""
    say("mixed", case[0], N)
    tol = 1e-10
    h = B.amg_setup(case[1], case[3], N, B.amg_default_opts(precision=B.AMG_MIXED))
    try:
        b = B.amg_manufactured_rhs(case[1], case[3], N)
        x = torch.zeros(2 * N - 1, device="cuda", dtype=torch.float64)
        st, it, rel = B.amg_solve(h, dev(b), x, tol)
        H = oracle_hier(case, N)
        xg = host(x)
        relo = np.linalg.norm(b - H.matvec(xg)) / np.linalg.norm(b)
        assert relo < 1.01 * tol
        xo, ito, _ = tpx.solve(H, b, tol=1e-12, max_iter=400)
        kap = np.linalg.cond(H.levels[-1].dense())
        err = np.abs(xg - xo).max() / np.abs(xo).max()
        say("mixed iters", it, "fp64 oracle iters", ito, "error vs FP64 oracle", err)
        assert err <= 4 * kap * tol
        assert it <= 2 * ito + 5
    finally:
        B.amg_destroy(h)


def test_mixed_vcycle_close_to_fp64():
    """The FP32 V-cycle approximates the FP64 one to FP32 accuracy."""
    case, N = CONST25, 16384
    say("mixed_vcycle", N)
    h = B.amg_setup(case[1], case[3], N, B.amg_default_opts(precision=B.AMG_MIXED))
    try:
        r = synthetic.random_vector(2 * N - 1, seed=3)
        e = torch.empty(2 * N - 1, device="cuda", dtype=torch.float32)
        B.amg_vcycle(h, dev(r, torch.float32), e)
        er = tpx.vcycle(oracle_hier(case, N), r)
        err = np.abs(host(e) - er).max() / np.abs(er).max()
        assert err < 5e-5, err
    finally:
        B.amg_destroy(h)


WEIGHT25 = ("weighted-0.25", B.kernel(B.AMG_K_WEIGHTED, wl=1.2, wr=0.8),
            D.Kernel(D.WEIGHTED, 0.25, wl=1.2, wr=0.8), 0.25)


@pytest.mark.parametrize("case", [CONST25, CONST05, WEIGHT25, WEIGHT05], ids=lambda c: c[0])
def test_large_n_2_20(case):
    """N = 2^20 (the benchmark size), every plain-method case of that size
    (delta = 0.05, 0.25; constant and weighted 1.2/0.8 kernels): finest
    matvec against the oracle's FFT matvec and one V-cycle against the
    oracle's; FP64 and mixed solves to 1e-10 whose residual the oracle
    evaluates, the FP64 iteration count within one of the oracle's own
    stationary solve, the mixed one within two."""
    N = 2 ** 20
    say("large", case[0], N)
    H = oracle_hier(case, N)
    b = B.amg_manufactured_rhs(case[1], case[3], N)
    xo, ito, _ = tpx.solve(H, b, tol=1e-10, max_iter=100)
    for prec in (B.AMG_FP64, B.AMG_MIXED):
        h = B.amg_setup(case[1], case[3], N, B.amg_default_opts(precision=prec))
        try:
            if prec == B.AMG_FP64:
                x = synthetic.random_vector(2 * N - 1, seed=9)
                y = torch.empty(2 * N - 1, device="cuda", dtype=torch.float64)
                B.amg_matvec(h, dev(x), y)
                yr = H.matvec(x)
                assert np.abs(host(y) - yr).max() / np.abs(yr).max() < 1e-13
                e = torch.empty_like(y)
                B.amg_vcycle(h, dev(x), e)
                er = tpx.vcycle(H, x)
                assert np.abs(host(e) - er).max() / np.abs(er).max() < max(1e-13, kappa_tol(H))
            xs = torch.zeros(2 * N - 1, device="cuda", dtype=torch.float64)
            st, it, rel = B.amg_solve(h, dev(b), xs, 1e-10)
            xg = host(xs)
            relo = np.linalg.norm(b - H.matvec(xg)) / np.linalg.norm(b)
            err = np.abs(xg - xo).max() / np.abs(xo).max()
            say("large solve", case[0], prec, "iters", it, "oracle iters", ito, "relres", rel,
                "oracle-evaluated", relo, "error vs oracle solution", err)
            assert relo < 1.01e-10
            assert abs(it - ito) <= (1 if prec == B.AMG_FP64 else 2), (it, ito)
        finally:
            B.amg_destroy(h)


def test_not_converged_keeps_last_iterate():
    case, N = CONST25, 1024
    say("not_converged", N)
    h = B.amg_setup(case[1], case[3], N, B.amg_default_opts(max_iter=2))
    try:
        b = B.amg_manufactured_rhs(case[1], case[3], N)
        x = torch.zeros(2 * N - 1, device="cuda", dtype=torch.float64)
        st, it, rel = B.amg_solve(h, dev(b), x, 1e-10, allow=(B.AMG_NOT_CONVERGED,))
        assert st == B.AMG_NOT_CONVERGED and it == 2
        xo, ito, _ = tpx.solve(oracle_hier(case, N), b, tol=1e-10, max_iter=2)
        assert ito == 2
        assert np.abs(host(x) - xo).max() <= 1e-11 * np.abs(xo).max()
    finally:
        B.amg_destroy(h)


def test_divergence_detected():
    """omega = 1 with the fractional kernel diverges (lambda_max(D^-1 A) > 2,
    checked by the oracle on the CPU); the solver must stop with
    AMG_DIVERGED instead of spinning."""
    case, N = FRAC04, 1024
    say("diverged", N)
    h = B.amg_setup(case[1], case[3], N, B.amg_default_opts(omega_pre=1.0, omega_post=1.0))
    try:
        b = B.amg_manufactured_rhs(case[1], case[3], N)
        x = torch.zeros(2 * N - 1, device="cuda", dtype=torch.float64)
        st, it, rel = B.amg_solve(h, dev(b), x, 1e-10, allow=(B.AMG_DIVERGED,))
        assert st == B.AMG_DIVERGED and it < 10
    finally:
        B.amg_destroy(h)


def test_zero_rhs_and_exact_initial_guess():
    case, N = CONST25, 256
    say("zero_rhs", N)
    h = B.amg_setup(case[1], case[3], N)
    try:
        b = torch.zeros(2 * N - 1, device="cuda", dtype=torch.float64)
        x = torch.zeros_like(b)
        st, it, rel = B.amg_solve(h, b, x, 1e-10)
        assert st == B.AMG_OK and it == 0 and rel == 0.0
        assert float(torch.abs(x).max()) == 0.0
    finally:
        B.amg_destroy(h)


@pytest.mark.parametrize("prec", [B.AMG_FP64, B.AMG_MIXED])
def test_solve_is_deterministic(prec):
    """Five solves of one problem are bitwise identical (fixed-order
    reductions; no block reads a value another block of the same launch
    writes)."""
    case, N = WEIGHT05, 16384
    say("deterministic", N, prec)
    h = B.amg_setup(case[1], case[3], N, B.amg_default_opts(precision=prec))
    try:
        b = dev(B.amg_manufactured_rhs(case[1], case[3], N))
        xs = []
        for _ in range(5):
            x = torch.zeros_like(b)
            B.amg_solve(h, b, x, 1e-10)
            xs.append(x)
        assert all(torch.equal(xs[0], x) for x in xs[1:])
    finally:
        B.amg_destroy(h)


def test_device_argument_errors():
    case, N = CONST25, 256
    h = B.amg_setup(case[1], case[3], N)
    try:
        x = torch.zeros(2 * N - 1, device="cuda", dtype=torch.float64)
        s = torch.cuda.current_stream().cuda_stream
        import ctypes
        assert B.lib.amg_matvec(h, None, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(s)) == B.AMG_EINVAL
        assert B.lib.amg_matvec(h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(x.data_ptr()),
                                ctypes.c_void_p(s)) == B.AMG_EINVAL
        assert B.lib.amg_level_matvec(h, 17, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(8),
                                      ctypes.c_void_p(s)) == B.AMG_EINVAL
        it = ctypes.c_int()
        rr = ctypes.c_double()
        assert B.lib.amg_solve(h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(8), -1.0,
                               ctypes.c_void_p(s), ctypes.byref(it), ctypes.byref(rr)) == B.AMG_EINVAL
    finally:
        B.amg_destroy(h)


def test_solve_batch_matches_solo_solves():
    """amg_solve_batch: instances of different N, kernel and precision run
    concurrently; each result is bitwise the solo solve's (same kernels, same
    order of operations per instance) and passes the oracle's residual check."""
    say("solve_batch")
    cases = [(CONST25, 4096, B.AMG_FP64), (WEIGHT05, 16384, B.AMG_MIXED),
             (CONST05, 1024, B.AMG_FP64), (FRAC04, 2048, B.AMG_MIXED),
             (CONST25, 32768, B.AMG_MIXED)]
    hs, bs, xs, solo = [], [], [], []
    try:
        for case, N, prec in cases:
            h = B.amg_setup(case[1], case[3], N, B.amg_default_opts(precision=prec, max_iter=400))
            hs.append(h)
            b = dev(B.amg_manufactured_rhs(case[1], case[3], N))
            bs.append(b)
            x1 = torch.zeros_like(b)
            B.amg_solve(h, b, x1, 1e-10)
            solo.append((x1, B.amg_residual_history(h)))
            xs.append(torch.zeros_like(b))
        st, its, rels = B.amg_solve_batch(hs, bs, xs, [1e-10] * len(hs))
        assert st == B.AMG_OK
        for (case, N, prec), x, (x1, h1), it, h in zip(cases, xs, solo, its, hs):
            assert torch.equal(x, x1), (case[0], N)
            assert it == len(h1) - 1
            np.testing.assert_array_equal(B.amg_residual_history(h), h1)
            H = oracle_hier(case, N)
            bh = host(bs[cases.index((case, N, prec))])
            relo = np.linalg.norm(bh - H.matvec(host(x))) / np.linalg.norm(bh)
            assert relo < 1.01e-10 + kappa_tol(H)
    finally:
        for h in hs:
            B.amg_destroy(h)


@pytest.mark.parametrize("prec", [B.AMG_FP64, B.AMG_MIXED])
def test_graph_replay_matches_eager(prec):
    """V-cycles replayed from the captured graph give bit-identical results to
    eager launches.  The graph is captured at a handle's second V-cycle, so the
    first solve already mixes eager, capture and replay rounds; later solves
    and amg_vcycle calls replay it, with eager work and synchronisation in
    between, and every one is compared with the eager handle's result."""
    case, N = CONST25, 2 ** 17
    say("graph replay", prec, N)
    b = dev(B.amg_manufactured_rhs(case[1], case[3], N))
    he = B.amg_setup(case[1], case[3], N, B.amg_default_opts(precision=prec, flags=B.AMG_FLAG_EAGER))
    hg = B.amg_setup(case[1], case[3], N, B.amg_default_opts(precision=prec))
    try:
        xe = torch.zeros_like(b)
        ste = B.amg_solve(he, b, xe, 1e-10)
        dt = torch.float32 if prec == B.AMG_MIXED else torch.float64
        r = dev(synthetic.random_vector(2 * N - 1, seed=77), dt)
        ee = torch.empty_like(r)
        B.amg_vcycle(he, r, ee)
        for k in range(4):
            xg = torch.zeros_like(b)
            stg = B.amg_solve(hg, b, xg, 1e-10)
            assert stg == ste, (k, stg, ste)
            assert torch.equal(xg, xe), k
            eg = torch.empty_like(r)
            B.amg_vcycle(hg, r, eg)
            assert torch.equal(eg, ee), k
            _ = (xg * 2).sum().item()  # eager work and a synchronisation between replays
    finally:
        B.amg_destroy(he)
        B.amg_destroy(hg)


@pytest.mark.parametrize("case,N", [(CONST25, 2 ** 14), (CONST05, 4096), (FRAC04, 4096),
                                    (NEAR07, 4096), (NEAR09, 1024)])
def test_pcg_matches_oracle(case, N):
    """V-cycle-preconditioned CG in FP64 against the oracle's pcg (same steps,
    same Polak-Ribiere update): iteration counts within one, and the
    solution's residual, evaluated by the oracle, below tol (plus the
    hierarchy tolerance: the recurrence's residual and the true one differ by
    rounding amplified by the condition number)."""
    say("pcg", case[0], N)
    H = oracle_hier(case, N)
    b = synthetic.random_vector(2 * N - 1, seed=N + 5)
    xo, ito, ho = tpx.pcg(H, b, tol=1e-10, max_iter=300)
    h = B.amg_setup(case[1], case[3], N, B.amg_default_opts(inner=B.AMG_INNER_PCG, max_iter=300))
    try:
        x = torch.zeros(2 * N - 1, device="cuda", dtype=torch.float64)
        st, it, rel = B.amg_solve(h, dev(b), x, 1e-10)
        say("pcg iterations gpu/oracle", it, ito, rel)
        assert st == B.AMG_OK and rel < 1e-10
        assert abs(it - ito) <= 1, (it, ito)
        hist = B.amg_residual_history(h)
        assert len(hist) == it + 1 and hist[0] == 1.0
        relo = np.linalg.norm(b - H.matvec(host(x))) / np.linalg.norm(b)
        assert relo < 1e-10 + kappa_tol(H), relo
    finally:
        B.amg_destroy(h)


def test_pcg_mixed_and_fractional():
    """PCG with the FP32 V-cycle as preconditioner (FP64 recurrence): the
    fractional kernel (alpha = 0.4) at N = 2^14, where the stationary
    iteration stalls, and the near-field rule at alpha = 0.7, converge to
    1e-10 (oracle-evaluated residual) within a few iterations of the FP64
    PCG; the constant kernel at N = 2^17 needs no more iterations than the
    stationary mixed iteration."""
    for case, N, stationary_too in ((FRAC04, 2 ** 14, False), (NEAR07, 2 ** 12, False),
                                    (CONST25, 2 ** 17, True)):
        say("pcg mixed", case[0], N)
        H = oracle_hier(case, N)
        b = synthetic.random_vector(2 * N - 1, seed=N + 7)
        its = {}
        for prec in (B.AMG_FP64, B.AMG_MIXED):
            h = B.amg_setup(case[1], case[3], N,
                            B.amg_default_opts(inner=B.AMG_INNER_PCG, precision=prec, max_iter=400))
            try:
                x = torch.zeros(2 * N - 1, device="cuda", dtype=torch.float64)
                st, it, rel = B.amg_solve(h, dev(b), x, 1e-10)
                assert st == B.AMG_OK, (prec, st)
                relo = np.linalg.norm(b - H.matvec(host(x))) / np.linalg.norm(b)
                assert relo < 1e-10 + kappa_tol(H), (prec, relo)
                its[prec] = it
            finally:
                B.amg_destroy(h)
        say("pcg iterations fp64/mixed", its)
        assert its[B.AMG_MIXED] <= its[B.AMG_FP64] + 3
        if stationary_too:
            h = B.amg_setup(case[1], case[3], N, B.amg_default_opts(precision=B.AMG_MIXED))
            try:
                x = torch.zeros(2 * N - 1, device="cuda", dtype=torch.float64)
                _, it_stat, _ = B.amg_solve(h, dev(b), x, 1e-10)
            finally:
                B.amg_destroy(h)
            assert its[B.AMG_MIXED] <= it_stat, (its, it_stat)


def test_pcg_batch_matches_solo():
    """amg_solve_batch with CG handles (and one stationary handle in the mix)
    gives each solve's solo result bit for bit."""
    say("pcg batch")
    cases = [(CONST25, 8192, B.AMG_INNER_PCG, B.AMG_FP64), (FRAC04, 4096, B.AMG_INNER_PCG, B.AMG_MIXED),
             (CONST05, 2048, B.AMG_INNER_VCYCLE, B.AMG_FP64), (CONST25, 2 ** 15, B.AMG_INNER_PCG, B.AMG_MIXED),
             (NEAR07, 4096, B.AMG_INNER_PCG, B.AMG_MIXED)]
    hs, bs, xs, solo = [], [], [], []
    try:
        for case, N, inner, prec in cases:
            h = B.amg_setup(case[1], case[3], N,
                            B.amg_default_opts(inner=inner, precision=prec, max_iter=400))
            hs.append(h)
            b = dev(synthetic.random_vector(2 * N - 1, seed=N))
            bs.append(b)
            x1 = torch.zeros_like(b)
            B.amg_solve(h, b, x1, 1e-10)
            solo.append((x1, B.amg_residual_history(h)))
            xs.append(torch.zeros_like(b))
        st, its, rels = B.amg_solve_batch(hs, bs, xs, [1e-10] * len(hs))
        assert st == B.AMG_OK
        for (case, N, inner, prec), x, (x1, h1), h in zip(cases, xs, solo, hs):
            assert torch.equal(x, x1), (case[0], N, inner)
            np.testing.assert_array_equal(B.amg_residual_history(h), h1)
    finally:
        for h in hs:
            B.amg_destroy(h)


@pytest.mark.parametrize("case", [CONST25, WEIGHT05], ids=lambda c: c[0])
def test_rows_of_4096_at_2_22(case):
    """N = 2^22: the finest level (L = 2^23) runs rows of 4096 points (the
    register row pass on 512 threads) and column tiles of 4 x 2048, level 1
    (L = 2^22) rows of 4096 and column tiles of 8 x 1024.  The FP64 matvec of
    both levels against the oracle's FFT matvec (every output), and one FP32
    V-cycle against the oracle's FP64 V-cycle (FP32 rounding through FFTs of
    up to 2^23 points and the exact coarsest solve)."""
    N = 2 ** 22
    say("rows of 4096", case[0], N)
    h = B.amg_setup(case[1], case[3], N, B.amg_default_opts(precision=B.AMG_MIXED))
    try:
        H = oracle_hier(case, N)
        x = synthetic.random_vector(2 * N - 1, seed=41)
        y = torch.empty(2 * N - 1, device="cuda", dtype=torch.float64)
        B.amg_matvec(h, dev(x), y)
        yr = H.matvec(x)
        err = np.abs(host(y) - yr).max() / np.abs(yr).max()
        say("matvec err", err)
        assert err < 1e-13, err
        m1 = B.amg_level_size(h, 1)
        x1 = synthetic.random_vector(m1, seed=42)
        y1 = torch.empty(m1, device="cuda", dtype=torch.float64)
        B.amg_level_matvec(h, 1, dev(x1), y1)
        yr1 = H.levels[1].matvec(x1)
        err = np.abs(host(y1) - yr1).max() / np.abs(yr1).max()
        say("level-1 matvec err", err)
        assert err < 1e-13, err
        r = synthetic.random_vector(2 * N - 1, seed=43)
        e = torch.empty(2 * N - 1, device="cuda", dtype=torch.float32)
        B.amg_vcycle(h, dev(r, torch.float32), e)
        er = tpx.vcycle(H, r)
        err = np.abs(host(e) - er).max() / np.abs(er).max()
        say("fp32 vcycle err", err)
        assert err < 1e-4, err
    finally:
        B.amg_destroy(h)


def test_fractional_2_22_mixed_pcg():
    """The precision configuration's operator with the plain FP64 residual:
    N = 2^22 intervals (8,388,607 unknowns), delta = 0.1, fractional kernel
    alpha = 0.4, FP32 V-cycle with FP64 residual.  The finest FP64 matvec
    against the oracle's FFT matvec (every output), and a V-cycle-
    preconditioned CG solve at tol 1e-10 whose final residual the oracle
    evaluates.  The true residual b - A x, formed by the FP64 FFT, stops near
    2e-9 here (its evaluation error, about eps |A| |x| / |b|, measured by the
    oracle in extended precision), so the solve ends as AMG_NOT_CONVERGED once
    restarts stop improving it; AMG_FLAG_ACCURATE_RESIDUAL reaches 1e-10
    (test_gpu_precision)."""
    N = 2 ** 22
    kern, okern, delta = B.kernel(B.AMG_K_FRACTIONAL, alpha=0.4), D.Kernel(D.FRACTIONAL, 0.1, alpha=0.4), 0.1
    say("fractional 2^22")
    H = tpx.Hierarchy.build(tpx.from_stencil(okern, N), 5)
    # about 490 CG steps at this size (74 at 2^14, 294 at 2^20): the V-cycle's
    # contraction for this kernel degrades with N
    h = B.amg_setup(kern, delta, N, B.amg_default_opts(precision=B.AMG_MIXED,
                                                      inner=B.AMG_INNER_PCG, max_iter=800))
    try:
        x = synthetic.random_vector(2 * N - 1, seed=22)
        y = torch.empty(2 * N - 1, device="cuda", dtype=torch.float64)
        B.amg_matvec(h, dev(x), y)
        yr = H.matvec(x)
        err = np.abs(host(y) - yr).max() / np.abs(yr).max()
        say("matvec err", err)
        assert err < 1e-13
        b = B.amg_manufactured_rhs(kern, delta, N)
        xs = torch.zeros(2 * N - 1, device="cuda", dtype=torch.float64)
        st, it, rel = B.amg_solve(h, dev(b), xs, 1e-10, allow=(B.AMG_OK, B.AMG_NOT_CONVERGED))
        xh = host(xs)
        nb = np.linalg.norm(b)
        yo = H.matvec(xh)
        relo = np.linalg.norm(b - yo) / nb
        # both evaluations of b - A x sit at their FP64 floor here: they differ
        # by what the two FFT matvecs of this x differ by (|A| |x| >> |b|)
        yg = torch.empty_like(xs)
        B.amg_matvec(h, xs, yg)
        d = np.linalg.norm(host(yg) - yo) / nb
        rext = tpx.relres_extended(tpx.from_stencil_rowsum(okern, N), b, xh)
        say("pcg status", st, "iters", it, "rel", rel, "oracle rel", relo, "matvec gap", d,
            "extended", rext)
        assert rel < 1e-8 and rext < 1e-8
        assert abs(rel - relo) <= 1.01 * d + 1e-12
    finally:
        B.amg_destroy(h)


def test_binding_rejects_bad_tensors():
    """The binding refuses tensors the library would read past or misread
    (wrong dtype, length, layout or device) before any device work; the V-cycle
    of a mixed handle takes float32."""
    say("binding tensor checks")
    N = 256
    h = B.amg_setup(CONST25[1], CONST25[3], N)
    hm = B.amg_setup(CONST25[1], CONST25[3], N, B.amg_default_opts(precision=B.AMG_MIXED))
    try:
        m = 2 * N - 1
        good = torch.zeros(m, device="cuda", dtype=torch.float64)
        bad = [torch.zeros(m, device="cuda", dtype=torch.float32),
               torch.zeros(m - 1, device="cuda", dtype=torch.float64),
               torch.zeros(2 * m, device="cuda", dtype=torch.float64)[::2],
               torch.zeros(m, dtype=torch.float64)]
        for t in bad:
            with pytest.raises(ValueError):
                B.amg_solve(h, t, good.clone(), 1e-10)
            with pytest.raises(ValueError):
                B.amg_matvec(h, good, t)
        with pytest.raises(ValueError):
            B.amg_vcycle(hm, good, good.clone())
        r32 = torch.zeros(m, device="cuda", dtype=torch.float32)
        B.amg_vcycle(hm, r32, torch.empty_like(r32))
        torch.cuda.synchronize()
    finally:
        B.amg_destroy(h)
        B.amg_destroy(hm)


@pytest.mark.parametrize("m1,m2,coarsest,wpre,wpost", [(1, 1, 5, 2 / 3, 2 / 3), (2, 2, 5, 2 / 3, 2 / 3),
                                                       (2, 1, 3, 1.0, 0.5), (1, 3, 4, 0.8, 0.6),
                                                       (1, 1, 7, 2 / 3, 2 / 3)])
@pytest.mark.parametrize("case,N", [(CONST25, 4096), (WEIGHT05, 1024)])
@pytest.mark.parametrize("cycle", [1, 2])
def test_vcycle_bottom_levels(case, N, m1, m2, coarsest, wpre, wpost, cycle):
    """The cycle's levels of at most 255 unknowns (above the coarsest; for
    W-cycles, below the small-level kernel's first level) run as one dense
    product with the matrix of that sub-cycle (for W-cycles: of all the visits
    the level receives per descent), formed at setup from the unit vectors:
    one V- or W-cycle from zero against the oracle's recursive cycle, with
    several sweep counts, damping factors and coarsest levels (coarsest 2^7:
    no level qualifies, the plain recursion)."""
    say("cycle bottom levels", case[0], N, m1, m2, coarsest, wpre, wpost, cycle)
    H = oracle_hier(case, N, coarsest)
    opts = dense.Options(m1=m1, m2=m2, omega_pre=wpre, omega_post=wpost, cycle=cycle)
    b = synthetic.random_vector(2 * N - 1, seed=N + m1 + 10 * m2)
    er = tpx.vcycle(H, b, opts)
    for prec in (B.AMG_FP64, B.AMG_MIXED):
        h = B.amg_setup(case[1], case[3], N,
                        B.amg_default_opts(precision=prec, m1=m1, m2=m2, coarsest_log2=coarsest,
                                           omega_pre=wpre, omega_post=wpost, cycle=cycle))
        try:
            dt = torch.float64 if prec == B.AMG_FP64 else torch.float32
            e = torch.empty(2 * N - 1, device="cuda", dtype=dt)
            B.amg_vcycle(h, dev(b).to(dt), e)
            err = np.abs(host(e) - er).max() / np.abs(er).max()
            tol = max(1e-13, kappa_tol(H)) if prec == B.AMG_FP64 else 1e-4
            say("prec", prec, "err", err, "tol", tol)
            assert err < tol
        finally:
            B.amg_destroy(h)
