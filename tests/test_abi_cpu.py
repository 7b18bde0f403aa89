"""The C-ABI library on a machine without a GPU: it loads, exports every
symbol include/amg.h declares, validates arguments, and its host-side setup
(product-integration generators, Lemma 3.1 levels, manufactured RHS) agrees
with the oracle (no device compute is called here)."""
import ctypes

import numpy as np
import pytest

import synthetic
from oracle import discretize as D
from oracle import tpx
from paper_2202_11288_amd import binding as B

KERNELS = [
    (B.kernel(B.AMG_K_CONST), D.Kernel(D.CONST, 0.25), 0.25),
    (B.kernel(B.AMG_K_CONST), D.Kernel(D.CONST, 0.05), 0.05),
    (B.kernel(B.AMG_K_WEIGHTED, wl=1.2, wr=0.8), D.Kernel(D.WEIGHTED, 0.05, wl=1.2, wr=0.8), 0.05),
    (B.kernel(B.AMG_K_FRACTIONAL, alpha=0.4), D.Kernel(D.FRACTIONAL, 0.1, alpha=0.4), 0.1),
    (B.kernel(B.AMG_K_FRACTIONAL, alpha=0.2), D.Kernel(D.FRACTIONAL, 0.013, alpha=0.2), 0.013),
    (B.kernel(B.AMG_K_FRACTIONAL_NEAR, alpha=0.7), D.Kernel(D.FRACTIONAL_NEAR, 0.1, alpha=0.7), 0.1),
    (B.kernel(B.AMG_K_FRACTIONAL_NEAR, alpha=0.5), D.Kernel(D.FRACTIONAL_NEAR, 0.05, alpha=0.5), 0.05),
    (B.kernel(B.AMG_K_FRACTIONAL_NEAR, alpha=0.3), D.Kernel(D.FRACTIONAL_NEAR, 0.1, alpha=0.3), 0.1),
    (B.kernel(B.AMG_K_FRACTIONAL_NEAR, alpha=0.9), D.Kernel(D.FRACTIONAL_NEAR, 0.013, alpha=0.9),
     0.013),
]
IDS = ["const-0.25", "const-0.05", "weighted-0.05", "frac-0.4", "frac-0.2-small-delta",
       "near-0.7", "near-0.5", "near-0.3", "near-0.9-small-delta"]


def test_exports_every_declared_symbol():
    names = B.declared_symbols()
    assert len(names) >= 14
    missing = [s for s in names if not hasattr(B.lib, s)]
    assert not missing, missing


@pytest.mark.parametrize("kp", KERNELS, ids=IDS)
@pytest.mark.parametrize("N", [64, 512, 4096])
def test_manufactured_rhs_matches_oracle(kp, N):
    kern, okern, delta = kp
    b = B.amg_manufactured_rhs(kern, delta, N)
    ref = D.rhs_manufactured(okern, N)
    # both evaluate f = c * (u(x) delta - (U(x+delta) - U(x))) (or its fractional
    # analogue) in closed form; the difference cancels terms of size
    # c * (delta + int u) with rounding ~eps each, so that is the scale
    scale = okern.c * (delta ** (okern.beta + 1) if okern.kind in D.FRACTIONAL_KINDS
                       else delta + 1 / 30)
    assert np.abs(b - ref).max() <= 64 * np.finfo(float).eps * scale


def _compare_levels(h, T_levels):
    assert B.amg_num_levels(h) == len(T_levels)
    for l, To in enumerate(T_levels):
        T = B.amg_level_tpx(h, l)
        assert T["n"] == To.n
        scale = np.abs(To.a).max()
        for key in ("a", "b", "c", "d", "p", "q", "xi", "zeta"):
            np.testing.assert_allclose(T[key], getattr(To, key), rtol=0, atol=1e-14 * scale,
                                       err_msg=f"level {l} {key}")
        assert abs(T["o"] - To.o) <= 1e-14 * scale


def _oracle_levels(T0, coarsest_log2):
    Ts = [T0]
    while Ts[-1].n > 2 ** coarsest_log2 - 1:
        Ts.append(tpx.coarsen(Ts[-1]))
    return Ts


@pytest.mark.parametrize("delta_h", [0.4, 0.83, 1.6])
def test_host_near_rule_short_horizons(delta_h):
    """The near-field rule where the horizon ends inside the first cell
    (delta < h/2: no far part; h/2 < delta < h: a partial far part) or in
    the second: host generators equal the oracle's."""
    N = 64
    delta = delta_h / N
    k = B.kernel(B.AMG_K_FRACTIONAL_NEAR, alpha=0.7)
    h = B.amg_setup(k, delta, N, B.amg_default_opts(flags=B.AMG_FLAG_HOST_ONLY, coarsest_log2=4))
    try:
        To = tpx.from_stencil(D.Kernel(D.FRACTIONAL_NEAR, delta, alpha=0.7), N)
        _compare_levels(h, _oracle_levels(To, 4))
    finally:
        B.amg_destroy(h)


@pytest.mark.parametrize("kp", KERNELS, ids=IDS)
@pytest.mark.parametrize("N,cl", [(64, 5), (1024, 5), (2048, 6), (128, 6)])
def test_host_setup_matches_oracle(kp, N, cl):
    """C++ generators (Gauss-Legendre / closed form) and C++ Galerkin
    recurrences equal the oracle's (binomial series / Lemma 3.1 as printed)."""
    kern, okern, delta = kp
    h = B.amg_setup(kern, delta, N, B.amg_default_opts(flags=B.AMG_FLAG_HOST_ONLY, coarsest_log2=cl))
    try:
        _compare_levels(h, _oracle_levels(tpx.from_stencil(okern, N), cl))
    finally:
        B.amg_destroy(h)


def test_host_setup_generators_kind():
    N = 256
    gA, gB, gC, gD = synthetic.random_tpx_arrays(N - 1, seed=11)
    gen = np.ascontiguousarray(np.concatenate([gA, gB, gC, gD]))
    assert gen.size == 8 * N - 8
    h = B.amg_setup(B.kernel(B.AMG_K_GENERATORS, gen=gen), 0.0, N,
                    B.amg_default_opts(flags=B.AMG_FLAG_HOST_ONLY))
    try:
        _compare_levels(h, _oracle_levels(tpx.from_blocks(gA, gB, gC, gD, N), 5))
    finally:
        B.amg_destroy(h)


def _setup_status(kern, delta, N, **opts):
    flags = B.AMG_FLAG_HOST_ONLY | opts.pop("flags", 0)
    o = B.amg_default_opts(flags=flags, **opts)
    h = ctypes.c_void_p()
    st = B.lib.amg_setup(ctypes.byref(kern), float(delta), int(N), ctypes.byref(o), None,
                         ctypes.byref(h))
    if st == B.AMG_OK:
        B.lib.amg_destroy(h)
    return st


@pytest.mark.parametrize("case", [
    dict(N=100), dict(N=0), dict(N=-64), dict(N=32), dict(N=16), dict(N=2 ** 23),
    dict(delta=0.0), dict(delta=-0.1), dict(delta=0.5), dict(delta=float("nan")),
    dict(kind=B.AMG_K_FRACTIONAL, alpha=0.5), dict(kind=B.AMG_K_FRACTIONAL, alpha=0.0),
    dict(kind=B.AMG_K_FRACTIONAL_NEAR, alpha=1.0), dict(kind=B.AMG_K_FRACTIONAL_NEAR, alpha=0.0),
    dict(kind=6),
    dict(kind=B.AMG_K_WEIGHTED, wl=-1.0), dict(kind=7), dict(kind=B.AMG_K_GENERATORS),
    dict(opts=dict(coarsest_log2=1)), dict(opts=dict(coarsest_log2=8)),
    dict(opts=dict(omega_pre=0.0)), dict(opts=dict(precision=5)), dict(opts=dict(flags=32)),
    dict(opts=dict(inner=3)), dict(opts=dict(inner=-1)),
    dict(opts=dict(inner=B.AMG_INNER_GMRES, restart=0)), dict(opts=dict(restart=65)),
    dict(opts=dict(cycle=0)), dict(opts=dict(cycle=3)),
    dict(kind=B.AMG_K_WEIGHTED, wl=1.2, opts=dict(inner=B.AMG_INNER_PCG)),
])
def test_invalid_arguments_rejected(case):
    kind = case.get("kind", B.AMG_K_CONST)
    kern = B.kernel(kind, alpha=case.get("alpha", 0.3), wl=case.get("wl", 1.0), wr=1.0)
    st = _setup_status(kern, case.get("delta", 0.1), case.get("N", 256), **case.get("opts", {}))
    assert st == B.AMG_EINVAL


def test_accurate_residual_flag():
    """AMG_FLAG_ACCURATE_RESIDUAL is accepted for the stencil kernels and
    refused (AMG_ENOTSUP) where the finest matrix is not a row stencil in the
    points' order (caller generators, the weakly singular model's band);
    its far-field spectra and near-field output count in the footprint."""
    fl = B.AMG_FLAG_ACCURATE_RESIDUAL
    for kind in (B.AMG_K_CONST, B.AMG_K_WEIGHTED, B.AMG_K_FRACTIONAL, B.AMG_K_FRACTIONAL_NEAR):
        assert _setup_status(B.kernel(kind, alpha=0.3, wl=1.2, wr=0.8), 0.1, 4096, flags=fl) == B.AMG_OK
    gen = np.zeros(8 * 256 - 8)
    gen[255 - 1] = 1.0
    assert _setup_status(B.kernel(B.AMG_K_GENERATORS, gen=gen), 0.0, 256, flags=fl) == B.AMG_ENOTSUP
    assert _setup_status(B.kernel(B.AMG_K_WEAKLY_SINGULAR, gamma=0.5), 0.1, 256,
                         flags=fl) == B.AMG_ENOTSUP
    k = B.kernel(B.AMG_K_FRACTIONAL, alpha=0.4)
    f0 = B.amg_footprint_bytes(k, 0.1, 2 ** 20)
    f1 = B.amg_footprint_bytes(k, 0.1, 2 ** 20, B.amg_default_opts(flags=fl))
    assert f1 - f0 >= 2 * 2 ** 21 * 8 + (2 ** 21 - 1) * 8


def test_unsupported_sweep_counts():
    assert _setup_status(B.kernel(B.AMG_K_CONST), 0.1, 256, m1=0) == B.AMG_ENOTSUP


def test_null_pointers_and_host_only_handle():
    assert B.lib.amg_setup(None, 0.1, 256, None, None, None) == B.AMG_EINVAL
    h = B.amg_setup(B.kernel(B.AMG_K_CONST), 0.1, 256, B.amg_default_opts(flags=B.AMG_FLAG_HOST_ONLY))
    try:
        # device entry points refuse a host-only handle without touching a GPU
        assert B.lib.amg_matvec(h, ctypes.c_void_p(8), ctypes.c_void_p(16), None) == B.AMG_EINVAL
        assert B.lib.amg_vcycle(h, ctypes.c_void_p(8), ctypes.c_void_p(16), None) == B.AMG_EINVAL
        assert B.lib.amg_level_matvec(h, 99, ctypes.c_void_p(8), ctypes.c_void_p(16), None) == B.AMG_EINVAL
        assert B.amg_level_size(h, 0) == 511 and B.amg_level_size(h, 3) == 63
        assert B.amg_level_size(h, 4) == B.AMG_EINVAL
    finally:
        B.amg_destroy(h)
    assert B.lib.amg_destroy(None) == B.AMG_OK
    assert B.lib.amg_manufactured_rhs(None, 0.1, 64, None) == B.AMG_EINVAL


def test_footprint_and_strerror():
    k = B.kernel(B.AMG_K_CONST)
    f = [B.amg_footprint_bytes(k, 0.1, 2 ** K) for K in (10, 14, 20)]
    assert all(x > 0 for x in f) and f[0] < f[1] < f[2]
    assert B.amg_footprint_bytes(k, 0.1, 1000) == B.AMG_EINVAL
    fm = B.amg_footprint_bytes(k, 0.1, 2 ** 20, B.amg_default_opts(precision=B.AMG_MIXED))
    assert fm > f[2]
    for st in (0, 1, 2, -1, -2, -3, -4):
        assert B.strerror(st) and B.strerror(st) != "unknown status"


def test_solve_batch_argument_checks():
    DP = ctypes.POINTER(ctypes.c_void_p)
    assert B.lib.amg_solve_batch(0, None, None, None, None, None, None, None) == B.AMG_OK
    assert B.lib.amg_solve_batch(-1, None, None, None, None, None, None, None) == B.AMG_EINVAL
    assert B.lib.amg_solve_batch(2, None, None, None, None, None, None, None) == B.AMG_EINVAL
    h = B.amg_setup(B.kernel(B.AMG_K_CONST), 0.1, 256, B.amg_default_opts(flags=B.AMG_FLAG_HOST_ONLY))
    try:
        hs = (ctypes.c_void_p * 1)(h.value)
        ptrs = (ctypes.c_void_p * 1)(16)
        ptrs2 = (ctypes.c_void_p * 1)(32)
        tol = (ctypes.c_double * 1)(1e-10)
        # host-only handles are refused before any device work
        assert B.lib.amg_solve_batch(1, hs, ptrs, ptrs2, tol, None, None, None) == B.AMG_EINVAL
    finally:
        B.amg_destroy(h)


def test_conjugate_gradient_option():
    """inner = AMG_INNER_PCG: accepted for the symmetric kernels (constant,
    fractional), refused for the weighted (non-symmetric) one; the default is
    the stationary iteration; the footprint counts CG's three vectors; unknown
    option names are refused by the binding."""
    assert B.amg_default_opts().inner == B.AMG_INNER_VCYCLE
    for kern in (B.kernel(B.AMG_K_CONST), B.kernel(B.AMG_K_FRACTIONAL, alpha=0.4)):
        assert _setup_status(kern, 0.1, 1024, inner=B.AMG_INNER_PCG) == B.AMG_OK
    assert _setup_status(B.kernel(B.AMG_K_WEIGHTED, wl=1.2, wr=0.8), 0.1, 1024,
                         inner=B.AMG_INNER_PCG) == B.AMG_EINVAL
    k = B.kernel(B.AMG_K_CONST)
    f0 = B.amg_footprint_bytes(k, 0.1, 2 ** 16)
    f1 = B.amg_footprint_bytes(k, 0.1, 2 ** 16, B.amg_default_opts(inner=B.AMG_INNER_PCG))
    assert f1 - f0 >= 3 * (2 * 2 ** 16 - 1) * 8
    with pytest.raises(TypeError):
        B.amg_default_opts(innr=1)


def test_gmres_option():
    """inner = AMG_INNER_GMRES: accepted for every kernel (non-symmetric ones
    included); the footprint counts its 2 restart + 1 vectors."""
    for kern in (B.kernel(B.AMG_K_CONST), B.kernel(B.AMG_K_WEIGHTED, wl=1.2, wr=0.8),
                 B.kernel(B.AMG_K_CONST, scheme=B.AMG_SCHEME_STANDARD)):
        assert _setup_status(kern, 0.1, 1024, inner=B.AMG_INNER_GMRES) == B.AMG_OK
    assert B.amg_default_opts().restart == 30
    k = B.kernel(B.AMG_K_WEIGHTED, wl=1.2, wr=0.8)
    f0 = B.amg_footprint_bytes(k, 0.1, 2 ** 16)
    for R in (1, 30, 64):
        f1 = B.amg_footprint_bytes(k, 0.1, 2 ** 16, B.amg_default_opts(inner=B.AMG_INNER_GMRES,
                                                                        restart=R))
        assert f1 - f0 >= (2 * R + 1) * (2 * 2 ** 16 - 1) * 8


def test_plan_get_set_host_logic():
    """The geometry table is host state: defaults per size, candidates only,
    reset with logL1 = 0; sizes outside 13..23 are rejected."""
    d = {lg: B.amg_plan_get(lg) for lg in range(13, 24)}
    assert d[21]["logL1"] == 11 and d[21]["tcols"] == 8 and d[21]["us_best"] == 0.0
    assert d[13]["candidates"] == 1 and d[19]["candidates"] == 6
    try:
        B.amg_plan_set(19, 11, 4)
        assert (B.amg_plan_get(19)["logL1"], B.amg_plan_get(19)["tcols"]) == (11, 4)
        with pytest.raises(B.AmgError):
            B.amg_plan_set(19, 7, 4)  # 2^7 x 2^12: no column pass instance
        with pytest.raises(B.AmgError):
            B.amg_plan_get(12)
        with pytest.raises(B.AmgError):
            B.amg_plan_set(24, 12, 4)
    finally:
        B.amg_plan_set(19)
    assert (B.amg_plan_get(19)["logL1"], B.amg_plan_get(19)["tcols"]) == (10, 4)


def test_deep_fold_footprint():
    """AMG_FLAG_DEEP_FOLD adds the dense operator of the first small level
    (2 n + 1 unknowns, FP64 plus FP32 rounding in the mixed form) to the
    footprint when the problem has levels above it; none at or below 2^11."""
    k = B.kernel(B.AMG_K_CONST)
    for N, m in ((2 ** 20, 4095), (2 ** 12, 4095), (2 ** 11, 0), (2 ** 9, 0)):
        for prec, per in ((B.AMG_FP64, 8), (B.AMG_MIXED, 12)):
            f0 = B.amg_footprint_bytes(k, 0.1, N, B.amg_default_opts(precision=prec))
            f1 = B.amg_footprint_bytes(k, 0.1, N, B.amg_default_opts(precision=prec,
                                                                     flags=B.AMG_FLAG_DEEP_FOLD))
            assert f1 - f0 == m * m * per, (N, prec)
