"""C-ABI host logic of shifted operators shift*I + scale*A (Sec. 5, eq.
(bdf4)) against the oracle's shifted Toeplitz-plus-Cross hierarchy."""
from __future__ import annotations

import ctypes

import numpy as np
import pytest

from oracle import bdf4
from oracle import discretize as D
from oracle import tpx
from paper_2202_11288_amd import binding as B


@pytest.mark.parametrize("scheme", [B.AMG_SCHEME_SHIFTED, B.AMG_SCHEME_STANDARD])
@pytest.mark.parametrize("N,shift,scale", [(64, 25 / 12, 2 / 64), (1024, 25 / 12, 2 / 1024),
                                           (256, 0.0, 3.5), (512, -0.01, 1.0)])
def test_shifted_hierarchy_matches_oracle(scheme, N, shift, scale):
    osch = D.SHIFTED if scheme == B.AMG_SCHEME_SHIFTED else D.STANDARD
    kern = B.kernel(B.AMG_K_CONST, scheme=scheme)
    okern = D.Kernel(D.CONST, 0.25)
    h = B.amg_setup(kern, 0.25, N, B.amg_default_opts(flags=B.AMG_FLAG_HOST_ONLY, shift=shift,
                                                      scale=scale, coarsest_log2=4))
    try:
        Ts = [bdf4.shifted_tpx(tpx.from_stencil(okern, N, osch), shift, scale)]
        while Ts[-1].n > 2 ** 4 - 1:
            Ts.append(tpx.coarsen(Ts[-1]))
        assert B.amg_num_levels(h) == len(Ts)
        for l, To in enumerate(Ts):
            T = B.amg_level_tpx(h, l)
            sc = np.abs(To.a).max()
            for key in ("a", "b", "c", "d", "p", "q", "xi", "zeta"):
                np.testing.assert_allclose(T[key], getattr(To, key), rtol=0, atol=1e-14 * sc,
                                           err_msg=f"level {l} {key}")
            assert abs(T["o"] - To.o) <= 1e-14 * sc
    finally:
        B.amg_destroy(h)


def test_default_is_unshifted():
    o = B.amg_default_opts()
    assert o.shift == 0.0 and o.scale == 1.0


@pytest.mark.parametrize("shift,scale", [(0.0, 0.0), (0.0, -1.0), (0.0, float("nan")),
                                         (0.0, float("inf")), (float("nan"), 1.0),
                                         (float("inf"), 1.0)])
def test_bad_shift_or_scale_rejected(shift, scale):
    o = B.amg_default_opts(flags=B.AMG_FLAG_HOST_ONLY, shift=shift, scale=scale)
    h = ctypes.c_void_p()
    st = B.lib.amg_setup(ctypes.byref(B.kernel(B.AMG_K_CONST)), 0.1, 256, ctypes.byref(o), None,
                         ctypes.byref(h))
    assert st == B.AMG_EINVAL
    assert B.lib.amg_footprint_bytes(ctypes.byref(B.kernel(B.AMG_K_CONST)), 0.1, 256,
                                     ctypes.byref(o)) == B.AMG_EINVAL


def test_bdf4_step_argument_checks():
    """Host-only handles and null vectors are refused before any device work."""
    h = B.amg_setup(B.kernel(B.AMG_K_CONST), 0.1, 256, B.amg_default_opts(flags=B.AMG_FLAG_HOST_ONLY))
    try:
        fake = ctypes.c_void_p(4096)
        args = [fake] * 4 + [None, fake, 1e-10, None, None, None]
        assert B.lib.amg_bdf4_step(h, *args) == B.AMG_EINVAL
        assert B.lib.amg_bdf4_step(None, *args) == B.AMG_EINVAL
    finally:
        B.amg_destroy(h)
    with pytest.raises(ValueError):
        B.amg_bdf4_step(None, [None] * 3, None, None, 1e-10)
