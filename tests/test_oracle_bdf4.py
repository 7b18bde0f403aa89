"""Pins of the BDF4 oracle (Sec. 5, eq. (bdf4)) against the paper's printed
errors (Tables TT01, TT02) and against the dense form."""
from __future__ import annotations

import json
import os

import numpy as np
import pytest

from oracle import bdf4
from oracle import discretize as D
from oracle import tpx

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "bdf4_tables.json")))
SCHEME = {"shifted": D.SHIFTED, "standard": D.STANDARD}


def _delta(col, N):
    return 0.25 if col == "delta=1/4" else bdf4.paper_delta_sqrt_h(N)


def _close_to_printed(value, printed):
    """Within 1.5 units of the printed fifth significant digit."""
    unit = 10.0 ** (np.floor(np.log10(printed)) - 4)
    return abs(value - printed) <= 1.5 * unit


CASES = [(tab, col, i) for tab in ("TT01", "TT02") for col in ("delta=1/4", "delta=sqrt(h)")
         for i in range(4)]


@pytest.mark.parametrize("tab,col,i", CASES, ids=[f"{t}-{c}-N{GOLDEN['N'][i]}" for t, c, i in CASES])
def test_dense_bdf4_reproduces_paper_errors(tab, col, i):
    """All sixteen max-norm errors of Tables TT01 and TT02 to the printed
    digits: this pins both collocation rules, the non-zero volume data, the
    kernel constant, the right-hand side and the BDF4 recurrence together."""
    N = GOLDEN["N"][i]
    kern = D.Kernel(D.CONST, _delta(col, N))
    scheme = SCHEME[GOLDEN["tables"][tab]["scheme"]]
    printed = GOLDEN["tables"][tab][col]["error"][i]
    err = bdf4.run_dense(kern, N, scheme).error
    assert _close_to_printed(err, printed), (err, printed)


def test_planted_mistakes_break_the_pin():
    """A dropped history term, a wrong kernel constant or the shifted rule in
    place of the standard one each move the N = 64 error off the printed one."""
    kern = D.Kernel(D.CONST, 0.25)
    printed = GOLDEN["tables"]["TT02"]["delta=1/4"]["error"][1]
    assert not _close_to_printed(bdf4.run_dense(kern, 64, D.STANDARD, scale=1.0).error, printed)
    assert not _close_to_printed(bdf4.run_dense(kern, 64, D.SHIFTED).error, printed)
    saved = bdf4.BDF4
    try:
        bdf4.BDF4 = (4.0, -3.0, 4.0 / 3.0, 0.0)
        assert not _close_to_printed(bdf4.run_dense(kern, 64, D.STANDARD).error, printed)
    finally:
        bdf4.BDF4 = saved


def test_shifted_tpx_is_shift_plus_scaled_dense():
    kern = D.Kernel(D.WEIGHTED, 0.1, wl=1.2, wr=0.8)
    N = 64
    T = tpx.from_stencil(kern, N, D.STANDARD)
    Ts = bdf4.shifted_tpx(T, 25 / 12, 0.03)
    np.testing.assert_allclose(Ts.dense(), 25 / 12 * np.eye(2 * N - 1) + 0.03 * T.dense(),
                               rtol=0, atol=1e-15 * np.abs(T.dense()).max())
    # Lemma 3.1 on the shifted level equals the dense Galerkin R A P of it
    from oracle import dense
    Hd = dense.build_hierarchy(Ts.dense(), 4)
    Tl = Ts
    for l in range(1, Hd.nlevels):
        Tl = tpx.coarsen(Tl)
        np.testing.assert_allclose(Tl.dense(), Hd.A[l], rtol=0, atol=1e-13 * np.abs(Hd.A[0]).max())


def test_source_equals_dense_exterior_coupling():
    kern = D.Kernel(D.CONST, 0.25)
    N, tau, t = 64, 1 / 64, 0.5
    A, E, q = D.assemble_with_exterior(kern, N, D.STANDARD)
    s = bdf4.paper_scale(kern)
    x = D.points_block(N)
    ref = tau * (bdf4.forcing(kern, s, t, x) - s * E @ bdf4.exact(t, q / (2.0 * N)))
    np.testing.assert_allclose(bdf4.source(kern, N, D.STANDARD, s, tau, t), ref, rtol=1e-13,
                               atol=1e-13 * np.abs(ref).max())


@pytest.mark.parametrize("scheme", [D.SHIFTED, D.STANDARD])
def test_iterative_bdf4_matches_dense(scheme):
    """V-cycle iteration on the shifted hierarchy, tol 1e-13 per step, gives
    the dense run's solution (and therefore the paper's error)."""
    kern = D.Kernel(D.CONST, 0.25)
    N = 64
    rd = bdf4.run_dense(kern, N, scheme)
    ri = bdf4.run_tpx(kern, N, scheme, tol=1e-13, coarsest_log2=4)
    assert np.abs(ri.U - rd.U).max() <= 1e-9 * np.abs(rd.U).max()
    assert abs(ri.error - rd.error) <= 1e-3 * rd.error
    assert max(ri.iters) <= 20
