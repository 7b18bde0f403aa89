"""The entry point that allocates nothing (amg_matvec_noalloc): the same
kernels as amg_matvec with the library's static work memory.  Two calls in a
row, the second with a smaller input (and so a smaller part of the shared
array), each against amg_matvec of the same handle (bitwise) and against the
oracle's FFT matvec; then the limit and the argument checks."""
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


def test_noalloc_matvec_matches_matvec():
    cases = [(2 ** 18, B.kernel(B.AMG_K_WEIGHTED, wl=1.2, wr=0.8), D.Kernel(D.WEIGHTED, 0.05, wl=1.2, wr=0.8), 0.05),
             (2 ** 13, B.kernel(B.AMG_K_CONST), D.Kernel(D.CONST, 0.25), 0.25),
             (2 ** 10, B.kernel(B.AMG_K_FRACTIONAL, alpha=0.4), D.Kernel(D.FRACTIONAL, 0.1, alpha=0.4), 0.1)]
    for N, kern, okern, delta in cases:
        say("noalloc matvec", N)
        h = B.amg_setup(kern, delta, N)
        try:
            x = torch.from_numpy(synthetic.random_vector(2 * N - 1, seed=N)).cuda()
            y0 = torch.empty_like(x)
            y1 = torch.full_like(x, float("nan"))
            B.amg_matvec(h, x, y0)
            B.amg_matvec_noalloc(h, x, y1)
            torch.cuda.synchronize()
            assert torch.equal(y0, y1), N
            yr = tpx.Level.build(tpx.from_stencil(okern, N)).matvec(x.cpu().numpy())
            err = np.abs(y1.cpu().numpy() - yr).max() / np.abs(yr).max()
            say("err vs oracle", err)
            assert err < 1e-13
        finally:
            B.amg_destroy(h)


def test_noalloc_matvec_limits():
    say("noalloc limits")
    N = 2 ** 19
    h = B.amg_setup(B.kernel(B.AMG_K_CONST), 0.25, N)
    try:
        x = torch.zeros(2 * N - 1, device="cuda", dtype=torch.float64)
        with pytest.raises(B.AmgError) as ei:
            B.amg_matvec_noalloc(h, x, torch.empty_like(x))
        assert ei.value.status == B.AMG_EINVAL
        import ctypes
        s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        assert B.lib.amg_matvec_noalloc(None, None, None, s) == B.AMG_EINVAL
        assert B.lib.amg_matvec_noalloc(h, ctypes.c_void_p(x.data_ptr()),
                                        ctypes.c_void_p(x.data_ptr()), s) == B.AMG_EINVAL
    finally:
        B.amg_destroy(h)
