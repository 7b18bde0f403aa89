"""The geometry autotuner (amg_autotune) and every candidate geometry of the
level matvec: each computes the default geometry's product up to rounding
(and the oracle's at small sizes), and a solve with it converges in the
default's iteration count.  Plans are process-wide: every test restores the
defaults.

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

SIZES = range(13, 24)


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def reset():
    for lg in SIZES:
        B.amg_plan_set(lg)


def candidates(lg):
    """The candidate geometries of size 2^lg, found through amg_plan_set."""
    out = []
    for l1 in range(6, 13):
        for tc in (1, 2, 4, 8, 16, 32):
            try:
                B.amg_plan_set(lg, l1, tc)
                out.append((l1, tc))
            except B.AmgError:
                pass
    B.amg_plan_set(lg)
    return out


def test_autotune_all_sizes():
    """Every size: no candidate rejected by the tuner's product check, the
    chosen geometry is a candidate and not slower than the default."""
    say("autotune 13..23")
    try:
        B.amg_autotune(13, 23)
        for lg in SIZES:
            p = B.amg_plan_get(lg)
            say(p)
            assert p["rejected"] == 0
            assert (p["logL1"], p["tcols"]) in candidates(lg) or p["candidates"] == 1
            assert 0 < p["us_best"] <= p["us_default"]
    finally:
        reset()


@pytest.mark.parametrize("lg", [14, 16, 17, 18, 19, 20, 21, 22])
def test_candidate_geometry_matvec_and_solve(lg):
    """Each candidate geometry of size 2^lg (finest level of N = 2^(lg-1)):
    the FP64 level matvec equals the default geometry's to 1e-12 of its
    norm, the FP32 one to 1e-5 (a few FP32 rounding bounds), the oracle's to
    1e-12 at N <= 2^15, and a mixed-precision solve converges within one
    iteration of the default's count."""
    N = 2 ** (lg - 1)
    kern = B.kernel(B.AMG_K_WEIGHTED, wl=1.2, wr=0.8)
    opts = B.amg_default_opts(precision=B.AMG_MIXED, max_iter=60)
    x = torch.from_numpy(synthetic.random_vector(2 * N - 1, seed=lg)).cuda()
    b = torch.from_numpy(B.amg_manufactured_rhs(kern, 0.1, N)).cuda()

    def run():
        h = B.amg_setup(kern, 0.1, N, opts)
        try:
            y = torch.empty_like(x)
            B.amg_level_matvec(h, 0, x, y)
            y32 = torch.empty(2 * N - 1, device="cuda", dtype=torch.float32)
            B.amg_level_matvec_f32(h, 0, x.float(), y32)
            u = torch.zeros_like(b)
            st, it, rel = B.amg_solve(h, b, u, 1e-10)
            torch.cuda.synchronize()
            return y.cpu().numpy(), y32.cpu().numpy(), st, it
        finally:
            B.amg_destroy(h)

    try:
        y0, y0f, st0, it0 = run()
        ny = np.linalg.norm(y0)
        cands = candidates(lg)
        say("size", lg, "candidates", cands)
        for l1, tc in cands:
            B.amg_plan_set(lg, l1, tc)
            say("geometry", lg, l1, tc)
            y1, y1f, st1, it1 = run()
            say("diff64", np.linalg.norm(y1 - y0) / ny, "diff32", np.linalg.norm(y1f - y0f) / ny,
                "iters", it0, it1)
            assert np.linalg.norm(y1 - y0) <= 1e-12 * ny, (l1, tc)
            assert np.linalg.norm(y1f - y0f) <= 1e-5 * ny, (l1, tc)
            assert st1 == st0 == B.AMG_OK and abs(it1 - it0) <= 1, (l1, tc, it0, it1)
            if N <= 2 ** 15:
                T = tpx.from_stencil(D.Kernel(D.WEIGHTED, 0.1, wl=1.2, wr=0.8), N)
                yo = tpx.Level.build(T).matvec(x.cpu().numpy())
                assert np.linalg.norm(y1 - yo) <= 1e-12 * np.linalg.norm(yo)
    finally:
        reset()


def test_batch_mixes_geometries():
    """Hierarchies of one size set up under two geometries, solved together
    by amg_solve_batch: each result equals its own solo solve bit for bit."""
    N, lg = 2 ** 18, 19
    kern = B.kernel(B.AMG_K_CONST)
    opts = B.amg_default_opts(precision=B.AMG_MIXED, max_iter=60)
    say("batch with two geometries", lg)
    hs = []
    try:
        hs.append(B.amg_setup(kern, 0.2, N, opts))
        alt = [c for c in candidates(lg) if c != (B.amg_plan_get(lg)["logL1"], B.amg_plan_get(lg)["tcols"])]
        B.amg_plan_set(lg, *alt[0])
        hs.append(B.amg_setup(kern, 0.15, N, opts))
        reset()
        g = synthetic.rng(3)
        bs = [torch.from_numpy(g.standard_normal(2 * N - 1)).cuda() for _ in hs]
        xs = [torch.zeros_like(b) for b in bs]
        B.amg_solve_batch(hs, bs, xs, [1e-10] * 2)
        for h, b, x in zip(hs, bs, xs):
            u = torch.zeros_like(b)
            B.amg_solve(h, b, u, 1e-10)
            assert torch.equal(u, x)
    finally:
        reset()
        for h in hs:
            B.amg_destroy(h)
