"""The serving form (amg_server_*): requests that arrive while others are on
the GPU join the running rounds (continuous batching), and each result is
bitwise the result of the same request solved alone by amg_solve on a fresh
hierarchy.  Also: admission by device footprint under a small budget, the
cache of finished hierarchies, and the oracle's residual of the results.

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


def requests(count, seed):
    """Seeded requests shaped like the serving workload, at small sizes:
    N = 2^K (K on 10..14), delta on [0.02, 0.3], constant or weighted
    (1.2 / 0.8) kernel, tol 1e-8 or 1e-10, b ~ N(0, 1)."""
    g = synthetic.rng(seed)
    out = []
    for i in range(count):
        K = int(g.integers(10, 15))
        N = 2 ** K
        out.append(dict(N=N, delta=float(g.uniform(0.02, 0.3)), weighted=bool(g.integers(0, 2)),
                        tol=float([1e-8, 1e-10][int(g.integers(0, 2))]),
                        b=g.standard_normal(2 * N - 1)))
    return out


def kern_of(r):
    return (B.kernel(B.AMG_K_WEIGHTED, wl=1.2, wr=0.8) if r["weighted"]
            else B.kernel(B.AMG_K_CONST))


OPTS = dict(precision=B.AMG_MIXED, max_iter=100)


def solo(r):
    h = B.amg_setup(kern_of(r), r["delta"], r["N"], B.amg_default_opts(**OPTS))
    try:
        b = torch.from_numpy(r["b"]).cuda()
        x = torch.zeros_like(b)
        st, it, rel = B.amg_solve(h, b, x, r["tol"])
        return x, st, it, rel
    finally:
        B.amg_destroy(h)


@pytest.mark.parametrize("lanes", [0, 2 ** 12])
def test_serving_alone_vs_mix(lanes):
    """Twenty requests submitted in four waves, two rounds apart, so that
    later ones join rounds already running; every result equals the solo
    solve bit for bit (same kernels and arithmetic per request), with the
    same status and iteration count, and the oracle confirms the residual.
    With two lanes (N <= 2^12 on a stream of their own, three rounds per
    round of the others) the results are the same."""
    reqs = requests(20, seed=11)
    say("serving mix", lanes, [r["N"] for r in reqs])
    sv = B.amg_server_create(8 << 30, workers=3)
    if lanes:
        B.amg_server_lanes(sv, lanes, 3)
    try:
        opts = B.amg_default_opts(**OPTS)
        bs, xs, ids = [], [], {}
        for r in reqs:
            bs.append(torch.from_numpy(r["b"]).cuda())
            xs.append(torch.zeros_like(bs[-1]))
        torch.cuda.synchronize()  # the server reads b and x on its own stream
        results = {}
        for wave in range(4):
            for i in range(wave * 5, wave * 5 + 5):
                rid = B.amg_server_submit(sv, kern_of(reqs[i]), reqs[i]["delta"], reqs[i]["N"],
                                          bs[i], xs[i], reqs[i]["tol"], opts)
                ids[rid] = i
            for _ in range(2):
                B.amg_server_step(sv, 1)
                for res in B.amg_server_poll(sv):
                    results[ids[res[0]]] = res
        for _ in range(2000):
            if len(results) == len(reqs):
                break
            B.amg_server_step(sv, 1)
            for res in B.amg_server_poll(sv):
                results[ids[res[0]]] = res
        assert len(results) == len(reqs)
        stats = B.amg_server_stats(sv)
        say("stats", stats)
        for i, r in enumerate(reqs):
            xs_, st, it, rel = solo(r)
            _, st_s, it_s, rel_s, _ = results[i]
            say(i, r["N"], "solo", st, it, rel, "served", st_s, it_s, rel_s)
            assert st_s == st == B.AMG_OK and it_s == it and rel_s == rel
            assert torch.equal(xs[i], xs_), i
            if r["N"] <= 4096:
                k = (D.Kernel(D.WEIGHTED, r["delta"], wl=1.2, wr=0.8) if r["weighted"]
                     else D.Kernel(D.CONST, r["delta"]))
                T = tpx.from_stencil(k, r["N"])
                xh = xs[i].cpu().numpy()
                relo = np.linalg.norm(r["b"] - tpx.Level.build(T).matvec(xh)) / np.linalg.norm(r["b"])
                assert relo < 1.01 * r["tol"] + 1e-12, (i, relo)
    finally:
        B.amg_server_destroy(sv)


def test_serving_admission_and_cache():
    """A budget that holds one hierarchy of N = 2^13 at a time: requests wait
    for memory, the peak reservation stays within the budget, and a second
    wave of the same problems (same kernel, delta, N, options) takes the
    cached hierarchies; a third wave with another delta evicts the cached
    hierarchy and sets up in its memory.  Results still equal the solo
    solves."""
    N, delta = 2 ** 13, 0.1
    k = B.kernel(B.AMG_K_CONST)
    opts = B.amg_default_opts(**OPTS)
    fp = B.amg_footprint_bytes(k, delta, N, opts)
    say("serving admission", N, fp)
    sv = B.amg_server_create(int(fp * 1.5), workers=2)
    try:
        g = synthetic.rng(5)
        bs = [torch.from_numpy(g.standard_normal(2 * N - 1)).cuda() for _ in range(6)]
        xs = [torch.zeros_like(b) for b in bs]
        torch.cuda.synchronize()
        done = {}
        deltas = [delta] * 6 + [0.15] * 3
        bs += [torch.from_numpy(g.standard_normal(2 * N - 1)).cuda() for _ in range(3)]
        xs += [torch.zeros_like(b) for b in bs[6:]]
        torch.cuda.synchronize()
        for wave in range(3):
            for i in range(wave * 3, wave * 3 + 3):
                B.amg_server_submit(sv, k, deltas[i], N, bs[i], xs[i], 1e-10, opts)
            for _ in range(500):
                for res in B.amg_server_poll(sv):
                    done[res[0]] = res
                if len(done) == 3 * (wave + 1):
                    break
                B.amg_server_step(sv, 1)
        st = B.amg_server_stats(sv)
        say("stats", st)
        assert len(done) == 9 and all(r[1] == B.AMG_OK for r in done.values())
        assert st["peak_reserved_bytes"] <= int(fp * 1.5)
        assert st["cache_hits"] >= 3 and sum(r[4] for r in done.values()) >= 3
        assert st["evictions"] >= 1
        for d, idx in ((delta, range(6)), (0.15, range(6, 9))):
            h = B.amg_setup(k, d, N, opts)
            try:
                for i in idx:
                    x = torch.zeros_like(bs[i])
                    B.amg_solve(h, bs[i], x, 1e-10)
                    assert torch.equal(x, xs[i]), i
            finally:
                B.amg_destroy(h)
    finally:
        B.amg_server_destroy(sv)


def test_serving_rejects_unsupported():
    say("serving rejects")
    sv = B.amg_server_create(64 << 20, workers=1)
    try:
        b = torch.zeros(2 * 256 - 1, device="cuda", dtype=torch.float64)
        x = torch.zeros_like(b)
        with pytest.raises(B.AmgError):
            B.amg_server_submit(sv, B.kernel(B.AMG_K_CONST), 0.1, 256, b, x, 1e-10,
                                B.amg_default_opts(cycle=2))
        with pytest.raises(B.AmgError):
            B.amg_server_submit(sv, B.kernel(B.AMG_K_WEAKLY_SINGULAR, gamma=0.5), 0.1, 256, b, x,
                                1e-10)
        with pytest.raises(B.AmgError):
            B.amg_server_lanes(sv, 1024, 0)  # rounds outside 1..16
        with pytest.raises(B.AmgError):  # larger than the whole budget
            big = torch.zeros(2 * 2 ** 20 - 1, device="cuda", dtype=torch.float64)
            B.amg_server_submit(sv, B.kernel(B.AMG_K_CONST), 0.1, 2 ** 20, big, big.clone(), 1e-10)
    finally:
        B.amg_server_destroy(sv)
