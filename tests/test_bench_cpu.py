"""bench.py's host logic on the CPU: the one-GPU contract, the seeded
workload generators behind the batch and serving legs, and the kernel-trace
summary (no device is touched)."""
import math
import os
import subprocess
import sys

import numpy as np

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_a_message():
    """One GPU: --gpus 2 (or a launcher's WORLD_SIZE > 1) ends with status 2
    and says so, before any device work."""
    for argv, env in ((["--gpus", "2"], {}), ([], {"WORLD_SIZE": "2"})):
        r = subprocess.run([sys.executable, "bench.py", *argv], cwd=ROOT, capture_output=True,
                           text=True, timeout=300, env=dict(os.environ, **env))
        assert r.returncode == 2, (argv, r.returncode, r.stderr[-500:])
        assert "one MI355X" in r.stderr and r.stdout.strip() == ""


def test_batch_instances_are_the_stated_workload():
    """512 instances, seed 0: N = 2^K with K on 10..16, delta on [0.05,
    0.3], constant or fractional, alpha on [0.2, 0.8] (the near-field rule
    from 1/2 on), b ~ N(0,1); the same list on every call."""
    a, b = bench.batch_instances(512), bench.batch_instances(512)
    assert len(a) == 512
    for x, y in zip(a, b):
        assert (x["N"], x["delta"], x["frac"], x["alpha"]) == (y["N"], y["delta"], y["frac"], y["alpha"])
        assert np.array_equal(x["b"], y["b"])
    Ks = {int(math.log2(d["N"])) for d in a}
    assert Ks == set(range(10, 17))
    assert all(0.05 <= d["delta"] <= 0.3 and 0.2 <= d["alpha"] <= 0.8 for d in a)
    assert all(d["b"].shape == (2 * d["N"] - 1,) for d in a)
    frac = [d for d in a if d["frac"]]
    near = [d for d in frac if d["alpha"] >= 0.5]
    assert 200 < len(frac) < 312 and 0 < len(near) < len(frac)
    assert bench.batch_workload_id(type("A", (), {"batch": 512, "tol": 1e-10})()) == {
        "instances": 512, "seed": 0, "tol": 1e-10, "alpha": [0.2, 0.8]}


def test_serve_requests_are_the_stated_workload():
    """Poisson arrivals at 200/s for 60 s (seed 1): about 12,000 requests,
    increasing times, N = 2^K with K on 12..22, delta on [0.02, 0.3], tol
    1e-8 or 1e-10; the mean gap is 1/rate."""
    r = bench.serve_requests(60.0, 200.0)
    assert abs(len(r) - 12000) < 4 * math.sqrt(12000)
    t = np.array([x["t"] for x in r])
    assert np.all(np.diff(t) > 0) and t[-1] < 60.0
    assert abs(np.diff(t).mean() - 1 / 200) < 0.1 / 200
    assert {x["K"] for x in r} == set(range(12, 23))
    assert all(0.02 <= x["delta"] <= 0.3 and x["tol"] in (1e-8, 1e-10) for x in r)
    assert 0.45 < np.mean([x["weighted"] for x in r]) < 0.55
    assert r == bench.serve_requests(60.0, 200.0)


def test_rocprof_summary_groups_by_kernel_and_grid(tmp_path, capsys):
    """Call counts and average durations per (kernel, grid size) from a
    kernel-trace CSV, largest share first."""
    p = tmp_path / "trace.csv"
    rows = ["Kernel_Name,Grid_Size_X,Start_Timestamp,End_Timestamp"]
    rows += [f'"void amg::k_a<float>(int)",1024,{i * 100},{i * 100 + 30}' for i in range(4)]
    rows += [f'"void amg::k_a<float>(int)",2048,{1000 + i * 100},{1000 + i * 100 + 10}' for i in range(2)]
    rows += ['"void amg::k_b(double*)",256,5000,5100']
    p.write_text("\n".join(rows) + "\n")
    bench.rocprof_summary(str(p))
    out = capsys.readouterr().out.splitlines()
    body = [l.split() for l in out[1:-1]]
    # 4 x 30 ns, 1 x 100 ns, 2 x 10 ns of 240 ns
    assert [b[-4:] for b in body] == [["1024", "4", "0.03", "50.00"], ["256", "1", "0.10", "41.67"],
                                      ["2048", "2", "0.01", "8.33"]]
    assert out[-1] == "total kernel time 0.00 ms over 7 dispatches"
