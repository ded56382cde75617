"""Host-side behaviour of bench.py that needs no GPU."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    # the benchmark measures one GPU; larger counts exit with a message
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2, (r.returncode, r.stderr[-2000:])
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_recorded_plans_are_valid():
    # every recorded launch plan names a precision, a grid and a discretization,
    # and passes the checks gpe_set_plan makes (64, 128 or 256 threads per
    # pass, a multiple of the pass's threads per line, a fixed step placement)
    plans = json.load(open(os.path.join(ROOT, "profiles", "launch_plans_mi355x.json")))["plans"]
    assert plans
    for key, plan in plans.items():
        prec, grid, bc = key.split()
        assert prec in ("mixed", "fp64") and bc == "fourier", key
        n = [int(v) for v in grid.split("x")]
        assert plan["step_at"] in (0, 1, 2), key
        for a, na in enumerate(n):
            e = plan.get("elems", [8, 8, 8])[a]
            assert e in (4, 8), key
            t, tl = plan["threads"][a], na // e
            assert t in (64, 128, 256) and t >= tl and t % tl == 0, (key, a, t)


def test_recorded_traffic_weights_the_instances(tmp_path, monkeypatch):
    # the roofline's traffic is the evaluation-weighted mean of the two pass
    # instances' records, and null when a record needed is missing or stale
    sys.path.insert(0, ROOT)
    import bench
    rec = {}
    for prec in ("mixed", "fp64"):
        path = os.path.join(ROOT, "profiles", f"final_pass_rot2d_256_{prec}_traffic.json")
        if not os.path.exists(path):
            pytest.skip(f"no traffic record for {prec}")
        rec[prec] = json.load(open(path))["traffic_bytes_per_launch"]
    t32, t64 = bench.recorded_traffic("rot2d", 100, 0), bench.recorded_traffic("rot2d", 0, 100)
    if t32 is None or t64 is None:
        pytest.skip("the kernel sources changed since the counters were taken")
    assert t32 == round(rec["mixed"]) and t64 == round(rec["fp64"])
    assert bench.recorded_traffic("rot2d", 100, 300) == round((rec["mixed"] + 3 * rec["fp64"]) / 4)
    assert bench.recorded_traffic("lattice3d", 100, 300) is None
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.recorded_traffic("rot2d", 100, 300) is None


def test_roofline_prices_the_canonical_last_pass():
    # achieved = 3 b M per launch (b by the instance that ran) / mean event
    # time; the solver's own per-mode model is reported beside it
    sys.path.insert(0, ROOT)
    import argparse
    import bench
    import workloads as W
    p, _ = W.rotating_2d()
    r = {"nfe": 1000, "nfe_f": 100, "nfe_w": 880, "nfe_outer": 20, "nfe_mixed": [100, 300, 0],
         "pass_launches": 50, "pass_ms": 50 * 0.010, "storage": 0}
    a = argparse.Namespace(workload="harm1d", profile_every=61)
    roof = bench.roofline(a, [p], [[r]], cascade=False)
    m = 256 * 256
    canon = m * 3 * (8 * 400 + 16 * 600) / 1000
    assert roof["bytes_per_launch"] == round(canon)
    assert abs(roof["achieved"] - round(canon / 10e-6 / 1e9, 1)) < 1e-9
    assert abs(roof["frac"] - round(roof["achieved"] / 8000.0, 4)) < 1e-4
    model = m * (100 * 40 + 300 * 72 + 580 * 112 + 20 * 112) / 1000
    assert roof["solver_model_bytes_per_launch"] == round(model)
    assert bench.roofline(a, [p], [[r]], cascade=True)["achieved"] is None
    # real values two points to an element (storage 2): half the bytes of every array
    half = bench.roofline(a, [p], [[dict(r, storage=2)]], cascade=False)
    assert half["bytes_per_launch"] == round(canon / 2)
    assert half["solver_model_bytes_per_launch"] == round(model / 2)
