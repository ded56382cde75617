"""Benchmark: ground-state solves per second on one MI355X.

A step is one complete ground-state solve (every evaluation of the hot path:
directional spectral passes, pointwise gradient / Hessian-vector stage,
float64 reductions, retraction, BB step and trust-region control) of the
workload's problem(s) from the same initial data, with inputs resident in
HBM.  Default workload: the 2D rotating condensate (256x256 Fourier grid on
[-12,12]^2, beta = 1000, Omega = 0.9), mixed precision, residual 1e-6.

Prints one JSON line.  Extra fields: the roofline of the dominant kernel
(the last-axis pass, timed with HIP events stamped by the dispatch of every
k-th launch during the timed steps), the same solve on the plain
float64 path, the H(phi)phi bandwidth of gpe_apply_h on a 256^3 grid, and
the float64 CPU oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# Bytes the last-axis (final) pass must move per grid point in each mode:
# every input array read once, every output written once.
#   F-mode  : X_b, G_b, t read; Y, G_Y written                      -> 5 arrays of the iterate type
#   W-mode  : X_k, G_k (float64) + S_b, D_b, t read; S', D' written -> 2*16 + 5*b
#   outer   : X_k or X_f, S (src), t read; X_k, G_k written; S, D zeroed
FINAL_BYTES = {
    "mixed": {"f": 5 * 8, "w": 2 * 16 + 5 * 8, "o": 16 + 8 + 16 + 2 * 16 + 2 * 8},
    "fp64": {"f": 5 * 16, "w": 2 * 16 + 5 * 16, "o": 16 + 16 + 16 + 2 * 16 + 2 * 16},
}


def workload(name):
    import workloads as W
    if name == "rot2d":
        p, phi0 = W.rotating_2d()
        return [p], [phi0], "2D rotating BEC 256x256 on [-12,12]^2, beta=1000, Omega=0.9"
    if name == "harm1d":
        p, phi0 = W.harmonic_1d()
        return [p], [phi0 + 0j], "1D harmonic 512 points on [-16,16], beta=400"
    if name == "lattice3d":
        p, phi0 = W.lattice_3d()
        return [p], [phi0 + 0j], "3D optical lattice 128^3 on [-16,16]^3, beta=1600, A=100"
    if name == "batch2d":
        probs, phis = W.rotating_sweep_2d()
        return probs, phis, "64 rotating 2D problems, 64^2/128^2/256^2 on [-12,12]^2"
    if name == "cascade2d":
        probs, phis, _ = W.cascade_2d(count=CASCADE[0])
        return probs, phis, (f"{CASCADE[0]} rotating 2D problems, Omega from 0.80 in steps of 0.01, beta=5000 on "
                             f"[-20,20]^2, cascadic levels 64^2 -> {64 << (CASCADE[1] - 1)}^2 (Algorithm 3)")
    raise SystemExit(f"unknown workload {name}")


CASCADE = [16, 4]           # cascade2d: problems, levels (64^2 .. 512^2); --cascade-problems/--cascade-levels
CASCADE_LEVEL_TOL = 1e-4    # residual at which a coarse level hands over to the next


def cpu_baseline(probs, phi0s, gpu_nfe, budget_s, opts):
    """Time the float64 oracle's Algorithm 2 on the first problem for about
    `budget_s` seconds of one core, then scale to solves/s with the
    evaluation count the GPU solve needed."""
    os.environ.setdefault("OPENBLAS_NUM_THREADS", "1")
    import numpy as np
    from oracle import newton
    from oracle.unified import UnifiedProblem
    p, phi0 = probs[0], phi0s[0]
    up = UnifiedProblem(p)
    x0 = up.to_x(np.asarray(phi0, dtype=np.complex128))
    o = newton.Options(tol=opts["tol"])
    # probe the cost of one evaluation (after a warm-up call), then size the
    # sample to the budget
    up.f_and_grad(x0)
    t = time.perf_counter()
    for _ in range(5):
        up.f_and_grad(x0)
    per = (time.perf_counter() - t) / 5
    n_eval = max(300, int(budget_s / max(per, 1e-6)))
    # K_init steps, then Newton steps; their inner loops stop early on this
    # workload (about 50 evaluations per Newton step, at most K_sub = 200)
    o.max_outer = max(1, (n_eval - o.k_init) // 60)
    t = time.perf_counter()
    res = newton.regularized_newton(up, x0, o)
    dt = time.perf_counter() - t
    sec_per_eval = dt / max(res.nfe, 1)
    value = 1.0 / (sec_per_eval * gpu_nfe)
    return {"value": value, "unit": "solves/s", "cores": 1, "kind": "oracle",
            "sample": (f"first {res.nfe} float64 evaluations of Algorithm 2 on problem 0 "
                       f"({dt:.1f} s, {1e3 * sec_per_eval:.3f} ms/evaluation, 1 thread), scaled "
                       f"by the {gpu_nfe} evaluations of the GPU solve")}


PLANS_FILE = os.path.join(ROOT, "profiles", "launch_plans_mi355x.json")


def recorded_traffic(workload_name, ev32, ev64):
    """HBM bytes per final-pass launch from the committed rocprofv3 counter
    records of the pass's FP32 and FP64 instances, weighted by the evaluations
    each ran; None when a record needed is missing, for other sources or for
    another workload."""
    import hashlib
    if workload_name != "rot2d" or ev32 + ev64 == 0:
        return None
    tot = 0.0
    for prec, ev in (("mixed", ev32), ("fp64", ev64)):
        if ev == 0:
            continue
        path = os.path.join(ROOT, "profiles", f"final_pass_{workload_name}_256_{prec}_traffic.json")
        if not os.path.exists(path):
            return None
        rec = json.load(open(path))
        h = hashlib.sha256()
        for src in rec["kernel_sources"]:
            with open(os.path.join(ROOT, "paper_1504_02891_amd", "csrc", src), "rb") as fh:
                h.update(fh.read())
        if h.hexdigest() != rec["kernel_sha256"]:
            return None
        tot += ev * rec["traffic_bytes_per_launch"]
    return round(tot / (ev32 + ev64))


def hphi_bandwidth(n=256, reps=20):
    """H(phi)phi throughput through gpe_apply_h on an n^3 grid (the 3D lattice
    problem's potential and beta), float32 and float64.  Bytes per
    application: the canonical fused pass set (x pass: read phi, write t;
    y pass: read phi and t, write t; z pass: read phi and t, write H phi) plus
    the residual pass (read phi and H phi): 10 b M for element size b."""
    import torch
    import workloads as W
    from paper_1504_02891_amd import api
    p = W.Problem(dim=3, n=(n, n, n), lo=(-16.0,) * 3, hi=(16.0,) * 3, beta=1600.0, lattice_amp=100.0)
    m = n ** 3
    out = {"grid": f"{n}^3", "bytes_per_point": "10 b (b = 8 complex64, 16 complex128)"}
    for prec, dt, b in (("mixed", torch.complex64, 8), ("fp64", torch.complex128, 16)):
        gen = torch.Generator(device="cuda").manual_seed(7)
        x = (torch.randn(n, n, n, dtype=torch.float64, device="cuda", generator=gen) + 0j).to(dt)
        hx = torch.empty_like(x)
        api.apply_h(p, x, precision=prec, out=hx)          # warm-up (workspace, code objects)
        torch.cuda.synchronize()
        # back-to-back applications, every kernel (sums and residual included)
        # runs; the scalars stay on the device
        t0 = time.perf_counter()
        for _ in range(reps):
            api.apply_h(p, x, precision=prec, scalars=False, out=hx)
        torch.cuda.synchronize()
        dt_s = (time.perf_counter() - t0) / reps
        # one call with the host readback of the scalars, for the latency
        t1 = time.perf_counter()
        api.apply_h(p, x, precision=prec, out=hx)
        lat = time.perf_counter() - t1
        gbs = 10 * b * m / dt_s / 1e9
        out[prec] = {"us_per_apply": round(1e6 * dt_s, 1), "gbs": round(gbs, 1),
                     "frac": round(gbs / HBM_PEAK_GBS, 4), "us_with_readback": round(1e6 * lat, 1),
                     "working_set_mb": round(3 * b * m / 2 ** 20)}
        del x, hx
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="rot2d", choices=["rot2d", "harm1d", "lattice3d", "batch2d", "cascade2d"])
    ap.add_argument("--precision", default="mixed", choices=["mixed", "fp64"])
    ap.add_argument("--cascade-problems", type=int, default=16,
                    help="cascade2d: problems (the full configuration, 16, runs for minutes)")
    ap.add_argument("--cascade-levels", type=int, default=4, help="cascade2d: levels from 64^2 (4: up to 512^2)")
    ap.add_argument("--tol", type=float, default=None,
                    help="residual tolerance (default 1e-6; 1e-7 for cascade2d)")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--max-outer", type=int, default=20000,
                    help="Newton-step cap per solve (lower it only for short profiler runs)")
    ap.add_argument("--profile-every", type=int, default=61,
                    help="time every k-th launch of the final pass with HIP events (coprime with the "
                         "64-evaluation chunk, so the samples cover every position in a chunk: the first "
                         "evaluations after a host check run slower)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="no launch plans: the library's built-in workgroup sizes and step placement")
    ap.add_argument("--retune", action="store_true",
                    help="run gpe_autotune for every grid instead of taking the recorded plans")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--switch-resid", type=float, default=None,
                    help="mixed Algorithm 2: residual of the FP64 handover (library default 1e-4; 0: the "
                         "whole solve stays mixed)")
    ap.add_argument("--fp64-steps", type=int, default=1,
                    help="timed solves of the same workload on the plain float64 path (0: skip)")
    ap.add_argument("--no-hphi", action="store_true", help="skip the 256^3 H(phi)phi bandwidth measurement")
    ap.add_argument("--only-hphi", action="store_true", help="only the 256^3 H(phi)phi bandwidth measurement")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only copy a MIB-sized buffer 10 times (HBM counter calibration)")
    a = ap.parse_args()
    if a.copy_calibration:
        import torch
        n = a.copy_calibration * (1 << 20) // 8
        x = torch.ones(n, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        for _ in range(10):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_each_way": n * 8, "copies": 10}))
        return
    if a.only_hphi:
        print(json.dumps({"hphi": hphi_bandwidth()}), flush=True)
        return
    if a.gpus != 1:
        print(json.dumps({"error": "the benchmark measures one GPU (independent problems shard without "
                                   "communication); --gpus must be 1"}))
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1504_02891_amd import api

    CASCADE[:] = [a.cascade_problems, a.cascade_levels]
    probs, phi0s, desc = workload(a.workload)
    cascade = a.workload == "cascade2d"
    if a.tol is None:
        a.tol = 1e-7 if cascade else 1e-6
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    phis = [torch.from_numpy(np.asarray(f, dtype=np.complex128)).to(dev) for f in phi0s]
    opts = dict(tol=a.tol, precision=a.precision, max_outer=a.max_outer)
    if a.switch_resid is not None:
        opts["switch_resid"] = a.switch_resid

    # timed steps: plain launches with every k-th last-axis pass timed by
    # events stamped by its own dispatch (graph replay would need event
    # nodes, which add their packets' time to the interval)
    def step(profile):
        kw = dict(opts, profile=profile, use_graph=0 if profile else 1)
        if cascade:
            outs, rs = api.solve_cascadic(probs, phis, CASCADE[1], level_tol=CASCADE_LEVEL_TOL, **kw)
            return rs
        if len(probs) == 1:
            out, r = api.solve(probs[0], phis[0], **kw)
            return [r]
        outs, rs = api.solve_batched(probs, phis, **kw)
        return rs

    # launch plans (untimed): the plans gpe_autotune picked for these grids on
    # MI355X, recorded in PLANS_FILE, so that every run tiles the grids alike
    # and follows the same trajectory (the autotuner's choice between plans
    # within a few per cent of each other changes with timing noise, and the
    # tiling sets the order of the reductions); grids without a recorded plan,
    # or all with --retune, are tuned here.  A mixed solve's FP64 continuation
    # and the fp64 comparison solve take the FP64 plans.
    recorded = {}
    if not a.retune and os.path.exists(PLANS_FILE):
        recorded = json.load(open(PLANS_FILE))["plans"]
    plans = {}
    if not a.no_autotune:
        for p0 in probs:
            for lvl in range(CASCADE[1] if cascade else 1):      # every level's grid
                p = p0.with_n([n << lvl for n in p0.n]) if lvl else p0
                for prec in (("mixed", "fp64") if a.precision == "mixed" else ("fp64",)):
                    key = (prec, tuple(p.n[: p.dim]), getattr(p, "bc", "fourier"))
                    if key in plans:
                        continue
                    rec = recorded.get(f"{prec} {'x'.join(map(str, key[1]))} {key[2]}")
                    if rec is not None:
                        api.set_plan(p, prec, rec["threads"], rec["step_at"])
                        plans[key] = dict(rec, source="recorded")
                    else:
                        plans[key] = dict(api.autotune(p, prec), source="tuned")
    for _ in range(a.warmup):
        step(a.profile_every)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results = []
    for _ in range(a.steps):
        results.append(step(profile=a.profile_every))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    nsolves = a.steps * len(probs)
    value = nsolves / dt
    last = results[-1]
    conv = all(r["status"] == 0 for rs in results for r in rs)

    # roofline of the final pass over every timed step: algorithmic bytes per
    # launch (all problems' evaluations in that launch, by mode) divided by the
    # event-timed average launch duration (every k-th launch sampled)
    # (a mixed solve's evaluations after the FP64 handover run the FP64
    # instance of the pass: each is priced by the byte model of its precision)
    mb, m64 = FINAL_BYTES["mixed"], FINAL_BYTES["fp64"]
    pts = [int(np.prod(p.n[: p.dim])) for p in probs]
    byt, nlaunch = 0.0, 0
    launches, ms = 0, 0.0
    ev32 = ev64 = 0
    for rs in results:
        for r, m in zip(rs, pts):
            for k, key in enumerate(("nfe_f", "nfe_w", "nfe_outer")):
                mode = key[4]
                n32 = r["nfe_mixed"][k]
                byt += m * (n32 * mb[mode] + (r[key] - n32) * m64[mode])
                ev32 += n32
                ev64 += r[key] - n32
        nlaunch += max(r["nfe"] for r in rs)
        launches += rs[0]["pass_launches"]
        ms += rs[0]["pass_ms"]
    avg_ms = ms / max(launches, 1)
    bpl = byt / max(nlaunch, 1)
    achieved = bpl / (avg_ms * 1e-3) / 1e9 if launches else 0.0
    if cascade:
        # the result counters add the evaluations of all four grid sizes: no
        # per-launch byte count (the single-grid workloads carry the roofline)
        achieved, bpl = None, None
    roof = {"bound": "hbm", "achieved": None if achieved is None else round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": None if achieved is None else round(achieved / HBM_PEAK_GBS, 4),
            "traffic": recorded_traffic(a.workload, ev32, ev64),
            "kernel": "k_solver_pass<R_FINAL>", "evaluations": {"fp32_instance": ev32, "fp64_instance": ev64},
            "avg_launch_us": round(avg_ms * 1e3, 3),
            "timing": f"dispatch-stamped HIP events on every {a.profile_every}th launch of the timed steps",
            "timed_launches": launches, "launches": nlaunch,
            "bytes_per_launch": None if bpl is None else round(bpl)}

    out = {
        "metric": "ground-state solves/sec + H\u00b7\u03c6 HBM GB/s; mixed vs FP64 GPU at resid 1e-6",
        "value": round(value, 4), "unit": "solves/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": round(1e3 * dt / a.steps, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": ("f32 bulk + f64 reductions/state, then f64 from the handover residual" if a.precision == "mixed"
                  else "f64"),
        "data": "synthetic (seeded initial data of the paper's rotating/lattice workloads)",
        "config": {"workload": desc, "precision": a.precision, "tol": a.tol, "problems": len(probs),
                   "grid_points": pts},
        "converged": conv,
        "nfe_per_solve": [r["nfe"] for r in last],
        "energy": [r["energy"] for r in last][:4],
        "resid": [r["resid"] for r in last][:4],
        "roofline": roof,
        "launch_plans": {f"{k[0]} {'x'.join(map(str, k[1]))} {k[2]}": v for k, v in plans.items()},
    }
    if cascade:
        out["config"]["grid_points"] = [int(np.prod(p.n[: p.dim])) << (2 * (CASCADE[1] - 1)) for p in probs]
    if a.fp64_steps > 0 and a.precision == "mixed" and not cascade:
        o64 = dict(opts, precision="fp64")
        if len(probs) == 1:
            api.solve(probs[0], phis[0], **o64)            # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r64 = []
        for _ in range(a.fp64_steps):
            if len(probs) == 1:
                r64.append([api.solve(probs[0], phis[0], **o64)[1]])
            else:
                r64.append(api.solve_batched(probs, phis, **o64)[1])
        torch.cuda.synchronize()
        d64 = time.perf_counter() - t0
        out["fp64"] = {"value": round(a.fp64_steps * len(probs) / d64, 4), "unit": "solves/s",
                       "converged": all(r["status"] == 0 for rs in r64 for r in rs),
                       "nfe_per_solve": [r["nfe"] for r in r64[-1]],
                       "energy": [r["energy"] for r in r64[-1]][:4], "resid": [r["resid"] for r in r64[-1]][:4]}
    if not a.no_hphi:
        out["hphi"] = hphi_bandwidth()
    if not a.no_cpu_baseline and not cascade:      # the oracle's sample is one grid's Algorithm 2
        out["cpu_baseline"] = cpu_baseline(probs, phi0s, last[0]["nfe"], a.cpu_budget, opts)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
