"""Benchmark: ground-state solves per second on one MI355X.

A step is one complete ground-state solve (every evaluation of the hot path:
directional spectral passes, pointwise gradient / Hessian-vector stage,
float64 reductions, retraction, BB step and trust-region control) of the
workload's problem(s) from the same initial data, with inputs resident in
HBM.  Default workload: the 2D rotating condensate (256x256 Fourier grid on
[-12,12]^2, beta = 1000, Omega = 0.9), mixed precision, residual 1e-6.

Prints one JSON line.  The timed steps run the library's default path
(chunks of evaluations replayed as hipGraphs).  Extra fields: the roofline
of the dominant kernel (the last-axis pass, timed with HIP events stamped by
the dispatch of every k-th launch of one more, untimed, solve with plain
launches), the same solve on the plain float64 path, the batched sweep of 64
rotating problems in both precisions, the H(phi)phi bandwidth of gpe_apply_h
on a 512x512x256 grid (working set above 1 GB) and on 256^3, and the float64
CPU oracle timed on a bounded sample on one core and on every core.
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

# Algorithmic bytes of the last-axis pass per grid point, the canonical fused
# pass set of the method's evaluation: the last pass reads the point and the
# accumulated transforms of the other axes and writes the gradient, 3 b for
# element size b (8 complex64, 16 complex128; half that for a real problem
# whose arrays hold real values, result storage 2).
CANON_LAST_PASS = 3

# The solver's own model of the same pass, per mode (every array it reads or
# writes once: the fused retraction, Newton model and reductions add arrays):
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


def _oracle_sample(args):
    """One bounded run of the oracle's Algorithm 2 (single-threaded numpy):
    the K_init steps of Algorithm 1, then Newton steps, stopped after about
    n_eval evaluations (each Newton step runs at most K_sub + 1)."""
    p, phi0, tol, n_eval = args
    for v in ("OPENBLAS_NUM_THREADS", "OMP_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[v] = "1"
    import numpy as np
    from oracle import newton
    from oracle.unified import UnifiedProblem
    up = UnifiedProblem(p)
    x0 = up.to_x(np.asarray(phi0, dtype=np.complex128))
    o = newton.Options(tol=tol)
    o.max_outer = max(1, (n_eval - o.k_init) // (o.k_sub + 1))
    t = time.perf_counter()
    res = newton.regularized_newton(up, x0, o)
    return time.perf_counter() - t, res.nfe


def _cpu_model():
    try:
        import subprocess
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                return line.split(":", 1)[1].strip()
    except Exception:      # lscpu missing: the model stays unnamed
        pass
    return None


def cpu_baseline(probs, phi0s, gpu_nfe, budget_s, opts):
    """The float64 oracle's Algorithm 2 on the first problem on the host:
    one process on one core for about `budget_s` seconds, then one such
    process per core at once (independent solves, the way a host would run a
    batch of problems); each leg's seconds per evaluation are scaled to
    solves/s by the evaluation count the GPU solve needed."""
    import multiprocessing as mp
    import numpy as np
    from oracle.unified import UnifiedProblem
    p, phi0 = probs[0], phi0s[0]
    up = UnifiedProblem(p)
    x0 = up.to_x(np.asarray(phi0, dtype=np.complex128))
    # probe the cost of one evaluation (after a warm-up call), then size the
    # samples to the budget
    up.f_and_grad(x0)
    t = time.perf_counter()
    for _ in range(5):
        up.f_and_grad(x0)
    per = (time.perf_counter() - t) / 5
    n_eval = max(300, int(budget_s / max(per, 1e-6)))
    dt1, nfe1 = _oracle_sample((p, phi0, opts["tol"], n_eval))
    spe1 = dt1 / max(nfe1, 1)
    ncpu = os.cpu_count() or 1
    # at most 16 worker processes (the host share a one-GPU job is given)
    cores = max(1, min(ncpu, 16))
    t = time.perf_counter()
    with mp.get_context("spawn").Pool(cores) as pool:
        runs = pool.map(_oracle_sample, [(p, phi0, opts["tol"], n_eval)] * cores)
    wall = time.perf_counter() - t
    evals = sum(n for _, n in runs)
    spe_all = wall / max(evals, 1)          # aggregate seconds per evaluation over all processes
    value1 = 1.0 / (spe1 * gpu_nfe)
    return {"value": value1, "unit": "solves/s", "cores": 1, "kind": "oracle",
            "cpu_model": _cpu_model(), "cpu_count": ncpu,
            "sample": (f"first {nfe1} float64 evaluations of Algorithm 2 on problem 0 "
                       f"({dt1:.1f} s, {1e3 * spe1:.3f} ms/evaluation, 1 thread), scaled "
                       f"by the {gpu_nfe} evaluations of the GPU solve"),
            "all_cores": {"value": 1.0 / (spe_all * gpu_nfe), "unit": "solves/s", "cores": cores,
                          "sample": (f"{cores} processes at once, each the same bounded run "
                                     f"({evals} evaluations in {wall:.1f} s of wall time, "
                                     f"{1e3 * spe_all:.3f} ms per evaluation aggregate)")}}


PLANS_FILE = os.path.join(ROOT, "profiles", "launch_plans_mi355x.json")
HPHI_BIG = (512, 512, 256)    # H(phi)phi grid with a working set above 1 GB in both precisions


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


def hphi_bandwidth(dims=(256, 256, 256), reps=20):
    """H(phi)phi throughput through gpe_apply_h on a 3D grid (the 3D lattice
    problem's potential and beta), float32 and float64.  Bytes per
    application: the canonical fused pass set (x pass: read phi, write t;
    y pass: read phi and t, write t; z pass: read phi and t, write H phi) plus
    the residual pass (read phi and H phi): 10 b M for element size b."""
    import torch
    import workloads as W
    from paper_1504_02891_amd import api
    p = W.Problem(dim=3, n=dims, lo=(-16.0,) * 3, hi=(16.0,) * 3, beta=1600.0, lattice_amp=100.0)
    m = dims[0] * dims[1] * dims[2]
    n = dims
    out = {"grid": "x".join(map(str, dims)), "bytes_per_point": "10 b (b = 8 complex64, 16 complex128)"}
    for prec, dt, b in (("mixed", torch.complex64, 8), ("fp64", torch.complex128, 16)):
        gen = torch.Generator(device="cuda").manual_seed(7)
        x = (torch.randn(n[2], n[1], n[0], dtype=torch.float64, device="cuda", generator=gen) + 0j).to(dt)
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
        torch.cuda.synchronize()
        del x, hx
    return out


def install_plans(api, probs, precs, levels, retune):
    """Launch plans (untimed): the plans gpe_autotune picked for these grids on
    MI355X, recorded in PLANS_FILE, so that every run tiles the grids alike
    and follows the same trajectory (the autotuner's choice between plans
    within a few per cent of each other changes with timing noise, and the
    tiling sets the order of the reductions); grids without a recorded plan,
    or all with `retune`, are tuned here.  A mixed solve's FP64 continuation
    and the fp64 comparison solve take the FP64 plans."""
    recorded = {}
    if not retune and os.path.exists(PLANS_FILE):
        recorded = json.load(open(PLANS_FILE))["plans"]
    plans = {}
    for p0 in probs:
        for lvl in range(levels):      # every level's grid
            p = p0.with_n([n << lvl for n in p0.n]) if lvl else p0
            for prec in precs:
                key = (prec, tuple(p.n[: p.dim]), getattr(p, "bc", "fourier"))
                if key in plans:
                    continue
                rec = recorded.get(f"{prec} {'x'.join(map(str, key[1]))} {key[2]}")
                if rec is not None:
                    api.set_plan(p, prec, rec["threads"], rec["step_at"], rec.get("elems"))
                    plans[key] = dict(rec, source="recorded")
                else:
                    plans[key] = dict(api.autotune(p, prec), source="tuned")
    return {f"{k[0]} {'x'.join(map(str, k[1]))} {k[2]}": v for k, v in plans.items()}


def roofline(a, probs, results, cascade):
    """Roofline of the final pass from one profiled solve: algorithmic bytes
    per launch divided by the event-timed average launch duration (every k-th
    launch sampled).  The algorithmic bytes are the canonical last pass's,
    3 b per point with b the element size of the instance that ran (a mixed
    solve's evaluations after the FP64 handover run the FP64 instance); the
    solver's own per-mode byte model of the pass is given beside it."""
    import numpy as np
    mb, m64 = FINAL_BYTES["mixed"], FINAL_BYTES["fp64"]
    pts = [int(np.prod(p.n[: p.dim])) for p in probs]
    byt = canon = 0.0
    nlaunch = launches = 0
    ms = 0.0
    ev32 = ev64 = 0
    for rs in results:
        for r, m in zip(rs, pts):
            h = 0.5 if r["storage"] == 2 else 1.0     # real values, two points to an element
            for k, key in enumerate(("nfe_f", "nfe_w", "nfe_outer")):
                mode = key[4]
                n32 = r["nfe_mixed"][k]
                byt += h * m * (n32 * mb[mode] + (r[key] - n32) * m64[mode])
                canon += h * m * CANON_LAST_PASS * (8 * n32 + 16 * (r[key] - n32))
                ev32 += n32
                ev64 += r[key] - n32
        nlaunch += max(r["nfe"] for r in rs)
        launches += rs[0]["pass_launches"]
        ms += rs[0]["pass_ms"]
    avg_ms = ms / max(launches, 1)
    bpl, cpl = byt / max(nlaunch, 1), canon / max(nlaunch, 1)
    ok = launches > 0 and not cascade
    # (cascade: the result counters add the evaluations of four grid sizes,
    # so no per-launch byte count; the single-grid workloads carry the line)
    ach = cpl / (avg_ms * 1e-3) / 1e9 if ok else None
    mach = bpl / (avg_ms * 1e-3) / 1e9 if ok else None
    return {"bound": "hbm", "achieved": None if ach is None else round(ach, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": None if ach is None else round(ach / HBM_PEAK_GBS, 4),
            "traffic": recorded_traffic(a.workload, ev32, ev64),
            "kernel": "k_solver_pass<R_FINAL>", "evaluations": {"fp32_instance": ev32, "fp64_instance": ev64},
            "avg_launch_us": round(avg_ms * 1e3, 3),
            "timing": (f"dispatch-stamped HIP events on every {a.profile_every}th launch of one profiled solve "
                       "(plain launches) after the timed steps"),
            "timed_launches": launches, "launches": nlaunch,
            "bytes_per_launch": None if not ok else round(cpl),
            "bytes_model": "canonical last pass: read the point and the other axes' transforms, write the "
                           "gradient, 3 b per point",
            "solver_model_bytes_per_launch": None if not ok else round(bpl),
            "solver_model_frac": None if mach is None else round(mach / HBM_PEAK_GBS, 4)}


def batch_leg(api, torch, np, opts):
    """The batched sweep (64 rotating problems on 64^2/128^2/256^2, one launch
    sequence for all): one solve in each precision."""
    import workloads as W
    probs, phi0s = W.rotating_sweep_2d()
    phis = [torch.from_numpy(np.asarray(f, dtype=np.complex128)).cuda() for f in phi0s]
    install_plans(api, probs, ("mixed", "fp64"), 1, False)
    out = {"workload": "64 rotating 2D problems, 64^2/128^2/256^2 on [-12,12]^2, beta U[100,2000], "
                       "Omega U[0,0.95], one batch"}
    for prec in ("mixed", "fp64"):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, rs = api.solve_batched(probs, phis, **dict(opts, precision=prec))
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out[prec] = {"value": round(len(probs) / dt, 4), "unit": "solves/s", "seconds": round(dt, 2),
                     "converged": sum(r["status"] == 0 for r in rs), "max_nfe": max(r["nfe"] for r in rs),
                     "fp32_evaluations": int(sum(sum(r["nfe_mixed"]) for r in rs)),
                     "evaluations": int(sum(r["nfe"] for r in rs))}
    return out


def lattice_leg(api, torch, np, a, opts):
    """The 3D lattice (128^3, real data: the solver's real storage), the
    bandwidth-heavy single-grid workload: timed solves in each precision and
    the final pass's roofline from one profiled mixed solve."""
    probs, phi0s, desc = workload("lattice3d")
    phis = [torch.from_numpy(np.asarray(f, dtype=np.complex128)).cuda() for f in phi0s]
    install_plans(api, probs, ("mixed", "fp64"), 1, False)
    out = {"workload": desc}
    for prec, reps in (("mixed", 3), ("fp64", 2)):
        o = dict(opts, precision=prec)
        api.solve(probs[0], phis[0], **o)                  # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            _, r = api.solve(probs[0], phis[0], **o)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out[prec] = {"value": round(reps / dt, 4), "unit": "solves/s", "converged": r["status"] == 0,
                     "nfe": r["nfe"], "fp32_evaluations": int(sum(r["nfe_mixed"])), "storage": r["storage"],
                     "energy": r["energy"], "resid": r["resid"]}
    if a.profile_every > 0:
        la = argparse.Namespace(workload="lattice3d", profile_every=a.profile_every)
        _, r = api.solve(probs[0], phis[0], **dict(opts, precision="mixed", profile=a.profile_every, use_graph=0))
        out["roofline"] = roofline(la, probs, [[r]], False)
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
                    help="in the profiled solve, time every k-th launch of the final pass with HIP events "
                         "(coprime with the 64-evaluation chunk, so the samples cover every position in a "
                         "chunk: the first evaluations after a host check run slower); 0: no profiled solve")
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
    ap.add_argument("--no-batch", action="store_true", help="skip the batched sweep (both precisions)")
    ap.add_argument("--no-hphi", action="store_true", help="skip the H(phi)phi bandwidth measurement")
    ap.add_argument("--only-hphi", action="store_true", help="only the H(phi)phi bandwidth measurement")
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
        print(json.dumps({"hphi": hphi_bandwidth(HPHI_BIG), "hphi_256": hphi_bandwidth()}), flush=True)
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

    # one step: a full solve of the workload; profile > 0 gives the profiled
    # variant (plain launches, every k-th final pass timed by events stamped
    # by its own dispatch; graph replay would need event nodes, which add
    # their packets' time to the interval)
    def step(profile=0):
        kw = dict(opts, profile=profile, use_graph=0 if profile else 1)
        if cascade:
            outs, rs = api.solve_cascadic(probs, phis, CASCADE[1], level_tol=CASCADE_LEVEL_TOL, **kw)
            return rs
        if len(probs) == 1:
            out, r = api.solve(probs[0], phis[0], **kw)
            return [r]
        outs, rs = api.solve_batched(probs, phis, **kw)
        return rs

    plans = {}
    if not a.no_autotune:
        plans = install_plans(api, probs, ("mixed", "fp64") if a.precision == "mixed" else ("fp64",),
                              CASCADE[1] if cascade else 1, a.retune)
    for _ in range(a.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results = []
    for _ in range(a.steps):
        results.append(step())
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    nsolves = a.steps * len(probs)
    value = nsolves / dt
    last = results[-1]
    conv = all(r["status"] == 0 for rs in results for r in rs)
    same = all(r["nfe"] == l["nfe"] for rs in results for r, l in zip(rs, last))
    pts = [int(np.prod(p.n[: p.dim])) for p in probs]
    roof = None
    if a.profile_every > 0:
        roof = roofline(a, probs, [step(a.profile_every)], cascade)

    ev = sum(sum(r["nfe_mixed"]) for r in last)
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
        "same_trajectory_every_step": same,
        "nfe_per_solve": [r["nfe"] for r in last],
        "fp32_share_of_evaluations": round(ev / max(1, sum(r["nfe"] for r in last)), 4),
        "energy": [r["energy"] for r in last][:4],
        "resid": [r["resid"] for r in last][:4],
        "roofline": roof,
        "launch_plans": plans,
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
    if a.workload == "rot2d" and not a.no_batch:
        out["batch2d"] = batch_leg(api, torch, np, dict(tol=a.tol, max_outer=a.max_outer))
        out["lattice3d"] = lattice_leg(api, torch, np, a, dict(tol=a.tol, max_outer=a.max_outer))
    if not a.no_hphi:
        out["hphi"] = hphi_bandwidth(HPHI_BIG)
        out["hphi_256"] = hphi_bandwidth()
    if not a.no_cpu_baseline and not cascade:      # the oracle's sample is one grid's Algorithm 2
        out["cpu_baseline"] = cpu_baseline(probs, phi0s, last[0]["nfe"], a.cpu_budget, opts)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
