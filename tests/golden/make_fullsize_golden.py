"""Write the oracle's reference solutions of the full-size workloads.

    python tests/golden/make_fullsize_golden.py rot2d      # 2D rotating, 256^2 (tens of minutes, one core)
    python tests/golden/make_fullsize_golden.py lattice3d  # 3D lattice, 128^3

Calls only ``oracle/`` and ``workloads/``.  For each workload the oracle's
Algorithm 2 (§3.2) runs from the workload's seeded initial data to the
residual 1e-6 (the raw result), then again from that state to 1e-8 (the
polish: more iterations of the same Algorithm 2, so that the energy of a
near-degenerate vortex lattice or of weakly coupled lattice wells is fixed
to far better than 1e-9 relative).  Written next to this script:

    fullsize_<name>.json      E, mu, residual, rms, max|phi|^2, evaluation
                              counts of both stages, the key below
    fullsize_<name>_phi.npz   the polished phi (complex128, x fastest): every
                              point for the 2D grid; for the 3D grid (Omega = 0,
                              a real state) its real part at every SAMPLE_3D-th
                              point of each axis, to keep the file small

The key is a SHA-256 of the problem parameters, the seed recipe and the
method's constants, so a test can tell when a reference is stale.
"""
from __future__ import annotations

import dataclasses
import hashlib
import json
import math
import os
import sys
import time

for _v in ("OPENBLAS_NUM_THREADS", "OMP_NUM_THREADS", "MKL_NUM_THREADS"):
    os.environ.setdefault(_v, "1")

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import workloads as W  # noqa: E402
from oracle.newton import Options, regularized_newton  # noqa: E402
from oracle.unified import UnifiedProblem  # noqa: E402

RAW_TOL = 1e-6
POLISH_TOL = 1e-8
SAMPLE_3D = 8

WORKLOADS = {
    "rot2d": ("workloads.rotating_2d()", W.rotating_2d),
    "lattice3d": ("workloads.lattice_3d()", W.lattice_3d),
}


def key_of(name, p, opts):
    d = {"workload": WORKLOADS[name][0],
         "problem": {k: (list(v) if isinstance(v, tuple) else v)
                     for k, v in dataclasses.asdict(p).items() if k != "v"},
         "options": dataclasses.asdict(opts), "raw_tol": RAW_TOL, "polish_tol": POLISH_TOL}
    return hashlib.sha256(json.dumps(d, sort_keys=True).encode()).hexdigest()


def summary(up, x):
    o = up.outputs(x)
    return {"energy": o["energy"], "mu": o["mu"], "resid": o["resid"], "rms": o["rms"],
            "max_dens": o["max_dens"], "norm_err": o["norm_err"]}


def run(name):
    p, phi0 = WORKLOADS[name][1]()
    up = UnifiedProblem(p)
    opts = Options(tol=RAW_TOL, max_outer=20000)
    t0 = time.time()
    raw = regularized_newton(up, up.to_x(np.asarray(phi0, dtype=np.complex128)), opts, log=True)
    t1 = time.time()
    s_raw = summary(up, raw.x)
    print(f"{name}: raw r={s_raw['resid']:.3e} E={s_raw['energy']:.12f} nfe={raw.nfe} "
          f"outer={raw.outer} {t1 - t0:.0f}s", flush=True)
    pol = regularized_newton(up, raw.x, dataclasses.replace(opts, tol=POLISH_TOL), log=True)
    t2 = time.time()
    s_pol = summary(up, pol.x)
    print(f"{name}: polished r={s_pol['resid']:.3e} E={s_pol['energy']:.12f} nfe={pol.nfe} "
          f"outer={pol.outer} {t2 - t1:.0f}s", flush=True)
    rec = {"workload": WORKLOADS[name][0], "key": key_of(name, p, opts),
           "raw": dict(s_raw, converged=raw.converged, nfe=raw.nfe, outer=raw.outer, seconds=round(t1 - t0, 1)),
           "polished": dict(s_pol, converged=pol.converged, nfe=pol.nfe, outer=pol.outer,
                            seconds=round(t2 - t1, 1)),
           "raw_log_every_50": [list(r) for r in raw.log[::50]]}
    with open(os.path.join(HERE, f"fullsize_{name}.json"), "w") as fh:
        json.dump(rec, fh, indent=1)
    save_phi(name, p, up.to_phi(pol.x))


def save_phi(name, p, phi):
    if p.dim == 3:
        phi = np.ascontiguousarray(phi[::SAMPLE_3D, ::SAMPLE_3D, ::SAMPLE_3D].real)
    np.savez_compressed(os.path.join(HERE, f"fullsize_{name}_phi.npz"), phi=phi, sample=SAMPLE_3D if p.dim == 3 else 1)


if __name__ == "__main__":
    for n in sys.argv[1:] or list(WORKLOADS):
        run(n)
