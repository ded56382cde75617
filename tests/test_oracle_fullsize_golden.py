"""The stored full-size oracle references are current and what the oracle
says: their key matches the workloads and the method's constants, the 2D
reference state has the stored energy and a residual below 1e-8 when the
oracle evaluates it again, and the raw (1e-6) and polished (1e-8) results are
consistent."""
import importlib.util
import json
import os

import numpy as np
import pytest

from oracle.newton import Options
from oracle.unified import UnifiedProblem

HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = os.path.join(HERE, "golden")


def _maker():
    spec = importlib.util.spec_from_file_location("make_fullsize_golden",
                                                  os.path.join(GOLD, "make_fullsize_golden.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


@pytest.mark.parametrize("name", ["rot2d", "lattice3d"])
def test_fullsize_reference_is_current_and_consistent(name):
    path = os.path.join(GOLD, f"fullsize_{name}.json")
    if not os.path.exists(path):
        pytest.skip(f"no reference for {name}")
    M = _maker()
    rec = json.load(open(path))
    p, _ = M.WORKLOADS[name][1]()
    assert rec["key"] == M.key_of(name, p, Options(tol=M.RAW_TOL, max_outer=20000))
    raw, pol = rec["raw"], rec["polished"]
    assert raw["converged"] and pol["converged"]
    assert raw["resid"] < M.RAW_TOL and pol["resid"] <= M.POLISH_TOL
    assert abs(pol["norm_err"]) < 1e-13
    # the polish only moves along near-soft modes: the raw energy is above
    # the polished one by at most a residual-squared-sized amount
    assert pol["energy"] <= raw["energy"] + 1e-12 * abs(raw["energy"])
    arr = np.load(os.path.join(GOLD, f"fullsize_{name}_phi.npz"))
    if p.dim == 2:
        up = UnifiedProblem(p)
        o = up.outputs(up.to_x(arr["phi"]))
        assert o["resid"] <= M.POLISH_TOL
        assert abs(o["energy"] - pol["energy"]) <= 1e-12 * abs(pol["energy"])
        assert abs(o["mu"] - pol["mu"]) <= 1e-12 * abs(pol["mu"])
    else:
        assert arr["phi"].shape == tuple(n // M.SAMPLE_3D for n in reversed(p.n))
