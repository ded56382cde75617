"""Pins of the oracle's finite-difference discretization (§2.1).

The operator is the printed tridiagonal matrix (1/h^2 on the diagonal,
-1/(2 h^2) beside it, zero boundary values) per axis.  Pinned by
* the closed-form eigenpairs of that Toeplitz matrix: sin(j l pi / N) with
  eigenvalue (2/h^2) sin^2(l pi / (2N)), and their products in 2D/3D;
* second-order consistency with -1/2 f'' for a smooth f;
* the paper's printed FD accuracy tables (§4.1 Cases I and II, §4.2 Case I):
  the discrete ground states' errors against the sine-pseudospectral ground
  state on a fine grid (the sine oracle is itself pinned to the printed
  ground-state values).
"""
import math

import numpy as np
import pytest

import workloads as W
from conftest import read_golden
from oracle import discretization as disc
from oracle.newton import Options, feasible_only
from oracle.unified import UnifiedProblem


@pytest.mark.parametrize("dims", [(16,), (16, 32), (16, 8, 32)])
def test_fd_eigenpairs_closed_form(dims):
    d = len(dims)
    lo, hi = (-3.0, -1.0, 0.5)[:d], (5.0, 2.0, 4.5)[:d]
    p = W.Problem(dim=d, n=dims, lo=lo, hi=hi, bc=W.FD, gamma=(0.0, 0.0, 0.0))
    rng = np.random.default_rng(0)
    for _ in range(4):
        ls = [int(rng.integers(1, n)) for n in dims]
        f = np.ones(p.shape)
        lam = 0.0
        for ax, (n, l) in enumerate(zip(dims, ls)):
            h = (hi[ax] - lo[ax]) / n
            j = np.arange(1, n)
            shp = [1] * d
            shp[d - 1 - ax] = n - 1
            f = f * np.sin(j * l * math.pi / n).reshape(shp)
            lam += 2.0 / h ** 2 * math.sin(l * math.pi / (2 * n)) ** 2
        assert np.max(np.abs(disc.h_lin(p, f) - lam * f)) < 1e-12 * max(1.0, lam)


def test_fd_second_order_consistency():
    # f = exp(-x^2) on (-8, 8) (zero to 1e-27 at the ends): the discrete
    # -1/2 f'' differs from the exact one by -1/2 (h^2/12) f^(4) + O(h^4),
    # largest at x = 0 where f^(4) = 12, so the error over h^2 tends to 1/2
    errs = []
    for n in (64, 128, 256, 512):
        p = W.Problem(dim=1, n=(n,), lo=(-8.0,), hi=(8.0,), bc=W.FD, gamma=(0.0,))
        x = disc.axis_points(p, 0)
        f = np.exp(-x * x)
        exact = -0.5 * (4 * x * x - 2) * f
        h = 16.0 / n
        errs.append(float(np.max(np.abs(disc.h_lin(p, f) - exact))) / (h * h))
    assert abs(errs[-1] - 0.5) < 2e-3 and abs(errs[-2] - 0.5) < 5e-3, errs
    assert all(errs[i] < errs[i + 1] for i in range(3)), errs      # the O(h^4) terms lower it


def _ground(p, width, tol):
    # Algorithm 1 from a Gaussian of the given width, stop r < tol; the run
    # is checked to end at the ground state by its self-consistency (mu is
    # the lowest eigenvalue of H_lin + beta |phi|^2) where the grid is small
    up = UnifiedProblem(p)
    r2 = sum((c / width) ** 2 for c in disc.grid_coords(p))
    res = feasible_only(up, up.to_x(np.exp(-r2 / 2)), Options(tol=tol, max_iter_alg1=100000))
    assert res.converged
    return up, up.outputs(res.x), np.abs(res.x) / math.sqrt(up.hvol)


def _lowest(p, phi):
    m = phi.size
    H = np.zeros((m, m))
    for k in range(m):
        e = np.zeros(m)
        e[k] = 1.0
        H[:, k] = disc.h_lin(p, e.reshape(p.shape)).ravel()
    H += np.diag(p.beta * phi.ravel() ** 2)
    return float(np.linalg.eigvalsh(H)[0])


@pytest.mark.parametrize("case,amp,beta", [(1, 0.0, 400.0), (2, 25.0, 250.0)])
def test_fd_accuracy_tables_1d(case, amp, beta):
    gold = read_golden("fd_accuracy_1d.txt")
    ps = W.Problem(dim=1, n=(512,), lo=(-16.0,), hi=(16.0,), bc=W.SINE, beta=beta, lattice_amp=amp)
    _, og, phig = _ground(ps, 2.0, 1e-11)
    for k, h in enumerate(gold["h"]):
        n = int(round(32 / h))
        p = W.Problem(dim=1, n=(n,), lo=(-16.0,), hi=(16.0,), bc=W.FD, beta=beta, lattice_amp=amp)
        _, o, phi = _ground(p, 2.0, 1e-11)
        assert abs(o["mu"] - _lowest(p, phi)) < 1e-8 * o["mu"]      # the ground state
        s = 512 // n
        got = {"phi": float(np.max(np.abs(phi - phig[s - 1::s][: n - 1]))),
               "energy": abs(og["energy"] - o["energy"]), "mu": abs(og["mu"] - o["mu"])}
        # three printed digits; the h = 1/8 column lies 1.5-1.8% below ours
        # (ours falls exactly fourfold from h = 1/4), hence 2.5%
        for key, v in got.items():
            ref = gold[f"case{case}_{key}"][k]
            assert abs(v - ref) <= 0.025 * ref, (case, h, key, v, ref)


def test_fd_accuracy_table_3d():
    gold = read_golden("fd_accuracy_3d.txt")
    box = ((-8.0, 8.0), (-6.0, 6.0), (-4.0, 4.0))
    mk = lambda n, bc: W.Problem(dim=3, n=(n,) * 3, lo=tuple(b[0] for b in box), hi=tuple(b[1] for b in box),
                                 bc=bc, beta=200.0, gamma=(1.0, 2.0, 4.0))
    _, og, phig = _ground(mk(64, W.SINE), 2.0, 1e-10)
    for k, h in enumerate(gold["h"]):
        n = int(round(16 / h))
        _, o, phi = _ground(mk(n, W.FD), 2.0, 1e-10)
        s = 64 // n
        ref = phig[s - 1::s, s - 1::s, s - 1::s][: n - 1, : n - 1, : n - 1]
        got = {"phi": float(np.max(np.abs(phi - ref))),
               "energy": abs(og["energy"] - o["energy"]), "mu": abs(og["mu"] - o["mu"])}
        # h = 1 agrees to 0.4%; the h = 1/2 column lies 1.2-1.6% below ours
        for key, v in got.items():
            ref_v = gold[f"case1_{key}"][k]
            assert abs(v - ref_v) <= 0.025 * ref_v, (h, key, v, ref_v)
