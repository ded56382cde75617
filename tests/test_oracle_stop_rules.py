"""Oracle: the paper's step-length stop rules and the monotone line search (§3.1, §4).

crit1 ||X^{k+1} - X^k||_inf / tau_k <= eps0 stops Algorithm 1; crit2
||X^{k+1} - X^k||_inf <= delta0 stops Algorithm 2 on an accepted Newton step.
The printed results of §4.1 (sine, eps0 = 1e-12) and of Table 6 (Algorithm 2,
crit2 with delta0 = 1e-8) were produced with these rules.
"""
import math

import numpy as np

import workloads as W
from oracle import discretization as disc
from oracle.feasible import feasible_gradient
from oracle.newton import Options, feasible_only, regularized_newton
from oracle.unified import UnifiedProblem

from conftest import read_golden


def _harmonic_1d_sine(lattice):
    p = W.Problem(dim=1, n=(256,), lo=(-16.0,), hi=(16.0,), bc="sine",
                  beta=250.0 if lattice else 400.0, lattice_amp=25.0 if lattice else 0.0)
    xs = disc.axis_points(p, 0)
    return p, np.exp(-xs * xs / 2)


def test_crit1_reproduces_printed_sec4_1():
    # §4.1 runs the sine discretization with crit1 at eps0 = 1e-12
    for lattice, golden in ((False, "sec4_1_case1.txt"), (True, "sec4_1_case2.txt")):
        p, f0 = _harmonic_1d_sine(lattice)
        up = UnifiedProblem(p)
        res = feasible_only(up, up.to_x(f0), Options(stop_rule="crit1", eps0=1e-12))
        assert res.converged
        out = up.outputs(res.x)
        gold = read_golden(golden)
        assert round(out["energy"], 4) == gold["energy"]
        assert round(out["mu"], 4) == gold["mu"]
        assert round(out["rms"][0], 4) == gold["x_rms"]
        assert out["resid"] < 1e-9                     # the step rule implies a small residual here


def test_crit1_special_cases():
    # eps0 = inf: the first accepted step stops the iteration; eps0 = 0: the
    # rule never holds and the iteration cap ends it
    p, f0 = _harmonic_1d_sine(False)
    up = UnifiedProblem(p)
    res = feasible_only(up, up.to_x(f0), Options(stop_rule="crit1", eps0=math.inf))
    assert res.converged and res.inner == 1
    res = feasible_only(up, up.to_x(f0), Options(stop_rule="crit1", eps0=0.0, max_iter_alg1=7))
    assert not res.converged and res.inner == 7
    # crit2 on Algorithm 1 alone: the same shape without the division by tau
    res = feasible_only(up, up.to_x(f0), Options(stop_rule="crit2", crit2_tol=math.inf))
    assert res.converged and res.inner == 1


def test_crit2_reproduces_table6():
    # Table 6 (§4.3): Algorithm 2 with crit2 (delta0 = 1e-8), Omega = 0.25,
    # initial datum (d); 128 points already resolve the printed digits
    gold = read_golden("table6_beta500.txt")
    p = W.Problem(dim=2, n=(128, 128), lo=(-10.0, -10.0), hi=(10.0, 10.0), beta=500.0, omega=0.25)
    up = UnifiedProblem(p)
    res = regularized_newton(up, up.to_x(W.phi_d(p, 0.25)), Options(stop_rule="crit2"))
    assert res.converged
    out = up.outputs(res.x)
    col = gold["omega"].index(0.25)
    assert round(out["energy"], 4) == gold["energy_d"][col]


def test_crit2_special_case():
    # crit2_tol = inf: Algorithm 2 stops at the evaluation after its first
    # accepted Newton step (a rejected step leaves X unchanged and is no step)
    p, phi0 = W.harmonic_1d(beta=400.0)
    up = UnifiedProblem(p)
    res = regularized_newton(up, up.to_x(phi0), Options(stop_rule="crit2", crit2_tol=math.inf))
    assert res.converged and res.outer == res.rejections + 1


def _accepted_energies(eta):
    p, phi0 = W.harmonic_1d(beta=400.0)
    up = UnifiedProblem(p)
    x0 = up.to_x(phi0)
    x0 = x0 / math.sqrt(float(np.vdot(x0, x0).real))
    fs = []
    f, g = up.f_and_grad(x0)

    def stop(x, f_, g_, P_):
        fs.append(f_)
        return up.residual(x, g_) < 1e-8

    feasible_gradient(up.f_and_grad, x0, f, g, maxit=5000, tau_init=1e-3, stop=stop, eta=eta)
    return np.array(fs)


def test_monotone_search_never_raises_the_energy():
    # monotone Armijo (C = F(X_k), i.e. eta = 0): F never increases beyond
    # rounding along the accepted iterates; the default Zhang-Hager search
    # (eta = 0.85) does accept increases
    mono = np.diff(_accepted_energies(0.0))
    assert np.max(mono) <= 1e-12 * 21.4
    nonmono = np.diff(_accepted_energies(0.85))
    assert np.max(nonmono) > 1e-3
    # the option maps onto eta = 0
    from oracle.newton import _fg_kwargs
    assert _fg_kwargs(Options(monotone=True))["eta"] == 0.0
