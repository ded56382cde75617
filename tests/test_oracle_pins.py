"""Pins of the oracle's trust-region ratio, its BB and nonmonotone-search
bookkeeping and its cascade driver, each against a characterisation that does
not share the oracle's formula: a direct difference of energies, the
least-squares property of the two BB steps, the closed form of the
Zhang-Hager reference value as a weighted mean, and the composition of the
cascade from its parts (§3.1, §3.2, Algorithm 3)."""
import math

import numpy as np
import pytest
from scipy.optimize import minimize_scalar

import workloads as W
from oracle.cascade import cascadic, prolong_fourier
from oracle.feasible import feasible_gradient
from oracle.newton import Options, actual_reduction, regularized_newton
from oracle.unified import UnifiedProblem, re_dot


def _smooth_random(p, rng, amp):
    """A Gaussian with a smooth random modulation (bounded kinetic energy)."""
    c = W.coords(p)
    r2 = sum(a * a for a in c)
    mod = sum((rng.standard_normal() + 1j * rng.standard_normal()) * np.cos((k + 1) * a / 3.0)
              for k, a in enumerate(c))
    return np.exp(-r2 / 2) * (1.0 + amp * mod)


@pytest.mark.parametrize("dim,beta,omega", [(1, 400.0, 0.0), (2, 100.0, 0.0), (2, 1000.0, 0.9),
                                            (2, 5000.0, 0.5), (3, 200.0, 0.4)])
@pytest.mark.parametrize("scale", [0.3, 1e-2])
def test_actual_reduction_equals_direct_energy_difference(dim, beta, omega, scale):
    # rho's numerator (§3.2) is F(Z) - F(X_k); the oracle evaluates it in
    # difference form.  Computed directly as two energies it must agree; the
    # direct difference loses about eps * F / |F(Z) - F(X_k)| of its digits.
    n = {1: (128,), 2: (32, 32), 3: (16, 16, 16)}[dim]
    p = W.Problem(dim=dim, n=n, lo=(-8.0,) * dim, hi=(8.0,) * dim, beta=beta, omega=omega)
    up = UnifiedProblem(p)
    rng = np.random.default_rng(11 + dim)
    xk = up.to_x(_smooth_random(p, rng, 0.3))
    xk = xk / math.sqrt(re_dot(xk, xk))
    s = scale * up.to_x(_smooth_random(p, rng, 1.0)) * (0.5 + 0.5j)
    z = xk + s
    fk, gk = up.f_and_grad(xk)
    direct = up.F(z) - fk
    ared = actual_reduction(up, xk, gk, z)
    tol = 1e-12 * abs(direct) + 4e-16 * (abs(up.F(z)) + abs(fk))
    assert abs(ared - direct) <= tol, (ared, direct)


def _trace_alg1(p, seed, eta, iters=40):
    up = UnifiedProblem(p)
    x = up.to_x(W.rotating_initial(p, p.omega, seed, amp=0.05))
    x = x / math.sqrt(re_dot(x, x))
    f, g = up.f_and_grad(x)
    tr = []
    feasible_gradient(up.f_and_grad, x, f, g, maxit=iters, tau_init=1e-3, stop=lambda *a: False,
                      eta=eta, trace=tr)
    nx, a = re_dot(x, x), re_dot(x, g)
    start = {"x": x, "f": f, "g": g, "P": nx * g - a * x}
    return start, tr


def test_bb_steps_solve_their_secant_least_squares_problems():
    # §3.1: with S = X_k - X_{k-1} and W = P_k - P_{k-1}, the long BB step is
    # the tau for which S / tau fits W best and the short one the tau for which
    # tau W fits S best (signs taken so that tau > 0); the oracle alternates
    # them, long on odd k.  Each used step must minimise its own residual,
    # found here by a bounded scalar search.
    p = W.Problem(dim=2, n=(24, 24), lo=(-6.0, -6.0), hi=(6.0, 6.0), beta=300.0, omega=0.6)
    start, tr = _trace_alg1(p, 5, 0.85)
    pts = [start] + tr
    checked = 0
    for j in range(1, len(tr)):
        tau = tr[j]["tau_bb"]
        if not (1e-20 < tau < 1e20):
            continue
        S = (pts[j]["x"] - pts[j - 1]["x"]).ravel()
        Wd = (pts[j]["P"] - pts[j - 1]["P"]).ravel()
        S = np.concatenate([S.real, S.imag])
        Wd = np.concatenate([Wd.real, Wd.imag])
        sg = math.copysign(1.0, float(S @ Wd))
        if j % 2 == 1:
            res = lambda lt: float(np.sum((S * math.exp(-lt) - sg * Wd) ** 2))
        else:
            res = lambda lt: float(np.sum((S - math.exp(lt) * sg * Wd) ** 2))
        lt = math.log(tau)
        best = minimize_scalar(res, bounds=(lt - 3.0, lt + 3.0), method="bounded",
                               options={"xatol": 1e-10})
        assert abs(best.x - lt) < 1e-5, (j, tau, math.exp(best.x))
        checked += 1
    assert checked >= 30


@pytest.mark.parametrize("eta", [0.85, 0.0])
def test_nonmonotone_reference_is_weighted_mean_of_energies(eta):
    # The Zhang-Hager recursion Q_{k+1} = eta Q_k + 1,
    # C_{k+1} = (eta Q_k C_k + f_{k+1}) / Q_{k+1} from C_0 = f_0, Q_0 = 1 is the
    # mean of f_0..f_k with weights eta^(k-i); Q_k = sum_{i<=k} eta^i.  eta = 0
    # (the monotone search) gives C_k = f_k.  Every accepted step satisfies the
    # Armijo test against the previous C (no step here used all backtracks).
    p = W.Problem(dim=2, n=(24, 24), lo=(-6.0, -6.0), hi=(6.0, 6.0), beta=300.0, omega=0.6)
    start, tr = _trace_alg1(p, 6, eta)
    fs = [start["f"]] + [t["f"] for t in tr]
    c_prev, p_prev = start["f"], start["P"]
    for k, t in enumerate(tr, start=1):
        w = np.array([eta ** (k - i) for i in range(k + 1)])
        assert abs(t["C"] - float(w @ np.array(fs[: k + 1])) / float(w.sum())) <= 1e-13 * abs(t["C"])
        assert abs(t["Q"] - float(w.sum())) <= 1e-14 * t["Q"]
        assert t["m"] < 20
        assert t["f"] <= c_prev - 1e-4 * t["t"] * re_dot(p_prev, p_prev)
        assert abs(t["t"] - 0.5 * t["tau_bb"] * 0.5 ** t["m"]) <= 1e-15 * t["t"]
        c_prev, p_prev = t["C"], t["P"]


def _cascade_case():
    p = W.Problem(dim=2, n=(16, 16), lo=(-6.0, -6.0), hi=(6.0, 6.0), beta=80.0, omega=0.4)
    return p, W.rotating_initial(p, 0.4, 21, amp=0.02)


def test_cascadic_is_the_composition_of_its_levels():
    # Algorithm 3: each coarse level runs Algorithm 2 to the level tolerance,
    # its state, interpolated to the next grid, starts the next level; the
    # finest runs to the final tolerance; the output lies on the unit sphere.
    p, phi0 = _cascade_case()
    levels = (16, 32, 64)
    opts = Options(tol=1e-9)
    x, pf, res = cascadic(p, phi0, levels, opts, level_tol=1e-4)
    phi = np.asarray(phi0, dtype=np.complex128)
    for li, n in enumerate(levels):
        q = p.with_n((n, n))
        up = UnifiedProblem(q)
        o = Options(tol=1e-4 if li < len(levels) - 1 else 1e-9)
        r = regularized_newton(up, up.to_x(phi), o)
        assert r.converged
        assert r.nfe == res[li].nfe and r.outer == res[li].outer
        rr = up.outputs(r.x)["resid"]
        assert rr < o.tol
        if li < len(levels) - 1:
            assert rr > 1e-9           # coarse levels stop at their own tolerance
        phi = up.to_phi(r.x)
        if li < len(levels) - 1:
            phi = prolong_fourier(phi)
    up = UnifiedProblem(pf)
    assert pf.n == (64, 64)
    assert np.array_equal(x, up.to_x(phi) / math.sqrt(re_dot(up.to_x(phi), up.to_x(phi))))
    assert abs(re_dot(x, x) - 1.0) < 1e-14


def test_cascadic_reaches_the_fine_grid_ground_state():
    # Omega = 0: the ground state is unique, so the cascade must end where a
    # direct solve on the finest grid ends (an independent path).
    p = W.Problem(dim=2, n=(16, 16), lo=(-6.0, -6.0), hi=(6.0, 6.0), beta=60.0)
    phi0 = W.gaussian_times_noise(p, 0.05, 8) + 0j
    x, pf, _ = cascadic(p, phi0, (16, 32), Options(tol=1e-10), level_tol=1e-4)
    up = UnifiedProblem(pf)
    xs = W.coords(pf)
    direct = regularized_newton(up, up.to_x(np.exp(-(xs[0] ** 2 + xs[1] ** 2) / 2) + 0j), Options(tol=1e-10))
    assert direct.converged
    e_c, e_d = up.outputs(x)["energy"], up.outputs(direct.x)["energy"]
    assert abs(e_c - e_d) < 1e-12 * e_d
    sgn = np.sign(re_dot(x, direct.x))
    assert np.max(np.abs(sgn * x - direct.x)) / math.sqrt(up.hvol) < 1e-7
