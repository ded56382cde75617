"""Pins of the oracle's optimizers (Theorem 3.3, Algorithms 1-3) against the
paper's printed values, closed forms, invariants and brute-force eigensolves."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import discretization as disc
from oracle.cascade import prolong_fourier
from oracle.feasible import cayley_coefficients, cayley_point
from oracle.newton import Options, feasible_only, regularized_newton
from oracle.unified import UnifiedProblem, re_dot

from conftest import read_golden


def _embed(z):
    """C^M -> R^{2M}."""
    return np.concatenate([z.real.ravel(), z.imag.ravel()])


def test_cayley_closed_form_equals_dense_solve():
    # Theorem 3.3 in the real reading: Y = (I + tau A)^-1 (I - tau A) X with
    # A = G X^T - X G^T on R^{2M}; the closed form p X + q G must agree.
    rng = np.random.default_rng(1)
    m = 20
    x = rng.standard_normal(m) + 1j * rng.standard_normal(m)
    x /= np.linalg.norm(x)
    g = 3.0 * (rng.standard_normal(m) + 1j * rng.standard_normal(m))
    xr, gr = _embed(x), _embed(g)
    A = np.outer(gr, xr) - np.outer(xr, gr)
    for tau in (1e-3, 0.1, 2.0):
        y_dense = np.linalg.solve(np.eye(2 * m) + tau * A, (np.eye(2 * m) - tau * A) @ xr)
        y = cayley_point(x, g, tau)
        assert np.max(np.abs(_embed(y) - y_dense)) < 1e-13
        assert abs(np.linalg.norm(y) - np.linalg.norm(x)) < 1e-14


def test_cayley_preserves_unnormalised_norm_and_slope():
    # ||Y(tau)|| = ||X|| for any ||X|| (n_x explicit), and Y'(0) = -2 P.
    rng = np.random.default_rng(2)
    x = 1.7 * (rng.standard_normal(30) + 1j * rng.standard_normal(30))
    g = rng.standard_normal(30) + 1j * rng.standard_normal(30)
    for tau in (0.01, 0.3):
        assert abs(np.linalg.norm(cayley_point(x, g, tau)) - np.linalg.norm(x)) < 1e-12
    P = re_dot(x, x) * g - re_dot(x, g) * x
    t = 1e-6
    slope = (cayley_point(x, g, t) - cayley_point(x, g, -t)) / (2 * t)
    assert np.max(np.abs(slope + 2 * P)) < 1e-6 * np.max(np.abs(P))
    p0, q0 = cayley_coefficients(0.0, 1.0, 1.0, 1.0)
    assert (p0, q0) == (1.0, 0.0)


def _check_golden_1d(bc, n, golden, lattice):
    p = W.Problem(dim=1, n=(n,), lo=(-16.0,), hi=(16.0,), bc=bc,
                  beta=250.0 if lattice else 400.0, lattice_amp=25.0 if lattice else 0.0)
    up = UnifiedProblem(p)
    xs = disc.axis_points(p, 0)
    res = feasible_only(up, up.to_x(np.exp(-xs * xs / 2)), Options(tol=1e-9))
    assert res.converged
    out = up.outputs(res.x)
    gold = read_golden(golden)
    assert round(out["energy"], 4) == gold["energy"]
    assert round(out["mu"], 4) == gold["mu"]
    assert round(out["rms"][0], 4) == gold["x_rms"]


def test_alg1_fourier_reproduces_printed_case1():
    _check_golden_1d("fourier", 512, "sec4_1_case1.txt", lattice=False)


def test_alg1_sine_reproduces_printed_case1():
    _check_golden_1d("sine", 256, "sec4_1_case1.txt", lattice=False)


def test_alg1_sine_reproduces_printed_case2_lattice():
    _check_golden_1d("sine", 256, "sec4_1_case2.txt", lattice=True)


def test_alg2_harmonic_1d_matches_printed_and_alg1():
    p, phi0 = W.harmonic_1d(beta=400.0)
    up = UnifiedProblem(p)
    r2 = regularized_newton(up, up.to_x(phi0), Options(tol=1e-8))
    r1 = feasible_only(up, up.to_x(phi0), Options(tol=1e-8))
    assert r2.converged and r1.converged
    o2, o1 = up.outputs(r2.x), up.outputs(r1.x)
    gold = read_golden("sec4_1_case1.txt")
    assert round(o2["energy"], 4) == gold["energy"]
    assert round(o2["mu"], 4) == gold["mu"]
    assert round(o2["rms"][0], 4) == gold["x_rms"]
    assert abs(o2["energy"] - o1["energy"]) < 1e-12 * o1["energy"]
    assert abs(o2["mu"] - o1["mu"]) < 1e-9 * o1["mu"]
    sgn = np.sign(re_dot(r1.x, r2.x))
    assert np.max(np.abs(sgn * r2.x - r1.x)) / math.sqrt(up.hvol) < 1e-6
    assert o2["resid"] < 1e-8
    assert abs(o2["norm_err"]) < 1e-13


def test_beta0_gives_exact_harmonic_energy():
    p, phi0 = W.harmonic_1d(beta=0.0)
    up = UnifiedProblem(p)
    res = regularized_newton(up, up.to_x(phi0), Options(tol=1e-8))
    out = up.outputs(res.x)
    assert res.converged
    assert abs(out["energy"] - 0.5) < 1e-13
    assert abs(out["rms"][0] - math.sqrt(0.5)) < 1e-7


def test_virial_identity_at_convergence():
    # For phi -> lambda^{d/2} phi(lambda x) stationarity:
    # 2 E_kin - <x . grad V> + d E_int = 0, with <x.grad V> = 2 E_pot for a
    # harmonic trap.  E_kin excludes rotation (the L_z term is scale invariant).
    for p, phi0, tol in ((W.harmonic_1d()[0], W.harmonic_1d()[1], 1e-9),):
        up = UnifiedProblem(p)
        res = regularized_newton(up, up.to_x(phi0), Options(tol=tol))
        x = res.x
        p0 = W.Problem(dim=p.dim, n=p.n, lo=p.lo, hi=p.hi, gamma=(0.0, 0.0, 0.0))
        e_kin = re_dot(x, disc.kinetic(p0, x))
        e_pot = re_dot(x, up.v * x)
        e_int = up.alpha * float(np.sum(np.abs(x) ** 4))
        assert abs(2 * e_kin - 2 * e_pot + p.dim * e_int) < 1e-7


def test_thomas_fermi_limit_trend():
    # E / E_TF -> 1 from above as beta grows; 1D mu_TF = 1/2 (3 beta/2)^{2/3},
    # E_TF = 3/5 mu_TF.
    ratios = []
    for beta in (400.0, 1600.0, 6400.0):
        p = W.Problem(dim=1, n=(1024,), lo=(-32.0,), hi=(32.0,), beta=beta)
        up = UnifiedProblem(p)
        xs = disc.axis_points(p, 0)
        res = feasible_only(up, up.to_x(np.exp(-xs * xs / 50)), Options(tol=1e-7))
        e_tf = 0.6 * 0.5 * (1.5 * beta) ** (2.0 / 3.0)
        ratios.append(up.outputs(res.x)["energy"] / e_tf)
    assert ratios[0] > ratios[1] > ratios[2] > 1.0
    assert ratios[2] < 1.01


def _dense_h_lin(p):
    m = p.size
    cols = []
    for k in range(m):
        e = np.zeros(m, dtype=complex)
        e[k] = 1.0
        cols.append(disc.h_lin(p, e.reshape(p.shape)).ravel())
    return np.array(cols).T


def test_linear_rotating_ground_state_equals_dense_eigensolve():
    # beta = 0: the minimiser of F on the sphere is the lowest eigenvector of
    # the Hermitian H_lin (library eigensolver on the dense 256 x 256 matrix).
    p = W.Problem(dim=2, n=(16, 16), lo=(-5.0, -5.0), hi=(5.0, 5.0), omega=0.5)
    H = _dense_h_lin(p)
    w, V = np.linalg.eigh(H)
    up = UnifiedProblem(p)
    phi0 = W.rotating_initial(p, 0.5, 9, amp=0.05)
    res = regularized_newton(up, up.to_x(phi0), Options(tol=1e-9))
    assert res.converged
    assert abs(up.outputs(res.x)["energy"] - w[0]) < 1e-11
    v0 = V[:, 0].reshape(p.shape)
    ph = np.vdot(v0, res.x)
    assert np.max(np.abs(res.x - v0 * ph / abs(ph))) < 1e-7


def test_nonlinear_ground_state_is_lowest_mode_of_own_mean_field():
    # beta > 0, Omega = 0: the ground state is the lowest eigenvector of
    # H_lin + beta |phi|^2 with eigenvalue mu (self-consistency, brute force).
    p = W.Problem(dim=2, n=(16, 16), lo=(-6.0, -6.0), hi=(6.0, 6.0), beta=50.0)
    up = UnifiedProblem(p)
    res = regularized_newton(up, up.to_x(W.gaussian_times_noise(p, 0.05, 4)), Options(tol=1e-10))
    assert res.converged
    phi = up.to_phi(res.x)
    H = _dense_h_lin(p) + np.diag((p.beta * np.abs(phi) ** 2).ravel())
    w, V = np.linalg.eigh(H)
    assert abs(w[0] - up.outputs(res.x)["mu"]) < 1e-9
    v0 = V[:, 0].reshape(p.shape)
    ph = np.vdot(v0, res.x)
    assert np.max(np.abs(res.x - v0 * ph / abs(ph))) < 1e-8
    assert w[1] - w[0] > 0.1


def test_second_order_condition_at_rotating_minimiser():
    # Lemma 3.2: Hess F[D,D] - theta ||D||^2 >= 0 on the tangent space, checked
    # on the dense real 2M x 2M Hessian of a converged rotating state.
    p = W.Problem(dim=2, n=(12, 12), lo=(-5.0, -5.0), hi=(5.0, 5.0), beta=40.0, omega=0.4)
    up = UnifiedProblem(p)
    res = regularized_newton(up, up.to_x(W.rotating_initial(p, 0.4, 3, amp=0.05)),
                             Options(tol=1e-10))
    x = res.x
    f, g = up.f_and_grad(x)
    theta = re_dot(x, g)
    m = p.size
    cols = []
    for k in range(2 * m):
        d = np.zeros(m, dtype=complex)
        d[k % m] = 1.0 if k < m else 1j
        cols.append(_embed(up.hess(x, d.reshape(p.shape))))
    Hr = np.array(cols).T
    assert np.max(np.abs(Hr - Hr.T)) < 1e-9 * np.max(np.abs(Hr))
    xr = _embed(x)
    Q = np.linalg.qr(np.column_stack([xr, np.eye(2 * m)]))[0][:, 1:]   # tangent basis
    ev = np.linalg.eigvalsh(Q.T @ (Hr - theta * np.eye(2 * m)) @ Q)
    assert ev[0] > -1e-7


def test_newton_model_is_second_order_taylor():
    # F is a quartic polynomial in (Re X, Im X); expanding |X+S|^4 by hand, its
    # Taylor remainder after the quadratic model f_W (delta = 0) is exactly
    # alpha sum (4 Re(conj(X) S) |S|^2 + |S|^4).  Independent of Lemma 3.1.
    rng = np.random.default_rng(4)
    p = W.Problem(dim=2, n=(16, 16), lo=(-4.0, -4.0), hi=(4.0, 4.0), beta=200.0, omega=0.7)
    up = UnifiedProblem(p)
    x = rng.standard_normal(p.shape) + 1j * rng.standard_normal(p.shape)
    x /= math.sqrt(re_dot(x, x))
    s = 0.05 * (rng.standard_normal(p.shape) + 1j * rng.standard_normal(p.shape))
    f0, g0 = up.f_and_grad(x)
    fw = re_dot(s, g0) + 0.5 * re_dot(s, up.hess(x, s))
    s2 = np.abs(s) ** 2
    rem = up.alpha * float(np.sum(4 * np.real(np.conj(x) * s) * s2 + s2 * s2))
    assert abs(up.F(x + s) - f0 - fw - rem) < 1e-11 * abs(fw)


def test_prolongation_interpolates():
    # Trigonometric interpolation keeps the coarse samples and reproduces a
    # band-limited (to roundoff) Gaussian on the fine grid.
    pc = W.Problem(dim=2, n=(64, 64), lo=(-10.0, -10.0), hi=(10.0, 10.0))
    pf = pc.with_n((128, 128))
    xc, yc = disc.grid_coords(pc)
    xf, yf = disc.grid_coords(pf)
    gc = np.exp(-(xc ** 2 + yc ** 2) / 3) * (1 + 0.3j * xc)
    gf = np.exp(-(xf ** 2 + yf ** 2) / 3) * (1 + 0.3j * xf)
    pr = prolong_fourier(gc)
    assert np.max(np.abs(pr - gf)) < 1e-12
    rng = np.random.default_rng(0)
    u = rng.standard_normal((16, 16)) + 1j * rng.standard_normal((16, 16))
    assert np.max(np.abs(prolong_fourier(u)[::2, ::2] - u)) < 1e-13
