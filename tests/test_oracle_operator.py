"""Pins of the oracle's discretization (§2.2, §2.3) and unified problem (§3).

Each check compares against mathematics the oracle does not itself encode:
closed-form eigenfunctions, Hermiticity, Taylor expansions, brute force.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import discretization as disc
from oracle.unified import UnifiedProblem, re_dot


def _gauss(p):
    r2 = sum(c * c for c in disc.grid_coords(p))
    return np.exp(-r2 / 2)


@pytest.mark.parametrize("dim,n,box", [(1, 512, 16.0), (2, 64, 12.0), (3, 64, 10.0)])
def test_harmonic_gaussian_is_exact_eigenfunction(dim, n, box):
    # beta = 0, Omega = 0: exp(-|x|^2/2) is the harmonic ground state with
    # H_lin phi = (d/2) phi; the spectral operator reproduces it to roundoff.
    p = W.Problem(dim=dim, n=(n,) * dim, lo=(-box,) * dim, hi=(box,) * dim)
    g = _gauss(p)
    hg = disc.h_lin(p, g)
    assert np.max(np.abs(hg - 0.5 * dim * g)) < 1e-11
    up = UnifiedProblem(p)
    x = up.to_x(g)
    x /= math.sqrt(re_dot(x, x))
    out = up.outputs(x)
    assert abs(out["energy"] - 0.5 * dim) < 1e-12
    assert abs(out["mu"] - 0.5 * dim) < 1e-12
    assert out["resid"] < 1e-10


@pytest.mark.parametrize("omega", [0.3, 0.9])
def test_landau_levels_fix_rotation_sign(omega):
    # -1/2 Lap + r^2/2 - Omega L_z with L_z = -i(x d_y - y d_x):
    # (x + iy) e^{-r^2/2} has L_z = +1 -> eigenvalue 2 - Omega,
    # (x - iy) e^{-r^2/2} has L_z = -1 -> eigenvalue 2 + Omega.
    p = W.Problem(dim=2, n=(128, 128), lo=(-12.0, -12.0), hi=(12.0, 12.0), omega=omega)
    x, y = disc.grid_coords(p)
    e = np.exp(-(x * x + y * y) / 2)
    for sgn, lam in ((1.0, 2.0 - omega), (-1.0, 2.0 + omega)):
        f = (x + sgn * 1j * y) * e
        assert np.max(np.abs(disc.h_lin(p, f) - lam * f)) < 1e-11


@pytest.mark.parametrize("omega", [0.4, -0.7])
def test_rotation_in_3d(omega):
    # 3D: the rotation acts in the x-y plane only.  With V = (x^2 + y^2 +
    # gz^2 z^2)/2, (x + iy) e^{-(x^2+y^2)/2} h_k(z) has eigenvalue
    # 2 - Omega + (k + 1/2) gz for the trap levels h_0 = e^{-gz z^2/2},
    # h_1 = z e^{-gz z^2/2}
    gz = 2.0
    p = W.Problem(dim=3, n=(64, 64, 64), lo=(-10.0,) * 3, hi=(10.0,) * 3, omega=omega,
                  gamma=(1.0, 1.0, gz))
    x, y, z = disc.grid_coords(p)
    e = (x + 1j * y) * np.exp(-(x * x + y * y) / 2) * np.exp(-gz * z * z / 2)
    for k, f in ((0, e), (1, z * e)):
        lam = 2.0 - omega + (k + 0.5) * gz
        assert np.max(np.abs(disc.h_lin(p, f) - lam * f)) < 1e-10


def test_fourier_plane_waves_and_nyquist():
    # sin(2 pi k (x-a)/L) has -1/2 d_xx eigenvalue (2 pi k / L)^2 / 2 for
    # |k| < N/2; the Nyquist grid function (-1)^j gets (pi N / L)^2 / 2.
    n, a, b = 32, -3.0, 5.0
    p = W.Problem(dim=1, n=(n,), lo=(a,), hi=(b,), gamma=(0.0,))
    xs = disc.axis_points(p, 0)
    L = b - a
    for k in (1, 5, n // 2 - 1):
        f = np.sin(2 * np.pi * k * (xs - a) / L)
        assert np.max(np.abs(disc.h_lin(p, f) - 0.5 * (2 * np.pi * k / L) ** 2 * f)) < 1e-10
    f = (-1.0) ** np.arange(n)
    assert np.max(np.abs(disc.h_lin(p, f) - 0.5 * (np.pi * n / L) ** 2 * f)) < 1e-9


def test_nyquist_rotation_term_kept_as_printed():
    # Reading: the first-derivative multiplier keeps lambda_{-N/2} = -pi N / L.
    # On f = (-1)^j along x (constant in y) the x-line multiplier gives
    # (lambda^2/2 + Omega*y*lambda) f with lambda = -pi N / L.
    n, L, om = 16, 8.0, 0.7
    p = W.Problem(dim=2, n=(n, n), lo=(-4.0, -4.0), hi=(4.0, 4.0), omega=om, gamma=(0.0, 0.0))
    x, y = disc.grid_coords(p)
    f = np.broadcast_to((-1.0) ** np.arange(n), (n, n)).astype(complex)
    lam = -np.pi * n / L
    expect = (0.5 * lam * lam + om * y * lam) * f
    # the y-lines see a constant function: zero contribution
    assert np.max(np.abs(disc.kinetic(p, f) - expect)) < 1e-10


@pytest.mark.parametrize("bc,omega", [("fourier", 0.0), ("fourier", 0.85), ("sine", 0.0)])
def test_h_lin_is_hermitian(bc, omega):
    rng = np.random.default_rng(7)
    p = W.Problem(dim=2, n=(32, 16), lo=(-5.0, -4.0), hi=(6.0, 4.0), bc=bc, omega=omega,
                  lattice_amp=3.0)
    if bc == "sine":
        u, v = rng.standard_normal(p.shape), rng.standard_normal(p.shape)
    else:
        u = rng.standard_normal(p.shape) + 1j * rng.standard_normal(p.shape)
        v = rng.standard_normal(p.shape) + 1j * rng.standard_normal(p.shape)
    lhs = np.vdot(u, disc.h_lin(p, v))
    rhs = np.vdot(disc.h_lin(p, u), v)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_sine_eigenvectors():
    # sin(l pi (x-a)/L) on the interior points is an eigenvector of the sine
    # pseudospectral -1/2 d_xx with eigenvalue (pi l / L)^2 / 2 (§2.2).
    n, a, b = 64, -16.0, 16.0
    p = W.Problem(dim=1, n=(n,), lo=(a,), hi=(b,), bc="sine", gamma=(0.0,))
    xs = disc.axis_points(p, 0)
    for l in (1, 7, n - 1):
        f = np.sin(l * np.pi * (xs - a) / (b - a))
        lam = np.pi * l / (b - a)
        assert np.max(np.abs(disc.kinetic(p, f) - 0.5 * lam * lam * f)) < 1e-9 * max(1, lam * lam)


def test_sine_operator_matches_dense_sum():
    # Brute force: B - V = (1/N) C Lambda C with c_jk = sin(jk pi/N) summed by hand.
    n, a, b = 8, 0.0, 3.0
    p = W.Problem(dim=1, n=(n,), lo=(a,), hi=(b,), bc="sine", gamma=(0.0,))
    rng = np.random.default_rng(3)
    f = rng.standard_normal(n - 1)
    lam2 = [(math.pi * l / (b - a)) ** 2 for l in range(1, n)]
    out = []
    for j in range(1, n):
        s = 0.0
        for l in range(1, n):
            cl = sum(math.sin(k * l * math.pi / n) * f[k - 1] for k in range(1, n))
            s += math.sin(j * l * math.pi / n) * lam2[l - 1] * cl
        out.append(s / n)
    assert np.max(np.abs(disc.kinetic(p, f) - np.array(out))) < 1e-12


def test_potential_closed_form():
    p = W.Problem(dim=3, n=(8, 8, 8), lo=(-4.0,) * 3, hi=(4.0,) * 3, gamma=(1.0, 2.0, 4.0),
                  lattice_amp=50.0)
    v = disc.potential(p)
    # point (j=1, k=2, l=3): x = -3, y = -2, z = -1
    x, y, z = -3.0, -2.0, -1.0
    expect = 0.5 * (x * x + 4 * y * y + 16 * z * z) + 50 * (
        math.sin(math.pi * x / 4) ** 2 + math.sin(math.pi * y / 4) ** 2 + math.sin(math.pi * z / 4) ** 2)
    assert abs(v[3, 2, 1] - expect) < 1e-12


def _rand_state(p, rng):
    x = rng.standard_normal(p.shape) + 1j * rng.standard_normal(p.shape)
    return x / math.sqrt(re_dot(x, x))


def test_lemma_gradient_and_hessian_taylor():
    # Lemma 3.1 checked by Taylor remainders of F itself:
    # F(X+tD)-F(X)-t gradF[D] = O(t^2);  ... - t^2/2 HessF[D,D] = O(t^3).
    rng = np.random.default_rng(11)
    p = W.Problem(dim=2, n=(16, 16), lo=(-4.0, -4.0), hi=(4.0, 4.0), beta=300.0, omega=0.6)
    up = UnifiedProblem(p)
    x, d = _rand_state(p, rng), _rand_state(p, rng)
    f0, g0 = up.f_and_grad(x)
    g1 = re_dot(d, g0)
    h2 = re_dot(d, up.hess(x, d))
    e1, e2 = [], []
    for t in (1e-2, 5e-3, 2.5e-3):
        ft = up.F(x + t * d)
        e1.append(abs(ft - f0 - t * g1))
        e2.append(abs(ft - f0 - t * g1 - 0.5 * t * t * h2))
    for a_, b_ in zip(e1, e1[1:]):
        assert 3.5 < a_ / b_ < 4.5
    for a_, b_ in zip(e2, e2[1:]):
        assert 7.0 < a_ / b_ < 9.0


def test_mu_theta_residual_relations():
    # theta = Re(X^*G) = 2 mu with mu = E + beta/2 int |phi|^4 (§1, §3), and
    # the residual in phi units equals ||H(phi)phi - mu phi||_inf.
    rng = np.random.default_rng(5)
    p = W.Problem(dim=2, n=(16, 32), lo=(-4.0, -5.0), hi=(4.0, 5.0), beta=100.0, omega=0.4)
    up = UnifiedProblem(p)
    x = _rand_state(p, rng)
    out = up.outputs(x)
    f, g = up.f_and_grad(x)
    assert abs(re_dot(x, g) - 2 * out["mu"]) < 1e-10 * abs(out["mu"])
    phi = up.to_phi(x)
    hphi = disc.h_full(p, phi)
    mu_int = out["energy"] + 0.5 * p.beta * up.hvol * float(np.sum(np.abs(phi) ** 4))
    assert abs(mu_int - out["mu"]) < 1e-10 * abs(mu_int)
    assert abs(np.max(np.abs(hphi - mu_int * phi)) - out["resid"]) < 1e-9 * out["resid"]
