"""Spatial discretization of the GP energy (§2): grid, trap, spectral operators.

Test infrastructure (see the package docstring).

Fourier pseudospectral (§2.3): per-axis DFT with wavenumbers
lambda_p = 2 pi p / (b - a), p = -N/2 .. N/2-1.  Turning the per-axis
Parseval form of the discrete energy into an operator gives

    H_lin phi = sum_axes F^-1[ m_axis * F phi ] + V phi,
    m_x(p; y) = lambda_p^2/2 + Omega*y*lambda_p,
    m_y(q; x) = eta_q^2/2   - Omega*x*eta_q,
    m_z(r)    = zeta_r^2/2,

i.e. -1/2 Laplacian + V - Omega L_z with L_z = -i(x d_y - y d_x) (§1).  The
Nyquist mode p = -N/2 is kept with its printed wavenumber.

Sine pseudospectral (§2.2, homogeneous Dirichlet, Omega = 0): per axis the
kinetic part is (1/N) C Lambda C with c_jl = sin(j l pi / N) and
Lambda = diag(lambda_l^2), lambda_l = pi l / (b - a), on interior points.
scipy's DST-I computes 2 C x, hence (1/N) C Lambda C x = dst1(Lambda dst1(x))/(4N).

Finite differences (§2.1, homogeneous Dirichlet, Omega = 0): on the interior
points the kinetic part is the symmetric tridiagonal matrix with 1/h^2 on the
diagonal and -1/(2 h^2) beside it, i.e. -1/2 (phi_{j+1} - 2 phi_j + phi_{j-1})/h^2
with phi_0 = phi_N = 0, applied along every axis (the paper's A minus V).
"""
from __future__ import annotations

import numpy as np
import scipy.fft as sfft

from workloads import FOURIER, SINE, FD, DIRICHLET


def axis_points(p, ax):
    """Grid points on axis ``ax``: x_j = a + j h, h = (b-a)/N.

    Fourier:  j = 0..N-1 (unique periodic points, §2.3).
    Sine, FD: j = 1..N-1 (interior points, §2.2, §2.1)."""
    h = (p.hi[ax] - p.lo[ax]) / p.n[ax]
    j = np.arange(1, p.n[ax]) if p.bc in DIRICHLET else np.arange(p.n[ax])
    return p.lo[ax] + j * h


def grid_coords(p):
    """[x, y, z] broadcastable to the (z, y, x) array shape."""
    out = []
    for ax in range(p.dim):
        c = axis_points(p, ax)
        shp = [1] * p.dim
        shp[p.dim - 1 - ax] = c.size
        out.append(c.reshape(shp))
    return out


def h_vol(p):
    """Quadrature weight prod h_i (trapezoid rule on unique points, §2)."""
    return float(np.prod([(p.hi[a] - p.lo[a]) / p.n[a] for a in range(p.dim)]))


def potential(p):
    """V on the grid: harmonic trap (§1) plus optical lattice (§4.2/§4.4),
    V = 1/2 sum gamma_i^2 x_i^2 + A sum sin^2(k x_i); or the explicit array."""
    if p.v is not None:
        return np.asarray(p.v, dtype=np.float64).reshape(p.shape)
    v = np.zeros(p.shape)
    for ax, c in enumerate(grid_coords(p)):
        v = v + 0.5 * (p.gamma[ax] * c) ** 2
        if p.lattice_amp != 0.0:
            v = v + p.lattice_amp * np.sin(p.lattice_k * c) ** 2
    return v


def _fourier_wavenumbers(n, length):
    # fftfreq(n, 1/n) gives p = 0..n/2-1, -n/2..-1 in FFT bin order.
    return 2.0 * np.pi * np.fft.fftfreq(n, d=1.0 / n) / length


def _kinetic_fourier(p, phi):
    d = p.dim
    coords = grid_coords(p)
    out = np.zeros(phi.shape, dtype=np.complex128)
    for ax in range(d):
        npax = d - 1 - ax
        length = p.hi[ax] - p.lo[ax]
        lam = _fourier_wavenumbers(p.n[ax], length)
        shp = [1] * d
        shp[npax] = lam.size
        lam = lam.reshape(shp)
        m = 0.5 * lam * lam
        if p.omega != 0.0 and d >= 2:
            if ax == 0:          # x-lines: + Omega * y * lambda
                m = m + p.omega * coords[1] * lam
            elif ax == 1:        # y-lines: - Omega * x * eta
                m = m - p.omega * coords[0] * lam
        out += np.fft.ifft(m * np.fft.fft(phi, axis=npax), axis=npax)
    return out


def _kinetic_sine(p, phi):
    d = p.dim
    out = np.zeros(phi.shape, dtype=np.float64)
    for ax in range(d):
        npax = d - 1 - ax
        n = p.n[ax]
        lam = np.pi * np.arange(1, n) / (p.hi[ax] - p.lo[ax])
        shp = [1] * d
        shp[npax] = lam.size
        lam2 = (lam * lam).reshape(shp)
        out += sfft.dst(lam2 * sfft.dst(phi, type=1, axis=npax), type=1, axis=npax) / (4.0 * n)
    return out


def _kinetic_fd(p, phi):
    d = p.dim
    out = np.zeros(phi.shape, dtype=phi.dtype)
    for ax in range(d):
        npax = d - 1 - ax
        h = (p.hi[ax] - p.lo[ax]) / p.n[ax]
        # the boundary values phi_0 = phi_N = 0 as explicit zeros
        pad = [(0, 0)] * d
        pad[npax] = (1, 1)
        q = np.pad(phi, pad)
        sl = lambda a, b: tuple(slice(a, b) if k == npax else slice(None) for k in range(d))
        m = phi.shape[npax]
        lap = (q[sl(2, m + 2)] - 2.0 * q[sl(1, m + 1)] + q[sl(0, m)]) / (h * h)
        out = out - 0.5 * lap
    return out


def kinetic(p, phi):
    """Kinetic (+ rotation) part of H_lin: everything but V."""
    if p.bc == FD:
        if p.omega != 0.0:
            raise ValueError("the finite-difference discretization here needs Omega = 0")
        phi = np.asarray(phi)
        return _kinetic_fd(p, phi.astype(np.complex128 if np.iscomplexobj(phi) else np.float64))
    if p.bc == SINE:
        if p.omega != 0.0:
            raise ValueError("sine pseudospectral discretization needs Omega = 0")
        return _kinetic_sine(p, np.asarray(phi, dtype=np.float64))
    return _kinetic_fourier(p, np.asarray(phi, dtype=np.complex128))


def h_lin(p, phi, v=None):
    """H_lin phi = (-1/2 Laplacian + V - Omega L_z) phi on the grid."""
    if v is None:
        v = potential(p)
    return kinetic(p, phi) + v * phi


def h_full(p, phi, v=None):
    """H(phi) phi = H_lin phi + beta |phi|^2 phi (the Euler-Lagrange operator, §1)."""
    return h_lin(p, phi, v) + p.beta * np.abs(phi) ** 2 * phi
