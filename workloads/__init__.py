"""Seeded synthetic workloads: problem parameters and initial data.

This module is shared by the CPU oracle, the GPU binding's tests and the
benchmark.  It holds *no* arithmetic of the method itself: only problem
parameters (grid, domain, trap, beta, Omega) and the initial functions the
paper lists for its experiments, sampled on the grid with seeded noise.

Grid convention (Fourier pseudospectral, §2.3): ``n`` unique periodic points
per axis, ``x_j = lo + j*h``, ``h = (hi-lo)/n``, ``j = 0..n-1`` (the paper's
"2^k+1 nodes" with the periodic copy dropped).  Sine pseudospectral (§2.2)
and finite differences (§2.1), both homogeneous Dirichlet: ``n`` intervals,
interior points ``j = 1..n-1``.  Arrays are numpy arrays in
C order with x fastest: shape ``(nx,)``, ``(ny, nx)`` or ``(nz, ny, nx)``.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional, Sequence

import numpy as np

FOURIER = "fourier"
SINE = "sine"
FD = "fd"
DIRICHLET = (SINE, FD)      # grids of interior points


@dataclasses.dataclass
class Problem:
    """The paper's statement of a ground-state problem (§1, §2, §4).

    dim          spatial dimension d (1, 2, 3)
    n            points per axis (x, y, z order); see the module docstring
    lo, hi       computational box U = prod (lo_i, hi_i)
    bc           FOURIER (periodic), SINE or FD (homogeneous Dirichlet)
    beta         interaction constant
    omega        rotation speed (0 unless FOURIER and dim >= 2)
    gamma        harmonic trap frequencies, V = 1/2 sum gamma_i^2 x_i^2
    lattice_amp  optical-lattice amplitude A in A * sum sin^2(k x_i)
    lattice_k    optical-lattice wavenumber k (pi/4 in the paper)
    v            optional explicit potential array (overrides the analytic V)
    """

    dim: int
    n: Sequence[int]
    lo: Sequence[float]
    hi: Sequence[float]
    bc: str = FOURIER
    beta: float = 0.0
    omega: float = 0.0
    gamma: Sequence[float] = (1.0, 1.0, 1.0)
    lattice_amp: float = 0.0
    lattice_k: float = math.pi / 4
    v: Optional[np.ndarray] = None

    def __post_init__(self):
        self.n = tuple(int(v) for v in self.n)[: self.dim]
        self.lo = tuple(float(v) for v in self.lo)[: self.dim]
        self.hi = tuple(float(v) for v in self.hi)[: self.dim]
        g = tuple(float(v) for v in self.gamma) + (1.0,) * 3
        self.gamma = g[:3]

    @property
    def shape(self):
        """numpy shape, x fastest."""
        if self.bc in DIRICHLET:
            return tuple(n - 1 for n in reversed(self.n))
        return tuple(reversed(self.n))

    @property
    def size(self):
        return int(np.prod(self.shape))

    def with_n(self, n):
        return dataclasses.replace(self, n=tuple(n), v=None)


def _axis_points(p: Problem, axis: int) -> np.ndarray:
    h = (p.hi[axis] - p.lo[axis]) / p.n[axis]
    if p.bc in DIRICHLET:
        j = np.arange(1, p.n[axis])
    else:
        j = np.arange(p.n[axis])
    return p.lo[axis] + j * h


def coords(p: Problem):
    """Coordinate arrays broadcastable to ``p.shape`` (x, y, z order)."""
    out = []
    for ax in range(p.dim):
        c = _axis_points(p, ax)
        shp = [1] * p.dim
        shp[p.dim - 1 - ax] = c.size
        out.append(c.reshape(shp))
    return out


# ---------------------------------------------------------------------------
# Initial data of §4.3: (a) Gaussian, (b) vortex, (d) their Omega-weighted mix.
# phi_a and phi_b are unit-normalised in L2(R^2) and orthogonal, so the L2
# norm of (1-W) phi_a + W phi_b is sqrt((1-W)^2 + W^2).
# ---------------------------------------------------------------------------

def phi_a(p: Problem):
    x, y = coords(p)[:2]
    return np.exp(-(x * x + y * y) / 2) / math.sqrt(math.pi) + 0j


def phi_b(p: Problem):
    x, y = coords(p)[:2]
    return (x + 1j * y) * np.exp(-(x * x + y * y) / 2) / math.sqrt(math.pi)


def phi_d(p: Problem, omega: float):
    w = float(omega)
    return ((1 - w) * phi_a(p) + w * phi_b(p)) / math.sqrt((1 - w) ** 2 + w ** 2)


def gaussian_times_noise(p: Problem, amp: float, seed: int):
    """exp(-|x|^2/2) * (1 + amp * xi), xi ~ N(0,1) iid (real)."""
    r2 = sum(c * c for c in coords(p))
    rng = np.random.default_rng(seed)
    xi = rng.standard_normal(p.shape)
    return np.exp(-r2 / 2) * (1.0 + amp * xi)


def rotating_initial(p: Problem, omega: float, seed: int, amp: float = 1e-3):
    """phi_d plus amp*(xi + i*zeta), xi, zeta ~ N(0,1) iid, drawn in that order."""
    rng = np.random.default_rng(seed)
    xi = rng.standard_normal(p.shape)
    zeta = rng.standard_normal(p.shape)
    return phi_d(p, omega) + amp * (xi + 1j * zeta)


# ---------------------------------------------------------------------------
# Workloads: 1D harmonic trap; 2D rotating condensate; 3D optical lattice;
# a batched sweep of rotating problems; a cascadic batch.
# ---------------------------------------------------------------------------

def harmonic_1d(beta: float = 400.0, n: int = 512):
    p = Problem(dim=1, n=(n,), lo=(-16.0,), hi=(16.0,), beta=beta)
    return p, gaussian_times_noise(p, 0.05, seed=1)


def rotating_2d(n: int = 256, beta: float = 1000.0, omega: float = 0.9, seed: int = 2):
    p = Problem(dim=2, n=(n, n), lo=(-12.0, -12.0), hi=(12.0, 12.0),
                beta=beta, omega=omega)
    return p, rotating_initial(p, omega, seed)


def lattice_3d(n: int = 128, beta: float = 1600.0, amp: float = 100.0, box: float = 16.0):
    p = Problem(dim=3, n=(n, n, n), lo=(-box,) * 3, hi=(box,) * 3, beta=beta,
                lattice_amp=amp)
    return p, gaussian_times_noise(p, 0.01, seed=3)


def rotating_sweep_params(count: int = 64):
    """(beta_i, omega_i, n_i) for the batched sweep, seed 4."""
    rng = np.random.default_rng(4)
    betas = rng.uniform(100.0, 2000.0, size=count)
    omegas = rng.uniform(0.0, 0.95, size=count)
    grids = [(64, 128, 256)[i % 3] for i in range(count)]
    return betas, omegas, grids


def rotating_sweep_2d(count: int = 64, grid_override=None):
    betas, omegas, grids = rotating_sweep_params(count)
    probs, phis = [], []
    for i in range(count):
        n = grids[i] if grid_override is None else grid_override
        p = Problem(dim=2, n=(n, n), lo=(-12.0, -12.0), hi=(12.0, 12.0),
                    beta=float(betas[i]), omega=float(omegas[i]))
        probs.append(p)
        phis.append(rotating_initial(p, p.omega, 1000 + i))
    return probs, phis


def cascade_2d(levels=(64, 128, 256, 512), count: int = 16, beta: float = 5000.0):
    omegas = [0.80 + 0.01 * i for i in range(count)]
    probs, phis = [], []
    for i, w in enumerate(omegas):
        p = Problem(dim=2, n=(levels[0],) * 2, lo=(-20.0, -20.0), hi=(20.0, 20.0),
                    beta=beta, omega=w)
        probs.append(p)
        phis.append(rotating_initial(p, w, 5000 + i))
    return probs, phis, tuple(levels)
