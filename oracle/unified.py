"""The unified finite-dimensional problem (§3).

Test infrastructure (see the package docstring).

§3 writes every discretization as  min F(X) = 1/2 X^* A X + alpha sum |X_j|^4
over the unit sphere ||X||_2 = 1, "via a proper rescaling" it leaves
unstated.  The rescaling used here:  X = sqrt(h_vol) Phi,  A = 2 H_lin,
alpha = beta / (2 h_vol).  Then F(X) = E_h(Phi), ||X||_2 = ||Phi||_h, and

    grad F  = A X + 4 alpha |X|^2 X            = 2 sqrt(h_vol) H(phi) phi,
    theta   = Re(X^* G) = 2 mu,   mu = F + alpha sum |X|^4   (§1, mu = E + beta/2 int |phi|^4),
    r       = ||H(phi)phi - mu phi||_inf = ||G - theta X||_inf / (2 sqrt(h_vol)).

Lemma 3.1 (first and second directional derivatives) gives, with the real
inner product Re(D^* .):

    grad F [D]   = Re(D^* A X) + 4 alpha sum |X_j|^2 Re(conj(X_j) D_j),
    Hess F [D,D] = D^* A D + 4 alpha sum (|X_j|^2 |D_j|^2 + 2 Re(conj(X_j) D_j)^2),

so the Hessian-vector product is  H[D] = A D + 4 alpha (|X|^2 D + 2 Re(conj(X) D) X).
"""
from __future__ import annotations

import math

import numpy as np

from . import discretization as disc


def re_dot(u, v):
    """Real inner product Re(u^* v) (the R^{2M} inner product of §3)."""
    return float(np.vdot(u, v).real)


class UnifiedProblem:
    """F(X), its gradient and Hessian for one discretized problem."""

    def __init__(self, p):
        self.p = p
        self.hvol = disc.h_vol(p)
        self.alpha = p.beta / (2.0 * self.hvol)
        self.v = disc.potential(p)
        self.coords = disc.grid_coords(p)
        self.dtype = np.float64 if p.bc in ("sine", "fd") else np.complex128

    # -- the linear operator A = 2 H_lin ---------------------------------
    def A(self, x):
        return 2.0 * disc.h_lin(self.p, x, self.v)

    # -- F, grad F ----------------------------------------------------------
    def F(self, x):
        return 0.5 * re_dot(x, self.A(x)) + self.alpha * float(np.sum(np.abs(x) ** 4))

    def grad(self, x):
        return self.A(x) + 4.0 * self.alpha * np.abs(x) ** 2 * x

    def f_and_grad(self, x):
        ax = self.A(x)
        q = np.abs(x) ** 2
        f = 0.5 * re_dot(x, ax) + self.alpha * float(np.sum(q * q))
        return f, ax + 4.0 * self.alpha * q * x

    def hess(self, x, d):
        """H[D] = A D + 4 alpha (|X|^2 D + 2 Re(conj(X) D) X)  (Lemma 3.1)."""
        return self.A(d) + 4.0 * self.alpha * (np.abs(x) ** 2 * d
                                               + 2.0 * np.real(np.conj(x) * d) * x)

    # -- outputs --------------------------------------------------------------
    def theta(self, x, g):
        """Lagrange multiplier theta = X^* G / X^* X (first-order conditions, §3)."""
        return re_dot(x, g) / re_dot(x, x)

    def residual(self, x, g):
        """||H(phi)phi - mu phi||_inf in phi units."""
        th = self.theta(x, g)
        return float(np.max(np.abs(g - th * x))) / (2.0 * math.sqrt(self.hvol))

    def to_x(self, phi):
        return np.asarray(phi, dtype=self.dtype) * math.sqrt(self.hvol)

    def to_phi(self, x):
        return np.asarray(x) / math.sqrt(self.hvol)

    def outputs(self, x):
        """E, mu, residual, rms per axis, max|phi|^2, ||phi||_h^2 - 1 (§1, §4 eq. rms)."""
        f, g = self.f_and_grad(x)
        quart = float(np.sum(np.abs(x) ** 4))
        dens = np.abs(x) ** 2
        rms = [math.sqrt(float(np.sum(c * c * dens))) for c in self.coords]
        return {
            "energy": f,
            "mu": f + self.alpha * quart,
            "resid": self.residual(x, g),
            "rms": rms,
            "max_dens": float(np.max(dens)) / self.hvol,
            "norm_err": re_dot(x, x) - 1.0,
        }
