"""Feasible gradient method on the sphere (§3.1, Theorem 3.3, Algorithm 1).

Test infrastructure (see the package docstring).

Reading of the complex case (§3.1 leaves it implicit): the sphere is the
real sphere in R^{2M} and every inner product is Re(u^* v), as in Lemma 3.1.
Then the skew operator  A(X) = G X^* - X G^*  acts as
A(X) X = ||X||^2 G - Re(X^* G) X  (the projected gradient P), and the implicit
Cayley curve  Y(tau) = (I + tau A)^-1 (I - tau A) X  has Theorem 3.3's closed
form  Y = p X + q G  with a = Re(X^* G), n_x = ||X||^2, n_g = ||G||^2:

    p = ((1 + tau a)^2 - tau^2 n_x n_g) / den,  q = -2 tau n_x / den,
    den = 1 - tau^2 a^2 + tau^2 n_x n_g.

n_x is carried explicitly (never assumed 1); the iterate is renormalised
when | ||Y||^2 - 1 | exceeds 1e-14 (§4, the normalisation step).

Step size: Barzilai-Borwein (§3.1) with S = X_k - X_{k-1},
W = P_k - P_{k-1}; odd k uses  ||S||^2 / |Re(S^* W)|, even k uses
|Re(S^* W)| / ||W||^2 (the paper says "or"; alternating is this reading),
k = 0 uses tau_init; unbounded values are clamped to [1e-20, 1e20] and a
zero |Re(S^* W)| keeps the previous value.  The trial step is
tau = 1/2 tau_BB sigma^m with the smallest m >= 0 that satisfies the
nonmonotone (Zhang-Hager) condition
    f(Y(tau)) <= C_k - rho_1 tau ||P_k||^2,
C_0 = f(X_0), Q_0 = 1, Q_{k+1} = eta Q_k + 1,
C_{k+1} = (eta Q_k C_k + f(X_{k+1})) / Q_{k+1}.  If no m <= m_max passes,
the last trial is taken.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

from .unified import re_dot


def cayley_coefficients(tau, a, nx, ng):
    """Theorem 3.3 coefficients (p, q) of Y(tau) = p X + q G."""
    den = 1.0 - tau * tau * a * a + tau * tau * nx * ng
    p = ((1.0 + tau * a) ** 2 - tau * tau * nx * ng) / den
    q = -2.0 * tau * nx / den
    return p, q


def cayley_point(x, g, tau):
    """Y(tau) for the curve through X along G (no renormalisation)."""
    a, nx, ng = re_dot(x, g), re_dot(x, x), re_dot(g, g)
    p, q = cayley_coefficients(tau, a, nx, ng)
    return p * x + q * g


@dataclasses.dataclass
class FGStats:
    iters: int = 0
    nfe: int = 0
    backtracks: int = 0


@dataclasses.dataclass
class FGResult:
    x: np.ndarray
    f: float
    g: np.ndarray
    tau_bb: float
    stopped: bool      # True when the stop test held (not the iteration cap)
    iters: int


def feasible_gradient(fun, x, f, g, *, maxit, tau_init, stop, rho1=1e-4, eta=0.85,
                      sigma=0.5, m_max=20, renorm_tol=1e-14, stats=None, stop_step=None,
                      trace=None):
    """Algorithm 1 from the feasible point ``x`` with f(x), grad f(x) given.

    ``fun(Y) -> (f, G)``; ``stop(x, f, g, P) -> bool`` is tested on every
    iterate before a step is taken; ``stop_step(x_new, x_old, t) -> bool``
    (optional) right after each accepted step of length t (the paper's
    step-length rules).  eta = 0 makes the search monotone: C is then
    f(X_k) itself.  ``trace`` (optional, for tests): a list that receives one
    dict per accepted step with the iterate, its f, g and P, the BB step used,
    the accepted trial length t, the backtracks m and the reference value C
    and weight Q after the update.  Returns an ``FGResult``."""
    if stats is None:
        stats = FGStats()
    nx, a = re_dot(x, x), re_dot(x, g)
    P = nx * g - a * x
    C, Q = f, 1.0
    tau_bb = tau_init
    x_prev = P_prev = None
    k = 0
    while True:
        if stop(x, f, g, P):
            return FGResult(x, f, g, tau_bb, True, k)
        if k >= maxit:
            return FGResult(x, f, g, tau_bb, False, k)
        if k > 0:
            S = x - x_prev
            Wd = P - P_prev
            sw = abs(re_dot(S, Wd))
            if sw > 0.0:
                tau_bb = re_dot(S, S) / sw if k % 2 == 1 else sw / re_dot(Wd, Wd)
            tau_bb = min(max(tau_bb, 1e-20), 1e20)
        ng = re_dot(g, g)
        nP2 = re_dot(P, P)
        t = 0.5 * tau_bb
        for m in range(m_max + 1):
            p, q = cayley_coefficients(t, a, nx, ng)
            y = p * x + q * g
            ny = re_dot(y, y)
            if abs(ny - 1.0) > renorm_tol:
                y = y / math.sqrt(ny)
            fy, gy = fun(y)
            stats.nfe += 1
            if fy <= C - rho1 * t * nP2:
                break
            if m < m_max:
                stats.backtracks += 1
                t *= sigma
        x_prev, P_prev = x, P
        x, f, g = y, fy, gy
        nx, a = re_dot(x, x), re_dot(x, g)
        P = nx * g - a * x
        Qn = eta * Q + 1.0
        C = (eta * Q * C + f) / Qn
        Q = Qn
        k += 1
        stats.iters += 1
        if trace is not None:
            trace.append({"k": k, "x": x, "f": f, "g": g, "P": P, "tau_bb": tau_bb, "t": t,
                          "m": m, "C": C, "Q": Q})
        if stop_step is not None and stop_step(x, x_prev, t):
            return FGResult(x, f, g, tau_bb, True, k)
