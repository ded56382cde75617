"""Regularized Newton method (§3.2, Algorithm 2).

Test infrastructure (see the package docstring).

At the outer iterate X_k (||X_k|| = 1), with G_k = grad F(X_k), q_k = |X_k|^2,
the model of §3.2 is the second-order Taylor expansion of F plus the proximal
term (delta/2)||X - X_k||^2.  Written in S = X - X_k (the reading of the
garbled printed W: delta belongs to the proximal term, not inside 2 alpha):

    f_W(X)  = Re(S^* G_k) + 1/2 Re(S^* H_k[S]) + (delta/2) ||S||^2,
    grad_W  = G_k + H_k[S] + delta S,
    H_k[S]  = A S + 4 alpha (q_k S + 2 Re(conj(X_k) S) X_k)       (Lemma 3.1).

The trust-region subproblem  min f_W on the sphere  is solved inexactly by
Algorithm 1 from X_k, for at most K_sub iterations or until
||P_W|| <= min(0.1, ||P_k||) ||P_k||, with the last BB step carried over.
For the trial Z = X_k + S the ratio rho = (F(Z) - F(X_k)) / (W(Z) - W(X_k))
uses the predicted reduction W(Z) - W(X_k) = f_W(Z) and the actual reduction
in difference form

    F(Z) - F(X_k) = Re(S^* A X_k) + 1/2 Re(S^* A S)
                    + alpha sum (2 Re(conj(X_k) S) + |S|^2)(|Z|^2 + q_k).

X_{k+1} = Z / ||Z|| if rho >= eta_1, else X_k; the regularization moves as
delta *= gamma_shrink (rho > eta_2), unchanged (eta_1 <= rho <= eta_2),
delta *= gamma_grow (rho < eta_1, including a non-negative predicted
reduction), clamped to [delta_min, delta_max].  The constants are not given
in the paper ("not very sensitive"); the defaults below are this reading.

Algorithm 2 starts with K_init iterations of Algorithm 1 on F itself.  The
stop test is the residual r < tol at an outer iterate, evaluated at every
outer step from a fresh evaluation of F at X_k.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

from .feasible import FGStats, feasible_gradient
from .unified import re_dot


@dataclasses.dataclass
class Options:
    tol: float = 1e-6
    k_init: int = 100
    k_sub: int = 200
    max_outer: int = 2000
    max_iter_alg1: int = 20000     # Algorithm 1 run on its own
    tau0: float = 1e-3
    rho1: float = 1e-4
    eta: float = 0.85
    sigma: float = 0.5
    m_max: int = 20
    renorm_tol: float = 1e-14
    eta1: float = 0.01
    eta2: float = 0.9
    gamma_shrink: float = 0.5
    gamma_grow: float = 4.0
    delta0: float = 1.0
    delta_min: float = 1e-12
    delta_max: float = 1e12
    # stop rule: "resid" (r < tol), or the paper's step-length rules (§4):
    # "crit1" ||X^{k+1} - X^k||_inf / tau_k <= eps0 on the steps of
    # Algorithm 1 (alone, and in the first K_init steps of Algorithm 2);
    # "crit2" ||X^{k+1} - X^k||_inf <= crit2_tol on accepted Newton steps of
    # Algorithm 2 (and on the steps of Algorithm 1 run alone).  Norms in X units.
    stop_rule: str = "resid"
    eps0: float = 1e-6
    crit2_tol: float = 1e-8
    monotone: bool = False      # monotone Armijo (C = F(X_k)) instead of Zhang-Hager


@dataclasses.dataclass
class SolveResult:
    x: np.ndarray
    converged: bool
    outer: int = 0
    inner: int = 0
    nfe: int = 0
    backtracks: int = 0
    rejections: int = 0
    log: list = dataclasses.field(default_factory=list)


def _fg_kwargs(o):
    return dict(rho1=o.rho1, eta=0.0 if o.monotone else o.eta, sigma=o.sigma, m_max=o.m_max,
                renorm_tol=o.renorm_tol)


def _inf_norm(d):
    return float(np.max(np.abs(d)))


def _alg1_stops(up, o):
    """(stop, stop_step) of Algorithm 1 on F under the configured rule."""
    never = lambda *a: False
    if o.stop_rule == "resid":
        return (lambda x_, f_, g_, P_: up.residual(x_, g_) < o.tol), None
    if o.stop_rule == "crit1":
        return never, (lambda xn, xo, t: _inf_norm(xn - xo) / t <= o.eps0)
    if o.stop_rule == "crit2":
        return never, (lambda xn, xo, t: _inf_norm(xn - xo) <= o.crit2_tol)
    raise ValueError(f"unknown stop rule {o.stop_rule}")


def feasible_only(up, x0, opts: Options):
    """Algorithm 1 on F alone (the paper's choice for Omega = 0), stop r < tol."""
    x = x0 / math.sqrt(re_dot(x0, x0))
    st = FGStats()
    f, g = up.f_and_grad(x)
    st.nfe += 1
    stop, stop_step = _alg1_stops(up, opts)
    res = feasible_gradient(up.f_and_grad, x, f, g, maxit=opts.max_iter_alg1,
                            tau_init=opts.tau0, stop=stop, stop_step=stop_step,
                            stats=st, **_fg_kwargs(opts))
    return SolveResult(res.x, res.stopped, 0, st.iters, st.nfe, st.backtracks)


def actual_reduction(up, xk, gk, z):
    """F(Z) - F(X_k) in difference form (the numerator of the ratio rho, §3.2).

    With S = Z - X_k, A X_k = G_k - 4 alpha |X_k|^2 X_k and
    |Z|^4 - |X_k|^4 = (|Z|^2 - |X_k|^2)(|Z|^2 + |X_k|^2),
    |Z|^2 - |X_k|^2 = 2 Re(conj(X_k) S) + |S|^2, the difference of the two
    energies is a sum of terms that vanish with S, so it keeps its relative
    accuracy when F(Z) and F(X_k) agree to many digits."""
    alpha = up.alpha
    s = z - xk
    qk = np.abs(xk) ** 2
    axk = gk - 4.0 * alpha * qk * xk
    return (re_dot(s, axk) + 0.5 * re_dot(s, up.A(s))
            + alpha * float(np.sum((2.0 * np.real(np.conj(xk) * s) + np.abs(s) ** 2)
                                   * (np.abs(z) ** 2 + qk))))


def regularized_newton(up, x0, opts: Options, log=False):
    """Algorithm 2 from x0 (need not be normalised)."""
    o = opts
    x = x0 / math.sqrt(re_dot(x0, x0))
    st = FGStats()
    f, g = up.f_and_grad(x)
    st.nfe += 1
    # the K_init steps of Algorithm 1: residual rule, or crit1 (crit2 is a
    # rule of the outer loop)
    if o.stop_rule == "crit1":
        stop, stop_step = _alg1_stops(up, o)
    else:
        stop, stop_step = (lambda x_, f_, g_, P_: up.residual(x_, g_) < o.tol), None
    res = feasible_gradient(up.f_and_grad, x, f, g, maxit=o.k_init, tau_init=o.tau0,
                            stop=stop, stop_step=stop_step, stats=st, **_fg_kwargs(o))
    x, tau = res.x, res.tau_bb
    delta = o.delta0
    out = SolveResult(x, False)
    alpha = up.alpha
    x_prev = None                # previous outer iterate when the last step was accepted
    for outer in range(o.max_outer + 1):
        f, g = up.f_and_grad(x)                  # outer evaluation at X_k
        st.nfe += 1
        r = up.residual(x, g)
        if log:
            out.log.append((outer, f, r, delta))
        if o.stop_rule == "crit2":
            # a rejected step leaves X unchanged and is not a step (reading)
            if x_prev is not None and _inf_norm(x - x_prev) <= o.crit2_tol:
                out.converged = True
                break
        elif r < o.tol:
            out.converged = True
            break
        if outer == o.max_outer:
            break
        nx, a = re_dot(x, x), re_dot(x, g)
        Pk = nx * g - a * x
        nPk = math.sqrt(re_dot(Pk, Pk))
        forcing = min(0.1, nPk) * nPk
        qk = np.abs(x) ** 2
        xk, gk, dk = x, g, delta

        def fun_w(y, xk=xk, gk=gk, qk=qk, dk=dk):
            s = y - xk
            hs = up.A(s) + 4.0 * alpha * (qk * s + 2.0 * np.real(np.conj(xk) * s) * xk)
            fw = re_dot(s, gk) + 0.5 * re_dot(s, hs) + 0.5 * dk * re_dot(s, s)
            return fw, gk + hs + dk * s

        inner = feasible_gradient(
            fun_w, xk, 0.0, gk, maxit=o.k_sub, tau_init=tau,
            stop=lambda x_, f_, g_, P_: math.sqrt(re_dot(P_, P_)) <= forcing,
            stats=st, **_fg_kwargs(o))
        tau = inner.tau_bb
        z = inner.x
        pred = inner.f
        ared = actual_reduction(up, xk, gk, z)
        rho = ared / pred if pred < 0.0 else -math.inf
        if rho >= o.eta1:
            x_prev = x
            x = z / math.sqrt(re_dot(z, z))
        else:
            x_prev = None
            out.rejections += 1
        if rho > o.eta2:
            delta *= o.gamma_shrink
        elif rho < o.eta1:
            delta *= o.gamma_grow
        delta = min(max(delta, o.delta_min), o.delta_max)
        out.outer += 1
    out.x = x
    out.inner = st.iters
    out.nfe = st.nfe
    out.backtracks = st.backtracks
    return out
