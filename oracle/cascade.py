"""Cascadic multigrid (Algorithm 3) with Fourier prolongation.

Test infrastructure (see the package docstring).

Algorithm 3 solves on the coarsest mesh, "refines the mesh uniformly" and
uses the coarse solution as the fine initial guess; the transfer operator is
not specified.  Reading used here: on periodic grids that share the origin
x = a (coarse points are every other fine point), the coarse grid function
is interpolated by its trigonometric interpolant -- per axis a DFT, the
spectrum zero-padded to 2N with the coarse Nyquist coefficient split half
and half between +N/2 and -N/2, and an inverse DFT -- then X is renormalised.
"""
from __future__ import annotations

import math

import numpy as np

from .newton import Options, regularized_newton
from .unified import UnifiedProblem, re_dot


def _pad_axis(c, npax):
    n = c.shape[npax]
    shp = list(c.shape)
    shp[npax] = 2 * n
    out = np.zeros(shp, dtype=np.complex128)

    def sl(a, b):
        idx = [slice(None)] * c.ndim
        idx[npax] = slice(a, b)
        return tuple(idx)

    half = n // 2
    out[sl(0, half)] = c[sl(0, half)]                  # p = 0 .. n/2-1
    out[sl(2 * n - half + 1, 2 * n)] = c[sl(half + 1, n)]  # p = -n/2+1 .. -1
    nyq = c[sl(half, half + 1)]                         # p = -n/2
    out[sl(half, half + 1)] = 0.5 * nyq
    out[sl(2 * n - half, 2 * n - half + 1)] = 0.5 * nyq
    return out


def prolong_fourier(phi_c):
    """Trigonometric interpolation of a periodic grid function to twice the
    points per axis (function values in, function values out)."""
    u = np.asarray(phi_c, dtype=np.complex128)
    for npax in range(u.ndim):
        n = u.shape[npax]
        c = np.fft.fft(u, axis=npax)
        u = np.fft.ifft(_pad_axis(c, npax), axis=npax) * (2 * n / n)
    return u


def cascadic(p_coarse, phi0, levels, opts: Options, level_tol=1e-4):
    """Algorithm 3 over grids ``levels`` (points per axis), coarse to fine.

    Returns (x_fine, fine_problem, per-level SolveResult list)."""
    results = []
    phi = np.asarray(phi0, dtype=np.complex128)
    prob = p_coarse.with_n((levels[0],) * p_coarse.dim)
    for li, n in enumerate(levels):
        prob = p_coarse.with_n((n,) * p_coarse.dim)
        up = UnifiedProblem(prob)
        o = Options(**{**opts.__dict__})
        if li < len(levels) - 1:
            o.tol = level_tol
        res = regularized_newton(up, up.to_x(phi), o)
        results.append(res)
        phi = up.to_phi(res.x)
        if li < len(levels) - 1:
            phi = prolong_fourier(phi)
    up = UnifiedProblem(prob)
    x = up.to_x(phi)
    return x / math.sqrt(re_dot(x, x)), prob, results
