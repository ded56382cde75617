"""Python binding of the C ABI (argument marshalling only).

Device memory and streams come from PyTorch: field arrays are CUDA/HIP
tensors, and every call runs on ``torch.cuda.current_stream()`` order.
All arithmetic happens in libgpe.so.
"""
from __future__ import annotations

import ctypes as C
import math

import torch

from . import _native as N


class GpeError(RuntimeError):
    def __init__(self, status, where):
        L = N.lib()
        msg = L.gpe_strerror(status).decode()
        extra = L.gpe_last_error().decode()
        super().__init__(f"{where}: status {status} ({msg}) {extra}".strip())
        self.status = status


def _check(status, where, allow=(N.GPE_OK,)):
    if status not in allow:
        raise GpeError(status, where)
    return status


_CTX = {}


def context(device=None):
    """Library context bound to ``device`` and the current torch stream."""
    if device is None:
        device = torch.cuda.current_device()
    stream = torch.cuda.current_stream(device).cuda_stream
    key = (int(device), int(stream))
    ctx = _CTX.get(key)
    if ctx is None:
        h = C.c_void_p()
        _check(N.lib().gpe_ctx_create(C.byref(h), int(device), C.c_void_p(stream)), "gpe_ctx_create")
        ctx = h
        _CTX[key] = ctx
    return ctx


def problem_struct(p, v=None):
    """gpe_problem from an object with the fields of workloads.Problem.
    ``v``: optional CUDA float64 tensor with the potential on the grid."""
    s = N.Problem()
    s.dim = int(p.dim)
    s.bc = {"fourier": N.GPE_BC_FOURIER, "sine": N.GPE_BC_SINE, "fd": N.GPE_BC_FD}[getattr(p, "bc", "fourier")]
    for i in range(3):
        s.n[i] = int(p.n[i]) if i < p.dim else 1
        s.lo[i] = float(p.lo[i]) if i < p.dim else 0.0
        s.hi[i] = float(p.hi[i]) if i < p.dim else 1.0
        s.gamma[i] = float(p.gamma[i])
    s.beta = float(p.beta)
    s.omega = float(p.omega)
    s.lattice_amp = float(getattr(p, "lattice_amp", 0.0))
    s.lattice_k = float(getattr(p, "lattice_k", math.pi / 4))
    if v is not None:
        _dev_tensor(v, torch.float64, "v", p)
    s.v = C.c_void_p(v.data_ptr()) if v is not None else None
    return s


def options(**kw):
    o = N.Options()
    N.lib().gpe_options_default(C.byref(o))
    prec = kw.pop("precision", None)
    if prec is not None:
        o.precision = {"fp64": N.GPE_PREC_FP64, "mixed": N.GPE_PREC_MIXED}.get(prec, prec)
    alg = kw.pop("algorithm", None)
    if alg is not None:
        o.algorithm = {"alg1": N.GPE_ALG1, "alg2": N.GPE_ALG2}.get(alg, alg)
    rule = kw.pop("stop_rule", None)
    if rule is not None:
        o.stop_rule = {"resid": N.GPE_STOP_RESID, "crit1": N.GPE_STOP_CRIT1,
                       "crit2": N.GPE_STOP_CRIT2}.get(rule, rule)
    step = kw.pop("step_at", None)
    if step is not None:
        o.step_at = {"auto": N.GPE_STEP_AUTO, "last_group": N.GPE_STEP_LAST_GROUP,
                     "kernel": N.GPE_STEP_KERNEL, "fused": N.GPE_STEP_FUSED}.get(step, step)
    thr = kw.pop("threads", None)
    if thr is not None:
        for i, t in enumerate(list(thr)[:3]):
            o.threads[i] = int(t)
    ept = kw.pop("elems", None)
    if ept is not None:
        for i, e in enumerate(list(ept)[:3]):
            o.elems[i] = int(e)
    for k, v in kw.items():
        if not hasattr(o, k):
            raise TypeError(f"unknown option {k}")
        setattr(o, k, v)
    return o


def _dev_tensor(t, dtype, name, p=None):
    if not (isinstance(t, torch.Tensor) and t.is_cuda):
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous {dtype} tensor")
    if p is not None and t.numel() != grid_points(p):
        raise ValueError(f"{name} has {t.numel()} elements; the grid of the problem has {grid_points(p)}")
    return t


def grid_points(p):
    """Number of grid values of a problem (the library reads exactly this many):
    n per axis (Fourier) or n - 1 interior points per axis (sine, finite
    differences)."""
    dirichlet = getattr(p, "bc", "fourier") in ("sine", "fd")
    m = 1
    for i in range(int(p.dim)):
        m *= int(p.n[i]) - (1 if dirichlet else 0)
    return m


SCALAR_NAMES = ("energy", "mu", "resid", "norm2", "rms_x", "rms_y", "rms_z", "max_dens",
                "e_kin", "e_pot")


def apply_h(p, phi, precision="fp64", v=None, scalars=True, out=None):
    """H(phi) phi on the problem's grid; returns (h_phi, scalars dict), or
    (h_phi, None) with ``scalars=False`` (no host wait: the call only
    enqueues work on the current stream).  ``out``: optional preallocated
    result tensor like ``phi``."""
    prec = N.GPE_PREC_FP64 if precision == "fp64" else N.GPE_PREC_MIXED
    dt = torch.complex128 if prec == N.GPE_PREC_FP64 else torch.complex64
    _dev_tensor(phi, dt, "phi", p)
    if out is None:
        out = torch.empty_like(phi)
    else:
        _dev_tensor(out, dt, "out", p)
    sc = (C.c_double * 10)() if scalars else None
    ps = problem_struct(p, v)
    _check(N.lib().gpe_apply_h(context(phi.device.index), C.byref(ps), prec, C.c_void_p(phi.data_ptr()),
                               C.c_void_p(out.data_ptr()), sc), "gpe_apply_h")
    return out, (dict(zip(SCALAR_NAMES, list(sc))) if scalars else None)


def apply_h_noalloc(p, phi, precision="fp64", v=None, out=None, scalars_out=None):
    """gpe_apply_h_noalloc: H(phi) phi through the library's fixed scratch
    (no device allocation in the call); ``scalars_out``: optional float64
    CUDA tensor of 10 elements receiving the scalars on the device."""
    prec, dt = _prec(precision)
    _dev_tensor(phi, dt, "phi", p)
    if out is None:
        out = torch.empty_like(phi)
    else:
        _dev_tensor(out, dt, "out", p)
    sp = None
    if scalars_out is not None:
        if not (isinstance(scalars_out, torch.Tensor) and scalars_out.is_cuda and scalars_out.dtype == torch.float64
                and scalars_out.is_contiguous() and scalars_out.numel() >= 10):
            raise TypeError("scalars_out must be a contiguous CUDA float64 tensor of at least 10 elements")
        sp = C.c_void_p(scalars_out.data_ptr())
    ps = problem_struct(p, v)
    _check(N.lib().gpe_apply_h_noalloc(context(phi.device.index), C.byref(ps), prec, C.c_void_p(phi.data_ptr()),
                                       C.c_void_p(out.data_ptr()), sp), "gpe_apply_h_noalloc")
    return out


def _prec(precision):
    prec = N.GPE_PREC_FP64 if precision == "fp64" else N.GPE_PREC_MIXED
    return prec, (torch.complex128 if prec == N.GPE_PREC_FP64 else torch.complex64)


def hess_vec(p, x_k, s, delta, v=None, precision="fp64"):
    """A s + 4 alpha (|x_k|^2 s + 2 Re(conj(x_k) s) x_k) + delta s (X units).
    x_k is complex128 in both precisions; s and the result are complex128
    ("fp64") or complex64 ("mixed")."""
    prec, dt = _prec(precision)
    _dev_tensor(x_k, torch.complex128, "x_k", p)
    _dev_tensor(s, dt, "s", p)
    out = torch.empty_like(s)
    ps = problem_struct(p, v)
    _check(N.lib().gpe_hess_vec(context(s.device.index), C.byref(ps), prec, C.c_void_p(x_k.data_ptr()),
                                C.c_void_p(s.data_ptr()), float(delta), C.c_void_p(out.data_ptr())),
           "gpe_hess_vec")
    return out


def retract(x, g, tau, precision="fp64"):
    """Cayley curve point y = p x + q g; returns (y, dict(p, q, a, nx, ng)).
    x, g and y are complex128 ("fp64") or complex64 ("mixed")."""
    prec, dt = _prec(precision)
    _dev_tensor(x, dt, "x")
    _dev_tensor(g, dt, "g")
    y = torch.empty_like(x)
    co = (C.c_double * 5)()
    _check(N.lib().gpe_retract(context(x.device.index), x.numel(), prec, C.c_void_p(x.data_ptr()),
                               C.c_void_p(g.data_ptr()), float(tau), C.c_void_p(y.data_ptr()), co),
           "gpe_retract")
    return y, dict(zip(("p", "q", "a", "nx", "ng"), list(co)))


def solve(p, phi0, v=None, **opts):
    """Ground state from phi0 (complex128 CUDA tensor); returns (phi, result dict)."""
    _dev_tensor(phi0, torch.complex128, "phi0", p)
    phi = phi0.clone()
    res = N.Result()
    ps = problem_struct(p, v)
    o = options(**opts)
    st = N.lib().gpe_solve(context(phi.device.index), C.byref(ps), C.byref(o), C.c_void_p(phi.data_ptr()),
                           C.byref(res))
    _check(st, "gpe_solve", allow=(N.GPE_OK, N.GPE_NOT_CONVERGED))
    return phi, res.as_dict()


def solve_batched(probs, phi0s, **opts):
    n = len(probs)
    phis = []
    for i, t in enumerate(phi0s):
        _dev_tensor(t, torch.complex128, f"phi0s[{i}]", probs[i])
        phis.append(t.clone())
    pa = (N.Problem * n)(*[problem_struct(p) for p in probs])
    ptrs = (C.c_void_p * n)(*[t.data_ptr() for t in phis])
    res = (N.Result * n)()
    o = options(**opts)
    st = N.lib().gpe_solve_batched(context(phis[0].device.index), n, pa, C.byref(o), ptrs, res)
    _check(st, "gpe_solve_batched", allow=(N.GPE_OK, N.GPE_NOT_CONVERGED))
    return phis, [r.as_dict() for r in res]


def autotune(p, precision="mixed", device=0):
    """Time the launch configurations for the grid of ``p`` and keep the
    fastest in the device's context; later solves on that grid use it where
    their options leave the choice open.  Returns the plan."""
    prec = N.GPE_PREC_FP64 if precision == "fp64" else N.GPE_PREC_MIXED
    thr = (C.c_int32 * 3)()
    ept = (C.c_int32 * 3)()
    step = C.c_int32()
    us = C.c_double()
    ps = problem_struct(p)
    _check(N.lib().gpe_autotune(context(device), C.byref(ps), prec, thr, ept, C.byref(step), C.byref(us)),
           "gpe_autotune")
    return {"threads": list(thr), "elems": list(ept), "step_at": step.value, "us_per_eval": us.value}


def set_plan(p, precision, threads, step_at, elems=None, device=0):
    """Keep a given launch plan (e.g. one returned by ``autotune`` earlier) for
    the grid of ``p`` in the device's context, as ``autotune`` keeps its own.
    ``elems``: points per thread of each pass (8 or 4; None for 8)."""
    prec = N.GPE_PREC_FP64 if precision == "fp64" else N.GPE_PREC_MIXED
    thr = (C.c_int32 * 3)(*[int(t) for t in list(threads)[:3]])
    ept = None if elems is None else (C.c_int32 * 3)(*[int(e) for e in list(elems)[:3]])
    ps = problem_struct(p)
    _check(N.lib().gpe_set_plan(context(device), C.byref(ps), prec, thr, ept, int(step_at)), "gpe_set_plan")


def prolong(p_coarse, p_fine, phi_c):
    _dev_tensor(phi_c, torch.complex128, "phi_c", p_coarse)
    shape = tuple(int(n) for n in reversed(p_fine.n[: p_fine.dim]))
    out = torch.empty(shape, dtype=torch.complex128, device=phi_c.device)
    a, b = problem_struct(p_coarse), problem_struct(p_fine)
    _check(N.lib().gpe_prolong(context(phi_c.device.index), C.byref(a), C.byref(b),
                               C.c_void_p(phi_c.data_ptr()), C.c_void_p(out.data_ptr())), "gpe_prolong")
    return out


def solve_cascadic(p_coarse_list, phi0s, nlevels, level_tol=1e-4, **opts):
    n = len(p_coarse_list)
    for i, t in enumerate(phi0s):
        _dev_tensor(t, torch.complex128, f"phi0s[{i}]", p_coarse_list[i])
    fine = []
    for p in p_coarse_list:
        shape = tuple(int(k) << (nlevels - 1) for k in reversed(p.n[: p.dim]))
        fine.append(torch.empty(shape, dtype=torch.complex128, device=phi0s[0].device))
    pa = (N.Problem * n)(*[problem_struct(p) for p in p_coarse_list])
    ins = (C.c_void_p * n)(*[t.data_ptr() for t in phi0s])
    outs = (C.c_void_p * n)(*[t.data_ptr() for t in fine])
    res = (N.Result * n)()
    o = options(**opts)
    st = N.lib().gpe_solve_cascadic(context(phi0s[0].device.index), n, pa, int(nlevels), float(level_tol),
                                    C.byref(o), ins, outs, res)
    _check(st, "gpe_solve_cascadic", allow=(N.GPE_OK, N.GPE_NOT_CONVERGED))
    return fine, [r.as_dict() for r in res]
