"""ctypes mirror of include/gpe.h and the loader of libgpe.so.

The library must have been built (python paper_1504_02891_amd/csrc/build.py);
there is no fallback implementation: loading fails loudly without it.
"""
from __future__ import annotations

import ctypes as C
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libgpe.so")

GPE_OK = 0
GPE_NOT_CONVERGED = 1
GPE_EINVAL = -1
GPE_EUNSUPPORTED = -2
GPE_ENOMEM = -3
GPE_EDEVICE = -4
GPE_ENONFINITE = -5

GPE_BC_FOURIER = 0
GPE_BC_SINE = 1
GPE_BC_FD = 2
GPE_PREC_FP64 = 0
GPE_PREC_MIXED = 1
GPE_ALG1 = 1
GPE_ALG2 = 2
GPE_STEP_AUTO = -1
GPE_STEP_LAST_GROUP = 0
GPE_STEP_KERNEL = 1
GPE_STEP_FUSED = 2
GPE_STOP_RESID = 0
GPE_STOP_CRIT1 = 1
GPE_STOP_CRIT2 = 2

EXPORTS = ("gpe_ctx_create", "gpe_ctx_destroy", "gpe_options_default", "gpe_strerror",
           "gpe_last_error", "gpe_apply_h", "gpe_apply_h_noalloc", "gpe_hess_vec", "gpe_retract", "gpe_solve",
           "gpe_solve_batched", "gpe_prolong", "gpe_solve_cascadic", "gpe_autotune", "gpe_set_plan")


class Problem(C.Structure):
    _fields_ = [("dim", C.c_int32), ("bc", C.c_int32), ("n", C.c_int32 * 3),
                ("lo", C.c_double * 3), ("hi", C.c_double * 3),
                ("beta", C.c_double), ("omega", C.c_double), ("gamma", C.c_double * 3),
                ("lattice_amp", C.c_double), ("lattice_k", C.c_double), ("v", C.c_void_p)]


class Options(C.Structure):
    _fields_ = [("precision", C.c_int32), ("algorithm", C.c_int32), ("tol", C.c_double),
                ("k_init", C.c_int32), ("k_sub", C.c_int32), ("max_outer", C.c_int32),
                ("max_iter", C.c_int32), ("m_max", C.c_int32),
                ("tau0", C.c_double), ("rho1", C.c_double), ("eta", C.c_double), ("sigma", C.c_double),
                ("renorm_tol", C.c_double),
                ("eta1", C.c_double), ("eta2", C.c_double), ("gamma_shrink", C.c_double),
                ("gamma_grow", C.c_double),
                ("delta0", C.c_double), ("delta_min", C.c_double), ("delta_max", C.c_double),
                ("chunk", C.c_int32), ("use_graph", C.c_int32), ("profile", C.c_int32),
                ("real_field", C.c_int32), ("threads", C.c_int32 * 3), ("step_at", C.c_int32),
                ("stop_rule", C.c_int32), ("monotone", C.c_int32), ("eps0", C.c_double),
                ("crit2_tol", C.c_double), ("switch_window", C.c_int32), ("reserved1", C.c_int32),
                ("switch_resid", C.c_double), ("elems", C.c_int32 * 3), ("reserved3", C.c_int32)]


class Result(C.Structure):
    _fields_ = [("status", C.c_int32), ("outer_iters", C.c_int32), ("inner_iters", C.c_int32),
                ("nfe", C.c_int32), ("nfe_fp64", C.c_int32), ("backtracks", C.c_int32),
                ("rejections", C.c_int32), ("switch_iter", C.c_int32),
                ("energy", C.c_double), ("mu", C.c_double), ("resid", C.c_double),
                ("norm_err", C.c_double), ("rms", C.c_double * 3), ("max_dens", C.c_double),
                ("delta", C.c_double), ("time_ms", C.c_double),
                ("nfe_f", C.c_int32), ("nfe_w", C.c_int32), ("nfe_outer", C.c_int32),
                ("pass_launches", C.c_int32), ("pass_ms", C.c_double),
                ("nfe_mixed", C.c_int32 * 3), ("storage", C.c_int32)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k not in ("rms", "nfe_mixed")}
        d["rms"] = list(self.rms)
        d["nfe_mixed"] = list(self.nfe_mixed)
        return d


_lib = None


def lib():
    """The loaded libgpe.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python paper_1504_02891_amd/csrc/build.py` (needs hipcc)")
    L = C.CDLL(LIB_PATH)
    vp, i32, dbl = C.c_void_p, C.c_int32, C.c_double
    L.gpe_ctx_create.argtypes = [C.POINTER(vp), C.c_int, vp]
    L.gpe_ctx_destroy.argtypes = [vp]
    L.gpe_options_default.argtypes = [C.POINTER(Options)]
    L.gpe_options_default.restype = None
    L.gpe_strerror.argtypes = [C.c_int]
    L.gpe_strerror.restype = C.c_char_p
    L.gpe_last_error.argtypes = []
    L.gpe_last_error.restype = C.c_char_p
    L.gpe_apply_h.argtypes = [vp, C.POINTER(Problem), i32, vp, vp, C.POINTER(dbl)]
    L.gpe_apply_h_noalloc.argtypes = [vp, C.POINTER(Problem), i32, vp, vp, vp]
    L.gpe_hess_vec.argtypes = [vp, C.POINTER(Problem), i32, vp, vp, dbl, vp]
    L.gpe_retract.argtypes = [vp, C.c_int64, i32, vp, vp, dbl, vp, C.POINTER(dbl)]
    L.gpe_solve.argtypes = [vp, C.POINTER(Problem), C.POINTER(Options), vp, C.POINTER(Result)]
    L.gpe_solve_batched.argtypes = [vp, i32, C.POINTER(Problem), C.POINTER(Options), C.POINTER(vp),
                                    C.POINTER(Result)]
    L.gpe_prolong.argtypes = [vp, C.POINTER(Problem), C.POINTER(Problem), vp, vp]
    L.gpe_autotune.argtypes = [vp, C.POINTER(Problem), i32, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32),
                               C.POINTER(dbl)]
    L.gpe_set_plan.argtypes = [vp, C.POINTER(Problem), i32, C.POINTER(i32), C.POINTER(i32), i32]
    L.gpe_solve_cascadic.argtypes = [vp, i32, C.POINTER(Problem), i32, dbl, C.POINTER(Options),
                                     C.POINTER(vp), C.POINTER(vp), C.POINTER(Result)]
    for name in EXPORTS:
        f = getattr(L, name)
        if f.restype is C.c_int:  # default
            f.restype = C.c_int
    _lib = L
    return L
