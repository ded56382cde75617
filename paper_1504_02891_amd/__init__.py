"""MI355X ground-state library: regularized Newton method for Bose-Einstein
condensates (Fourier pseudospectral discretization, feasible BB gradient
method, trust-region Newton, cascadic multigrid) as hand-written HIP kernels
behind a C ABI (include/gpe.h).  This package is the thin Python binding;
``paper_1504_02891_amd.api`` holds the torch-facing functions."""
from ._native import LIB_PATH, lib  # noqa: F401
