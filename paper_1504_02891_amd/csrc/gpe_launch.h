// Host-side launchers of the device kernels (one translation unit each).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <algorithm>
#include "gpe_state.h"

namespace gpe {
// bmap: null for a single problem; st_in/st_out: the state arrays read and
// (STEP_FUSED, first pass) written; par: the evaluation's parity under
// STEP_FUSED, else 0; ev0/ev1 (optional, plain launches only): events stamped
// by the dispatch itself at the kernel's start and end; reread (final and
// solo roles): the epilogue re-reads the trial inputs; fused (first role):
// the pass runs the previous evaluation's scalar step (STEP_FUSED); ept:
// transform points per thread of the pass (8 or 4); pair: the problems store
// real grid functions two points to an element (not the 1D pass)
void launch_solver_pass(hipStream_t s, int role, int prec64, int nblocks, int threads, size_t smem,
                        const ProbDev* probs, SolverState* st_in, SolverState* st_out, const int2* bmap,
                        const void* twd, const void* twf, int par, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr,
                        int reread = 0, int fused = 0, int ept = kE, int pair = 0);
void launch_apply_pass(hipStream_t s, int role, int fp64, int nblocks, int threads, size_t smem,
                       const ProbDev* probs, const ApplyArgs& a, const void* tw);
// the scalar step of every problem (its precision from its descriptor)
void launch_step(hipStream_t s, int nprob, const ProbDev* probs, SolverState* st);
void launch_init(hipStream_t s, const ProbDev* probs, int pi, int64_t m, const void* phi0, int prec64);
void launch_write_phi(hipStream_t s, const ProbDev* probs, const SolverState* st, int pi, int64_t m, void* phi,
                      int prec64);
// the last pass's nsum partials per slot into tot[SA_COUNT * 16] (16 chunk
// totals per slot), then per-block residual maxima (rpart) with mu from them
void launch_apply_resid(hipStream_t s, int nblk, const ProbDev* probs, int nsum, const void* phi,
                        const void* hphi, double* rpart, double* tot, int fp64);
// out[0..9]: the scalars of gpe_apply_h from tot and the residual maxima
void launch_apply_finalize(hipStream_t s, const ProbDev* probs, const double* tot, const double* rpart, int nr,
                           double* out);
// fp64: complex128 x, g, y; else complex64 (reductions and coefficients in float64 either way)
void launch_retract(hipStream_t s, int nblk, const void* x, const void* g, void* y, int64_t m, double tau,
                    double* part, double* coeffs, int fp64);
// per-block max |Im x_i| of a complex128 array (part[nblk])
void launch_max_imag(hipStream_t s, int nblk, const void* x, int64_t m, double* part);
// Fixed scratch of the no-allocation entry point (k_noalloc.hip):
// noalloc_init looks up the device's copy of the array (with `device`
// current; 0 or a hipError_t), noalloc_scratch returns it (null before init).
int noalloc_init(int device);
char* noalloc_scratch(int device);
void launch_setup_desc(hipStream_t s, const ProbDev& d, const VAxisParams& vp, ProbDev* dst, double* vaxis);
// trigonometric prolongation of a complex128 array of shape (n0, n1, n2)
// along axis `ax` (that length doubled in `out`); -1 for a length outside
// 16 .. 512
int launch_prolong_axis(hipStream_t s, const void* in, void* out, int n0, int n1, int n2, int ax,
                        const void* twd);
}  // namespace gpe
