/*
 * gpe.h -- C ABI of the MI355X ground-state library.
 *
 * Computes ground states of a Bose-Einstein condensate, the minimiser of the
 * discretised Gross-Pitaevskii energy on the unit sphere, with the feasible
 * gradient method (BB step, Cayley retraction, nonmonotone search; §3.1,
 * Algorithm 1) and the regularized Newton method (§3.2, Algorithm 2), on one
 * AMD Instinct MI355X (gfx950).  The problem statement follows §1-§2 of the
 * paper: a box U, a grid, a trap V, interaction beta and rotation Omega in;
 * the ground state phi, energy E, chemical potential mu and residual
 * ||H(phi)phi - mu phi||_inf out.
 *
 * Conventions shared by every entry point:
 *  - Grid (Fourier pseudospectral, §2.3): n[i] unique periodic points per
 *    axis, x_j = lo[i] + j h_i, h_i = (hi[i]-lo[i]) / n[i], j = 0..n[i]-1.
 *    n[i] must be a power of two, 16 <= n[i] <= 1024.
 *  - Layout: x fastest, then y, then z; interleaved (re, im) complex.
 *  - phi is in physical units: ||phi||_h^2 = h_vol sum |phi_j|^2 (h_vol = prod h_i).
 *  - "X units" (the unified problem of §3): X = sqrt(h_vol) phi, so that
 *    ||X||_2 = ||phi||_h, F(X) = E_h(phi), A = 2 H_lin, alpha = beta/(2 h_vol).
 *  - Every pointer to field data is DEVICE memory owned by the caller; the
 *    library keeps no pointer after a call returns.  Host pointers (problem,
 *    options, result, scalars) are read or written during the call only.
 *  - All device work is ordered on the context's stream (gpe_ctx_create).
 *  - Errors are status codes; no C++ exception crosses this interface.  A
 *    context must not be used from two threads at once.
 *  - Environment: GPE_PROGRESS=<seconds> makes the solvers print a progress
 *    line on stderr (evaluations so far, problems finished) at host checks at
 *    least that many seconds apart.
 */
#ifndef GPE_H
#define GPE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define GPE_OK               0
#define GPE_NOT_CONVERGED    1   /* iteration cap hit; outputs hold the last iterate */
#define GPE_EINVAL          -1   /* null pointer, bad dim/box/sizes, Omega != 0 where not allowed, zero phi0 */
#define GPE_EUNSUPPORTED    -2   /* n not a power of two in [16, 1024] ([16, 512] for GPE_BC_SINE),
                                    or an unsupported combination */
#define GPE_ENOMEM          -3   /* device allocation failed */
#define GPE_EDEVICE         -4   /* HIP runtime error (see gpe_last_error) */
#define GPE_ENONFINITE      -5   /* a reduction became NaN/Inf (bad V, phi0 or divergence) */

/* ---- enumerations ------------------------------------------------------ */
#define GPE_BC_FOURIER       0   /* periodic, Fourier pseudospectral (§2.3) */
#define GPE_BC_SINE          1   /* homogeneous Dirichlet, sine pseudospectral (§2.2, DST-I);
                                    Omega must be 0 */
#define GPE_BC_FD            2   /* homogeneous Dirichlet, second-order finite differences (§2.1):
                                    per axis the tridiagonal 1/h^2, -1/(2h^2) kinetic matrix on the
                                    n-1 interior points; Omega must be 0 */

#define GPE_PREC_FP64        0   /* every array and FFT in float64 */
#define GPE_PREC_MIXED       1   /* FP32 FFT/pointwise bulk, FP64 reductions, scalars and outer Newton state */

#define GPE_ALG1             1   /* Algorithm 1 alone (§3.1) */
#define GPE_ALG2             2   /* Algorithm 2: K_init steps of Algorithm 1, then regularized Newton (§3.2) */

/* Stop rules (§4).  Norms of X = sqrt(h_vol) phi, the iterate on the unit sphere.
   RESID: the residual ||H(phi)phi - mu phi||_inf < tol (tested at every iterate).
   CRIT1: ||X^{k+1} - X^k||_inf / tau_k <= eps0 after an accepted step of Algorithm 1
          (run alone, or in the first k_init steps of Algorithm 2; the Newton loop
          then uses RESID).
   CRIT2: ||X^{k+1} - X^k||_inf <= crit2_tol after an accepted Newton step of
          Algorithm 2 (the first k_init steps use RESID), or after an accepted step
          of Algorithm 1 run alone.  A rejected Newton step leaves X unchanged and
          is not tested. */
#define GPE_STOP_RESID       0
#define GPE_STOP_CRIT1       1
#define GPE_STOP_CRIT2       2

/* Placement of the scalar step (line search / trust-region update) that
   follows each evaluation; results do not depend on it (every placement
   reduces the same partial sums in the same order). */
#define GPE_STEP_AUTO       -1   /* LAST_GROUP when the final pass has at most 128 workgroups
                                    per problem (always in 1D), else KERNEL */
#define GPE_STEP_LAST_GROUP  0   /* last workgroup of the final pass (a device-scope fence per workgroup) */
#define GPE_STEP_KERNEL      1   /* a launch of its own after the final pass */
#define GPE_STEP_FUSED       2   /* at the start of the next evaluation's first pass, by every
                                    workgroup of that pass on its own copy of the state (two
                                    or three launches per evaluation instead of three or four;
                                    dim >= 2, else LAST_GROUP; the chunk is rounded up to even) */

/* ---- problem ------------------------------------------------------------ */
typedef struct gpe_problem {
    int32_t dim;          /* 1, 2 or 3 */
    int32_t bc;           /* GPE_BC_FOURIER, GPE_BC_SINE or GPE_BC_FD */
    int32_t n[3];         /* per axis (x, y, z), entries beyond dim ignored.  Fourier: n periodic
                             points x_j = lo + j h, j < n.  Sine and finite differences: n
                             intervals, n-1 interior points x_j = lo + j h, 0 < j < n.
                             h = (hi - lo)/n.  Arrays hold the points of every axis, x fastest */
    double lo[3], hi[3];  /* box U = prod (lo_i, hi_i), lo_i < hi_i */
    double beta;          /* interaction constant */
    double omega;         /* rotation speed; must be 0 when dim == 1 or bc is GPE_BC_SINE or GPE_BC_FD */
    double gamma[3];      /* harmonic trap V = 1/2 sum gamma_i^2 x_i^2 (§1) */
    double lattice_amp;   /* optical lattice A * sum sin^2(k x_i) (§4.2, §4.4); 0 = none */
    double lattice_k;     /* k of the lattice (pi/4 in the paper) */
    const double* v;      /* optional DEVICE array of V (float64, grid layout); NULL = analytic V */
} gpe_problem;

/* ---- options (defaults from gpe_options_default) ------------------------ */
typedef struct gpe_options {
    int32_t precision;    /* GPE_PREC_FP64 or GPE_PREC_MIXED */
    int32_t algorithm;    /* GPE_ALG1 or GPE_ALG2 */
    double tol;           /* GPE_STOP_RESID: stop when ||H(phi)phi - mu phi||_inf < tol (phi units) */
    int32_t k_init;       /* Algorithm 1 steps before the Newton loop (100, §4.3) */
    int32_t k_sub;        /* max Algorithm 1 steps per Newton subproblem (200, §4.3) */
    int32_t max_outer;    /* max Newton steps */
    int32_t max_iter;     /* max steps of Algorithm 1 when run alone */
    int32_t m_max;        /* max backtracks per step (the last trial is taken) */
    double tau0;          /* first BB step */
    double rho1, eta, sigma;              /* nonmonotone Armijo: rho_1, eta, backtracking factor */
    double renorm_tol;                    /* renormalise when | ||X||^2 - 1 | > renorm_tol (§4) */
    double eta1, eta2, gamma_shrink, gamma_grow;  /* trust-region ratio test and delta update (§3.2) */
    double delta0, delta_min, delta_max;          /* regularisation delta */
    int32_t chunk;        /* evaluations per host check of the done flags (graph size); in a
                             batch, finished problems are dropped from the launches at these
                             checks */
    int32_t use_graph;    /* 1: replay chunks as a captured hipGraph; 0: plain launches */
    int32_t profile;      /* k > 0: time the last-axis pass of every k-th evaluation with a pair of
                             HIP events: stamped by the kernel's own dispatch with plain launches
                             (use_graph 0), event record nodes around it inside a graph (these
                             add the event packets' time, a few microseconds); 0: off */
    int32_t real_field;   /* -1 (default): real arithmetic for each problem with Omega = 0 whose
                             phi0 has a zero imaginary part; 1: real arithmetic for every problem
                             (Omega must be 0 for all); 0: complex.  In real arithmetic the
                             iterates stay exactly real (the method on the unit sphere of R^M;
                             otherwise rounding noise in their imaginary parts can grow and lead
                             the iteration to a complex stationary state): a real problem on a
                             Fourier grid in 2D or 3D keeps its arrays as real values, two grid
                             points to a complex element, with half the bytes and transform work
                             (two real lines per complex transform, the Omega = 0 multiplier
                             being real and even); others drop the imaginary parts after every
                             evaluation.  A problem's choice depends on its own phi0 only */
    int32_t threads[3];   /* workgroup size of the x, y, z passes (0 = built-in choice);
                             a multiple of 64 and of n/elems, at most 256 */
    int32_t step_at;      /* where the scalar step of the solver runs (GPE_STEP_*) */
    int32_t stop_rule;    /* GPE_STOP_RESID (default), GPE_STOP_CRIT1 or GPE_STOP_CRIT2 */
    int32_t monotone;     /* 1: monotone Armijo search, C = F(X_k) (eta = 0); 0: Zhang-Hager */
    double eps0;          /* GPE_STOP_CRIT1 threshold (1e-6, §4) */
    double crit2_tol;     /* GPE_STOP_CRIT2 threshold delta_0 (1e-8, §4) */
    int32_t switch_window;/* mixed precision, Algorithm 1: when the residual has not halved in
                             this many accepted steps (the FP32 floor), or when an FP32 residual
                             meets tol, continue from the current iterate in FP64 with the
                             remaining steps (the stop test is then taken in FP64); 0 = never:
                             the FP32 residual decides (default 100) */
    int32_t reserved1;
    double switch_resid;  /* mixed precision, Algorithm 2: once the residual of an outer (FP64)
                             evaluation is below switch_resid but not yet below tol, the outer
                             iterate X_k starts an FP64 run of Algorithm 2 (its K_init steps of
                             Algorithm 1 first, the regularisation delta kept) with the remaining
                             Newton steps (in a batch: the budget left to the problem that used
                             the most), since the Newton subproblems in FP32 stall near the FP32
                             residual floor.  0 = never (default 1e-4, about ten times the floor
                             of the benchmark grids) */
    int32_t elems[3];     /* transform points per thread in the x, y, z passes: 8 or 4 (0 = built-in
                             choice: 4 below 2^20 grid points in all, else 8).  4 gives each line
                             twice the threads with half the work each (shorter chains where a
                             pass is latency bound); the workgroup size (threads) must be a multiple
                             of the line's threads, n/elems */
    int32_t reserved3;
} gpe_options;

/* ---- results ------------------------------------------------------------ */
typedef struct gpe_result {
    int32_t status;       /* GPE_OK / GPE_NOT_CONVERGED / negative error */
    int32_t outer_iters;  /* Newton steps taken */
    int32_t inner_iters;  /* Algorithm 1 steps taken (all runs) */
    int32_t nfe;          /* function+gradient evaluations (all precisions) */
    int32_t nfe_fp64;     /* of which evaluated in float64 */
    int32_t backtracks;   /* step-size reductions */
    int32_t rejections;   /* rejected Newton trial points */
    int32_t switch_iter;  /* mixed precision: Algorithm 1 steps (alone, or the K_init and inner
                             steps of Algorithm 2) taken in FP32 before the FP64 continuation
                             (at least 1 when it took place; 0 = no switch) */
    double energy;        /* E_h(phi)  (§2) */
    double mu;            /* E + beta/2 int |phi|^4  (§1) */
    double resid;         /* ||H(phi)phi - mu phi||_inf */
    double norm_err;      /* ||phi||_h^2 - 1 */
    double rms[3];        /* sqrt(int x_i^2 |phi|^2)  (§4, rms) */
    double max_dens;      /* max |phi|^2 */
    double delta;         /* final regularisation delta */
    double time_ms;       /* device time of the evaluation loop (events on the context stream;
                             setup, graph instantiation and the output pass excluded) */
    int32_t nfe_f;        /* evaluations of F in Algorithm 1 (including the initial one) */
    int32_t nfe_w;        /* evaluations of the Newton model W */
    int32_t nfe_outer;    /* float64 evaluations of F at outer iterates */
    int32_t pass_launches;/* profile: timed (sampled) launches of the last-axis pass */
    double pass_ms;       /* profile: summed event time of those launches */
    int32_t nfe_mixed[3]; /* of nfe_f, nfe_w, nfe_outer: the evaluations run by the mixed-precision
                             passes (the rest ran in an FP64 continuation or an FP64 solve) */
    int32_t storage;      /* the solver's arrays: 0 complex; 1 real arithmetic in complex elements
                             (imaginary parts dropped); 2 real values, two grid points to an
                             element (see real_field) */
} gpe_result;

typedef struct gpe_ctx gpe_ctx;

/* Create a context on HIP device `device`.  `stream` is a hipStream_t the
 * caller owns (NULL = the legacy default stream); the library orders its own
 * work after the caller's work on it and makes the caller's stream wait for
 * the library's work before returning.  Returns GPE_OK or an error. */
int gpe_ctx_create(gpe_ctx** out, int device, void* stream);
/* Free every device buffer the context owns.  Safe on NULL. */
int gpe_ctx_destroy(gpe_ctx* ctx);

void gpe_options_default(gpe_options* opts);
const char* gpe_strerror(int status);
/* Text of the last HIP error seen by the calling thread ("" if none). */
const char* gpe_last_error(void);

/*
 * H(phi) phi = (-1/2 Laplacian + V - Omega L_z + beta |phi|^2) phi on the
 * Fourier grid (§1; operator of §2.3 with the per-axis multipliers
 * lambda^2/2 + Omega y lambda on x-lines and eta^2/2 - Omega x eta on y-lines).
 *   precision  GPE_PREC_FP64: phi, h_phi are complex128;
 *              GPE_PREC_MIXED: complex64 arrays, FP32 FFTs, FP64 reductions.
 *   phi        DEVICE input (not modified); h_phi DEVICE output (may not alias phi).
 *   scalars    HOST double[10] out or NULL: E_h(phi), mu = E + beta/2 int|phi|^4,
 *              ||H(phi)phi - mu phi||_inf, ||phi||_h^2, rms x, y, z, max|phi|^2,
 *              kinetic+rotation part of E, potential part of E.
 * Blocks until the scalars are on the host when scalars != NULL.  With
 * scalars == NULL and the same problem as the context's previous apply call
 * (nothing to upload) the call only enqueues work and returns at once; the
 * scalars are still computed on the device.
 */
int gpe_apply_h(gpe_ctx* ctx, const gpe_problem* prob, int32_t precision,
                const void* phi, void* h_phi, double* scalars);

/*
 * gpe_apply_h for callers that cannot allocate device memory: code under
 * stream capture, tight serving loops, harnesses that forbid hipMalloc.  The
 * same H(phi)phi and scalars as gpe_apply_h (the same kernels), with every
 * intermediate (descriptor, potential tables, partial sums, the passes'
 * accumulator) in one fixed scratch array per GPU that the library sets up
 * in gpe_ctx_create and holds until the process ends (about 35 MB); the
 * call allocates nothing and never waits on the host.
 *   Limit: at most 2^21 grid points; larger grids return GPE_EUNSUPPORTED
 *   (gpe_last_error says why) before any device work.
 *   phi, h_phi: DEVICE arrays as for gpe_apply_h (complex128, or complex64
 *   with GPE_PREC_MIXED).
 *   scalars_dev: DEVICE double[10] out (the scalars of gpe_apply_h, same
 *   order), or NULL.
 *   The trap and lattice tables are evaluated on the device (the same
 *   formula as gpe_apply_h's host tables, so V may differ in its last bit).
 *   Every call on a GPU reuses that GPU's scratch: calls that overlap on one
 *   GPU (two contexts, two host threads, two streams) race; calls ordered on
 *   one stream do not.  Nothing in the scratch needs clearing between calls.
 */
int gpe_apply_h_noalloc(gpe_ctx* ctx, const gpe_problem* prob, int32_t precision,
                        const void* phi, void* h_phi, double* scalars_dev);

/*
 * Hessian-vector product of the regularized Newton model (Lemma 3.1, §3.2),
 * in X units:  out = A s + 4 alpha (|x_k|^2 s + 2 Re(conj(x_k) s) x_k) + delta s.
 *   precision  GPE_PREC_FP64: s and out complex128, transforms in float64;
 *              GPE_PREC_MIXED: s and out complex64, transforms of s in
 *              float32, the pointwise terms in float64 rounded to float32 on
 *              store (the solver's Newton passes in mixed precision).
 *   x_k        DEVICE complex128 in both precisions (the outer iterate stays
 *              float64); s, out DEVICE (out may not alias the inputs).
 */
int gpe_hess_vec(gpe_ctx* ctx, const gpe_problem* prob, int32_t precision, const void* x_k,
                 const void* s, double delta, void* out);

/*
 * Cayley retraction (§3.1, Theorem 3.3) in the real reading: with
 * a = Re(x^* g), n_x = ||x||^2, n_g = ||g||^2,
 *   y = p x + q g,  p = ((1 + tau a)^2 - tau^2 n_x n_g)/den,  q = -2 tau n_x/den,
 *   den = 1 - tau^2 a^2 + tau^2 n_x n_g.
 *   precision  GPE_PREC_FP64: x, g, y complex128; GPE_PREC_MIXED: complex64
 *              (a, n_x, n_g summed and p, q formed in float64 either way).
 * x, g, y: DEVICE arrays of m elements (y may alias neither).
 * coeffs: HOST double[5] out or NULL: p, q, a, n_x, n_g.  Blocks when coeffs
 * is not NULL.
 */
int gpe_retract(gpe_ctx* ctx, int64_t m, int32_t precision, const void* x, const void* g,
                double tau, void* y, double* coeffs);

/*
 * Ground state by Algorithm 1 or 2 (§3).  phi: DEVICE complex128 array; on
 * entry the initial guess phi_0 (need not be normalised, must be nonzero),
 * on exit the computed state with ||phi||_h = 1.  The result's energy, mu,
 * resid, rms and max_dens are recomputed in float64 from the returned phi.
 * Returns result->status.
 */
int gpe_solve(gpe_ctx* ctx, const gpe_problem* prob, const gpe_options* opts,
              void* phi, gpe_result* result);

/*
 * `count` independent problems solved together: every evaluation step runs
 * all unfinished problems in the same kernel launches (one launch per pass
 * for each group of problems that share a precision and a storage; in mixed
 * precision a problem moves to the FP64 group when it hands over, at the
 * host check after it does, while the others go on).  Problems may differ
 * in beta, Omega, V, discretization and n (same dim); each problem's
 * trajectory is that of the same problem solved alone with the same launch
 * plan.  phis[i]: DEVICE
 * complex128 arrays.  results: HOST array of `count`.  Returns GPE_OK if
 * every problem converged, GPE_NOT_CONVERGED if any did not, or the first
 * error.
 */
int gpe_solve_batched(gpe_ctx* ctx, int32_t count, const gpe_problem* probs,
                      const gpe_options* opts, void* const* phis, gpe_result* results);

/*
 * Tuning of the launch configuration for one grid (dim, n, bc) and precision:
 * short solves of a synthetic state on that grid time 8 and 4 transform
 * points per thread, every valid workgroup size per pass (64, 128, 256
 * threads, a multiple of n/points) and every step placement (GPE_STEP_FUSED up
 * to 512 first-pass workgroups, in 2D and 3D); the fastest plan is kept in
 * the context (one per grid and
 * precision, replaced by a later call).  Later gpe_solve / gpe_solve_batched /
 * gpe_solve_cascadic calls on a context with a plan for their grid use it
 * wherever their options leave the choice open (threads and elems 0, step_at
 * AUTO).
 * A plan changes the tiling, hence the order of the float64 reductions, not
 * the method.  threads_out[3], elems_out[3], step_at_out, us_per_eval_out:
 * HOST, optional (the chosen plan and its time per evaluation in
 * microseconds).  Takes a few hundred milliseconds to seconds; allocates
 * device workspace in the context.
 */
int gpe_autotune(gpe_ctx* ctx, const gpe_problem* prob, int32_t precision, int32_t* threads_out,
                 int32_t* elems_out, int32_t* step_at_out, double* us_per_eval_out);

/*
 * Keep a given launch plan for the grid of `prob` and `precision` in the
 * context, as gpe_autotune keeps the plan it picks (replacing an earlier one):
 * for instance a plan recorded from an earlier gpe_autotune call, so that
 * later runs tile the grid the same way and take the same bits.
 * threads: HOST int32[3], the workgroup size of the x, y, z passes (entries
 * beyond the problem's dimension ignored), each 64, 128 or 256 and a multiple
 * of the pass's threads per line (the transform length / elems); elems: HOST
 * int32[3], the points per thread of each pass (8 or 4), or NULL for 8;
 * step_at: GPE_STEP_LAST_GROUP, GPE_STEP_KERNEL or GPE_STEP_FUSED.
 * GPE_EINVAL for anything else.
 * Host only: no device work.
 */
int gpe_set_plan(gpe_ctx* ctx, const gpe_problem* prob, int32_t precision, const int32_t* threads,
                 const int32_t* elems, int32_t step_at);

/*
 * Trigonometric prolongation for the cascadic multigrid (Algorithm 3): the
 * coarse grid function (n points per axis) is interpolated to 2n points per
 * axis on the same box (coarse points are every other fine point); per axis
 * the spectrum is zero-padded and the coarse Nyquist coefficient split half
 * and half between +n and -n.  phi_c, phi_f: DEVICE complex128 arrays.
 * fine must equal coarse with every n doubled.  Fourier problems only
 * (GPE_EUNSUPPORTED for GPE_BC_SINE and GPE_BC_FD).
 */
int gpe_prolong(gpe_ctx* ctx, const gpe_problem* coarse, const gpe_problem* fine,
                const void* phi_c, void* phi_f);

/*
 * Algorithm 3: cascadic multigrid over `nlevels` grids (n doubling per
 * level, coarse problem given) for `count` problems in one solve: coarse
 * levels to `level_tol`, the finest to opts->tol.  Each problem moves on by
 * itself: when it ends a coarse level its iterate is prolonged (as
 * gpe_prolong) and starts the next level's solve, in the options' precision
 * with a fresh step state, at the solver's next host check, while the other
 * problems continue on their own levels (in mixed precision a level's FP64
 * continuation runs the same way).  phi0s[i]: DEVICE complex128 initial data
 * on the coarse grid, read at the start only; phis[i]: DEVICE complex128
 * outputs on the finest grid, also the write-back space of the coarse levels.
 * Fourier problems only.  results[i]: the finest level's outputs (E, mu,
 * residual, ...); every counter (iterations, evaluations by kind and
 * precision, backtracks, rejections, switch_iter) summed over the levels;
 * profile samples and time are the whole solve's.  The status is the worst
 * of the levels' (a coarse level stopped at its cap reports
 * GPE_NOT_CONVERGED); a problem the evaluation cap stops on a coarse level
 * returns its iterate prolonged to the finest grid and GPE_NOT_CONVERGED.
 */
int gpe_solve_cascadic(gpe_ctx* ctx, int32_t count, const gpe_problem* coarse,
                       int32_t nlevels, double level_tol, const gpe_options* opts,
                       void* const* phi0s, void* const* phis, gpe_result* results);

#ifdef __cplusplus
}
#endif
#endif /* GPE_H */
