// Plain structs shared by the host driver and the device kernels.
#pragma once
#include <stdint.h>

namespace gpe {

constexpr int kMaxN = 1024;          // largest points per axis
constexpr int kTwN = 1024;           // twiddle table length: exp(-2 pi i m / 1024)
constexpr int kE = 8;                // line elements held per thread in the passes

// Reduction slots of the first pass of an evaluation (sums and one max).
enum Slot1 { S1_NY = 0, S1_NP2, S1_COUNT_SUM, S1_RMAX = S1_COUNT_SUM, S1_COUNT };
// Reduction slots of the final pass of a solver evaluation.
enum SlotF {
  SF_F = 0,   // f(Y): F in F-mode, f_W in W-mode
  SF_A,       // Re(Y^* g_Y)
  SF_NG,      // ||g_Y||^2
  SF_NY,      // ||Y||^2 of the stored trial
  SF_SS,      // ||S||^2,  S = Y - X_base
  SF_SY,      // Re(S^* Y)
  SF_SG,      // Re(S^* g_Y)
  SF_SW0,     // Re(S^* W0)
  SF_W0W0,    // ||W0||^2
  SF_W0G,     // Re(W0^* g_Y)
  SF_W0Y,     // Re(W0^* Y)
  SF_ARED,    // actual reduction F(Z) - F(X_k) in difference form (W-mode)
  SF_COUNT_SUM,
  SF_SMAX = SF_COUNT_SUM,  // max |S_j|
  SF_COUNT
};
// Reduction slots of apply_h (phi units): sums of the last pass, sum
// Re(conj(phi) H phi), sum |phi|^4, sum V |phi|^2 ...
enum SlotA { SA_MU = 0, SA_QUART, SA_POT, SA_COUNT };
// ... and of the residual pass: norm, second moments, then the maxima of
// |phi|^2 and |H phi - mu phi|^2.
enum SlotR { SR_NORM = 0, SR_X2, SR_Y2, SR_Z2, SR_COUNT_SUM, SR_MAXD = SR_COUNT_SUM, SR_RES, SR_COUNT };

// Roles of the directional passes of one evaluation.
enum Role { R_FIRST = 0, R_MID = 1, R_FINAL = 2, R_SOLO = 3 };

// Evaluation modes (what the next launch sequence computes for a problem).
enum Mode : int32_t { M_IDLE = 0, M_F = 1, M_W = 2, M_OUTER = 3 };
// Solver phases.
enum Phase : int32_t { PH_INIT = 0, PH_ALG1 = 1, PH_OUTER = 2, PH_INNER = 3, PH_DONE = 4 };
// Where the scalar step after an evaluation runs (see the GPE_STEP_* values).
// STEP_FUSED: every workgroup of the next evaluation's first pass runs it on
// its own (the same bits in each), before forming its trial point.
enum StepAt : int32_t { STEP_LAST_GROUP = 0, STEP_KERNEL = 1, STEP_FUSED = 2 };

// Internal status: mixed-precision Algorithm 1 stalled at the FP32 floor; the
// host continues in FP64.
constexpr int kStatusStalled = 2;

// Stop rules (the GPE_STOP_* values).
enum StopRule : int32_t { STOP_RESID = 0, STOP_CRIT1 = 1, STOP_CRIT2 = 2 };

// Source of the point an M_OUTER evaluation starts from.
enum OuterSrc : int32_t { SRC_XK = 0, SRC_XK_PLUS_S = 1, SRC_XF = 2 };

// Boundary treatment of a problem (the GPE_BC_* values).
enum Bc : int32_t { BC_FOURIER = 0, BC_SINE = 1, BC_FD = 2 };

// Per-problem description used on the device (read only in kernels).
// Fourier: n[a] periodic points, each line transformed as it is.  Sine:
// n[a] = N-1 interior points of N intervals; each line is transformed as its
// odd extension of nl[a] = 2N points (zero at 0 and N, mirrored with a sign
// change above N), which turns the Fourier multiplier into the sine
// operator's.  Finite differences: n[a] = N-1 interior points held at line
// positions 1..N-1 of a line of nl[a] = N points whose position 0 is the
// boundary value 0 (the other boundary value sits past the line's end).
struct ProbDev {
  int32_t dim;
  int32_t n[3];          // array points per axis
  int32_t nl[3];         // line length per axis: n (Fourier), 2(n+1) (sine), n+1 (finite differences)
  int32_t bc;            // Bc
  int64_t stride[3];     // element stride of each axis: 1, nx, nx*ny
  int64_t m;             // number of grid points
  int32_t tiles[3];      // tiles (blocks) per pass along axis 0, 1, 2
  int32_t lanes[3];      // lines per tile in each pass
  int32_t has_v;         // 1: read v_arr, 0: separable v_axis tables
  int32_t step_at;       // StepAt: where the scalar step runs
  int32_t real;          // 1: drop the imaginary parts of every stored iterate and gradient
  int32_t prec64;        // 1: the problem's arrays and passes are float64 (else the mixed precision's)
  int32_t pair;          // 1: a real grid function, two x-neighbours to a complex element (the solver's
                         // arrays; n[0], strides and m describe that complex view, nl[0] the x lines)
  double lo[3], h[3], len[3];   // len: period of the transformed line (b-a, or 2(b-a) for sine)
  double x0[3];          // coordinate of array index 0 (lo, or lo + h for sine and finite differences)
  double ctr[3];         // centre of the box (lo + hi) / 2: Dirichlet grids take the coordinates of
                         // their points as ctr + (j + 1 - N/2) h, mirror images of each other exactly
  double beta, omega, hvol, sqrt_hvol, alpha;
  const double* v_arr;   // explicit V (float64), or null
  const double* v_axis;  // [3][kMaxN]: V = v_axis[0][x] + v_axis[1][y] + v_axis[2][z]
  // solver arrays (element type depends on precision, see api)
  void* xf[2];           // Algorithm 1 on F: iterate X (ping-pong)
  void* gf[2];           // ... and its gradient
  void* s[2];            // Newton subproblem: S = X - X_k (ping-pong)
  void* d[2];            // ... and grad_W - G_k
  void* xk;              // outer iterate X_k (complex double)
  void* gk;              // G_k = grad F(X_k) (complex double)
  void* t;               // accumulator of the directional passes (complex double sized)
  double* part1;         // [S1_COUNT][tiles[0]] (slot-major)
  double* part1x;        // second first-pass buffer (STEP_FUSED: evaluations alternate)
  double* partF;         // [SF_COUNT][tiles[dim-1]] (slot-major)
  int32_t* ticket;       // workgroups of the final pass done (reset by the last one)
  const void* user_in;   // apply / init input
  void* user_out;        // apply output
};

// Coordinate of array index j on axis i in the potential tables.  On a
// Dirichlet grid (N = n + 1 intervals) the points j and N - 2 - j are mirror
// images about the box centre, and this form makes their coordinates exact
// negatives relative to it, so a mirror-symmetric trap gives a mirror-symmetric
// table to the last bit; periodic grids take lo + j h.
inline __host__ __device__ double grid_coord(const ProbDev& d, int i, int j) {
  if (d.bc == BC_FOURIER) return d.x0[i] + d.h[i] * j;
  return d.ctr[i] + d.h[i] * (double)(j + 1 - (d.n[i] + 1) / 2);
}

// Per-problem solver state, written only by the step kernel.
struct SolverState {
  int32_t mode, phase, status, cur;       // cur: ping-pong index of xf/gf or s/d
  int32_t src, force_norm, alg, done;
  int32_t k, m, maxit, outer;
  int32_t nfe, nfe64, inner_total, backtracks;
  int32_t rejections, max_outer, nfe_f, nfe_w;
  int32_t nfe_o, stop_rule, switch_window, since_best;   // since_best: steps without halving best_r
  // trial coefficients of the retraction, Y = p X_b + q g_b (pm1 = p - 1)
  double p, q, pm1, t;
  // scalars of the current base point
  double f_b, a_b, n_b, ng_b;
  double np2_b;                            // ||P_b||^2 of the base (first trial)
  double n_hat;                            // c^2 ||Y_pre||^2 used in W0 (set by final pass rule)
  double C, Q, tau_bb, tau_last;
  double delta, forcing, f_outer, r_outer;
  double pred_acc, ared_acc;               // model and actual reduction of the accepted inner iterate
  double ss, sw, ww;                       // BB products of the last accepted step
  // options copy
  double tol, tau0, rho1, eta, sigma, renorm_tol;
  double eta1, eta2, gshrink, ggrow, delta_min, delta_max;
  double eps0, crit2_tol;                  // thresholds of the step-length stop rules
  double best_r;                           // best residual of Algorithm 1 (stall test)
  double switch_r;                         // mixed Algorithm 2: FP64 handover residual
  int32_t k_init, k_sub, m_max, max_iter;
  int32_t pending;                         // STEP_FUSED: partial sums of an evaluation await their step
  int32_t pad5;                            // whole 16-byte words (read with 16-byte loads)
};
static_assert(sizeof(SolverState) % 16 == 0, "SolverState is read in 16-byte words");

// LDS elements (complex) a tile of `lanes` lines of n points needs for its
// line data (must match LdsMap in the device code).
inline int lds_elems_host(int n, int lanes, bool strided) {
  return strided ? n * (lanes + 1) : lanes * (n + n / 16);
}

// Parameters of the analytic trap + lattice tables (computed on the device
// by the no-allocation entry point).
struct VAxisParams {
  double gamma[3], amp, k;
};

// Largest grid of gpe_apply_h_noalloc and the bytes of its fixed scratch:
// descriptor, potential tables, scalars and chunk totals, last-pass partial
// sums (at most one per 64 transform points plus one per tile), residual
// partials (at most 2048 blocks x 6 slots) and the pass accumulator (complex
// float64), each piece 256-byte aligned.
constexpr int64_t kNoAllocMaxPoints = (int64_t)1 << 21;
constexpr size_t kNoAllocAlign(size_t b) { return (b + 255) & ~(size_t)255; }
constexpr size_t kNoAllocDesc = 1024;
constexpr size_t kNoAllocVaxis = kNoAllocAlign(3 * 1024 * sizeof(double));
constexpr size_t kNoAllocOut = kNoAllocAlign(64 * sizeof(double));
constexpr size_t kNoAllocPart = kNoAllocAlign((size_t)(kNoAllocMaxPoints / 16 + 8192) * 3 * sizeof(double));
constexpr size_t kNoAllocRpart = kNoAllocAlign(2048 * 6 * sizeof(double));
constexpr size_t kNoAllocT = kNoAllocAlign((size_t)kNoAllocMaxPoints * 16);
constexpr size_t kNoAllocBytes = kNoAllocDesc + kNoAllocVaxis + kNoAllocOut + kNoAllocPart + kNoAllocRpart + kNoAllocT;
static_assert(sizeof(ProbDev) <= kNoAllocDesc, "the descriptor fits its scratch slot");

// Arguments of the stand-alone apply passes.
// kind 0: H(phi) phi in phi units; kind 1: Hessian-vector product in X units.
struct ApplyArgs {
  int32_t kind;
  double delta;            // Hessian-vector: regularisation delta
  const void* in;          // phi (kind 0) or s (kind 1)
  const void* xk;          // kind 1: X_k (complex double)
  void* out;
};

}  // namespace gpe
