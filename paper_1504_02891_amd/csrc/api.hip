// C ABI of the ground-state library: context, workspace, validation, launch
// geometry and the host loop that replays chunks of solver evaluations.
#include <hip/hip_runtime.h>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/gpe.h"
#include "gpe_launch.h"

using namespace gpe;

namespace {

thread_local std::string g_last_error;

#define HIPCHK(expr)                                                              \
  do {                                                                            \
    hipError_t e_ = (expr);                                                       \
    if (e_ != hipSuccess) {                                                       \
      g_last_error = std::string(#expr) + ": " + hipGetErrorString(e_);           \
      return GPE_EDEVICE;                                                         \
    }                                                                             \
  } while (0)

#define CHK(expr)                 \
  do {                            \
    int r_ = (expr);              \
    if (r_ < 0) return r_;        \
  } while (0)

constexpr int kSolverThreads = 128;   // threads per workgroup of every solver pass
constexpr int kApplyThreads = 128;
constexpr int64_t kRereadTiles = 1024;  // final-pass tiles from which its epilogue re-reads (256 CUs x 4)
// STEP_FUSED is tried by the autotuner only up to this many first-pass tiles
// (every one of them reduces all partial sums of the previous evaluation)
constexpr int64_t kFusedMaxTiles = 512;

// Workspace slots owned by a context (grown on demand, freed at destroy).
enum WsSlot {
  WS_PROB = 0, WS_STATE, WS_BMAP, WS_VAXIS, WS_ARENA,
  WS_APPLY_T, WS_APPLY_PART, WS_APPLY_OUT, WS_APPLY_RPART, WS_APPLY_PROB, WS_APPLY_VAXIS,
  WS_SCRATCH_OUT, WS_RETRACT, WS_PROLONG0, WS_PROLONG1, WS_LEVEL0, WS_IMAG, WS_TUNE, WS_COUNT
};

}  // namespace

// A tuned launch configuration (gpe_autotune) for one grid and precision.
struct TunedPlan {
  int dim, bc, n[3], prec;
  int threads[3], elems[3], step_at;
};

struct gpe_ctx {
  int device = 0;
  std::vector<TunedPlan> plans;
  hipStream_t user = nullptr;
  hipStream_t s = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr, t0 = nullptr, t1 = nullptr;
  void* twd = nullptr;
  void* twf = nullptr;
  void* ws[WS_COUNT] = {};
  size_t ws_size[WS_COUNT] = {};
  void* pinned = nullptr;       // host staging for uploads / small downloads
  size_t pinned_size = 0;
  bool staged = false;          // an upload from the staging buffer may still be pending
  std::vector<unsigned char> apply_key;   // descriptor + V tables last uploaded for apply calls
};

namespace {

int ws_get(gpe_ctx* c, int slot, size_t bytes, void** out) {
  if (bytes == 0) bytes = 256;
  if (c->ws_size[slot] < bytes) {
    if (c->ws[slot]) {
      HIPCHK(hipStreamSynchronize(c->s));
      HIPCHK(hipFree(c->ws[slot]));
      c->ws[slot] = nullptr;
      c->ws_size[slot] = 0;
    }
    c->apply_key.clear();
    size_t b = bytes + bytes / 8;
    if (hipMalloc(&c->ws[slot], b) != hipSuccess) {
      (void)hipGetLastError();
      g_last_error = "hipMalloc failed for " + std::to_string(b) + " bytes";
      return GPE_ENOMEM;
    }
    c->ws_size[slot] = b;
  }
  *out = c->ws[slot];
  return GPE_OK;
}

int pinned_get(gpe_ctx* c, size_t bytes, void** out) {
  if (c->pinned_size < bytes) {
    if (c->pinned) {
      HIPCHK(hipStreamSynchronize(c->s));
      HIPCHK(hipHostFree(c->pinned));
      c->pinned = nullptr;
    }
    HIPCHK(hipHostMalloc(&c->pinned, bytes + 4096, hipHostMallocDefault));
    c->pinned_size = bytes + 4096;
  }
  *out = c->pinned;
  return GPE_OK;
}

// Stream-ordered upload through the pinned staging buffer.  begin_call has
// waited for any upload of an earlier call, and uploads within one call use
// disjoint staging offsets, so the staging memory is free.
int upload(gpe_ctx* c, void* dst, const void* src, size_t bytes, size_t staging_off) {
  void* pin;
  CHK(pinned_get(c, staging_off + bytes, &pin));
  std::memcpy((char*)pin + staging_off, src, bytes);
  HIPCHK(hipMemcpyAsync(dst, (char*)pin + staging_off, bytes, hipMemcpyHostToDevice, c->s));
  c->staged = true;
  return GPE_OK;
}

// Every entry point starts here: the context stream waits for the caller's
// stream, and the host waits for the context stream only while an upload of
// an earlier call may still read the staging buffer.  A call that uploads
// nothing and reads nothing back (an apply with unchanged problem and no
// scalars) is therefore fully asynchronous.
int begin_call(gpe_ctx* c) {
  HIPCHK(hipSetDevice(c->device));
  if (c->staged) {
    HIPCHK(hipStreamSynchronize(c->s));
    c->staged = false;
  }
  HIPCHK(hipEventRecord(c->ev_in, c->user));
  HIPCHK(hipStreamWaitEvent(c->s, c->ev_in, 0));
  return GPE_OK;
}
int end_call(gpe_ctx* c) {
  HIPCHK(hipEventRecord(c->ev_out, c->s));
  HIPCHK(hipStreamWaitEvent(c->user, c->ev_out, 0));
  return GPE_OK;
}

bool pow2_ok(int n) { return n >= 16 && n <= kMaxN && (n & (n - 1)) == 0; }

// Validate a problem and fill the device descriptor's geometry and scalars
// (array pointers are set by the caller); `vaxis` receives the separable
// potential tables V_i(x_i) = 1/2 gamma_i^2 x_i^2 + A sin^2(k x_i).
int build_prob(const gpe_problem* p, ProbDev* d, double* vaxis) {
  if (!p || !d) return GPE_EINVAL;
  if (p->dim < 1 || p->dim > 3) return GPE_EINVAL;
  if (p->bc != GPE_BC_FOURIER && p->bc != GPE_BC_SINE && p->bc != GPE_BC_FD) return GPE_EINVAL;
  const bool sine = p->bc == GPE_BC_SINE, fd = p->bc == GPE_BC_FD, dirichlet = sine || fd;
  if (!std::isfinite(p->beta) || !std::isfinite(p->omega)) return GPE_EINVAL;
  if ((p->dim == 1 || dirichlet) && p->omega != 0.0) return GPE_EINVAL;
  std::memset(d, 0, sizeof(*d));
  d->dim = p->dim;
  d->bc = sine ? BC_SINE : (fd ? BC_FD : BC_FOURIER);
  d->m = 1;
  double hvol = 1.0;
  for (int i = 0; i < 3; ++i) {
    if (i < p->dim) {
      // sine: n intervals, n-1 interior points, transform of the 2n-point odd
      // extension; finite differences: n-1 interior points on lines of n
      // positions (position 0 the boundary)
      if (!pow2_ok(p->n[i]) || (sine && 2 * p->n[i] > kMaxN)) return GPE_EUNSUPPORTED;
      if (!(p->lo[i] < p->hi[i]) || !std::isfinite(p->lo[i]) || !std::isfinite(p->hi[i])) return GPE_EINVAL;
      const double box = p->hi[i] - p->lo[i];
      d->n[i] = dirichlet ? p->n[i] - 1 : p->n[i];
      d->nl[i] = sine ? 2 * p->n[i] : p->n[i];
      d->lo[i] = p->lo[i];
      d->h[i] = box / p->n[i];
      d->x0[i] = dirichlet ? p->lo[i] + d->h[i] : p->lo[i];
      d->ctr[i] = 0.5 * (p->lo[i] + p->hi[i]);
      d->len[i] = sine ? 2.0 * box : box;
      hvol *= d->h[i];
    } else {
      d->n[i] = 1;
      d->nl[i] = 1;
      d->lo[i] = 0.0;
      d->x0[i] = 0.0;
      d->len[i] = 1.0;
      d->h[i] = 1.0;
    }
  }
  d->stride[0] = 1;
  d->stride[1] = d->n[0];
  d->stride[2] = (int64_t)d->n[0] * d->n[1];
  d->m = (int64_t)d->n[0] * d->n[1] * d->n[2];
  d->beta = p->beta;
  d->omega = p->omega;
  d->hvol = hvol;
  d->sqrt_hvol = std::sqrt(hvol);
  d->alpha = p->beta / (2.0 * hvol);
  d->has_v = p->v != nullptr;
  d->v_arr = p->v;
  if (vaxis) {
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < kMaxN; ++j) {
        double v = 0.0;
        if (i < p->dim && j < d->n[i]) {
          const double x = grid_coord(*d, i, j);
          const double s = std::sin(p->lattice_k * x);
          v = 0.5 * p->gamma[i] * p->gamma[i] * x * x + p->lattice_amp * s * s;
        }
        vaxis[i * kMaxN + j] = v;
      }
  }
  return GPE_OK;
}

struct Geom {
  int threads, lanes, tiles;
  size_t smem;
};

// Tiling of a pass along axis `ax`: transform lines of N = nl[ax] points,
// TL = N/ept threads per line (ept = points per thread, 8 or 4), `threads /
// TL` lines per workgroup.
Geom pass_geom(const ProbDev& d, int ax, bool strided, int threads, size_t elem, int ept = kE) {
  Geom g;
  const int N = d.nl[ax];
  const int TL = N / ept;
  g.threads = threads < TL ? TL : threads;
  g.lanes = g.threads / TL;
  const int64_t cols = (d.pair && ax == 0) ? d.m / d.nl[0] : d.m / d.n[ax];   // pair storage: x lines are row pairs
  g.tiles = (int)((cols + g.lanes - 1) / g.lanes);
  // twiddle table (N entries) + line data
  g.smem = ((size_t)N + (size_t)gpe::lds_elems_host(N, g.lanes, strided)) * elem;
  return g;
}

// Built-in points per thread: 4 while the problems are small enough to be
// bound by the latency of the passes (shorter per-thread chains), else 8.
int default_elems(const std::vector<ProbDev>& pd) {
  int64_t m = 0;
  for (const ProbDev& d : pd) m += d.m;
  return m < ((int64_t)1 << 20) ? 4 : kE;
}

// Built-in workgroup size: one wavefront for 1D (a single line), 256 threads
// once the problem is large enough to be bandwidth bound, else 128.
int default_threads(const std::vector<ProbDev>& pd, int dim) {
  if (dim == 1) return 64;
  int64_t m = 0;
  for (const ProbDev& d : pd) m += d.m;
  return m >= ((int64_t)1 << 20) ? 256 : kSolverThreads;
}

void set_default(gpe_options* o) {
  o->precision = GPE_PREC_FP64;
  o->algorithm = GPE_ALG2;
  o->tol = 1e-6;
  o->k_init = 100;
  o->k_sub = 200;
  o->max_outer = 2000;
  o->max_iter = 20000;
  o->m_max = 20;
  o->tau0 = 1e-3;
  o->rho1 = 1e-4;
  o->eta = 0.85;
  o->sigma = 0.5;
  o->renorm_tol = 1e-14;
  o->eta1 = 0.01;
  o->eta2 = 0.9;
  o->gamma_shrink = 0.5;
  o->gamma_grow = 4.0;
  o->delta0 = 1.0;
  o->delta_min = 1e-12;
  o->delta_max = 1e12;
  o->chunk = 64;
  o->use_graph = 1;
  o->profile = 0;
  o->real_field = -1;
  o->threads[0] = o->threads[1] = o->threads[2] = 0;
  o->elems[0] = o->elems[1] = o->elems[2] = 0;
  o->reserved3 = 0;
  o->step_at = GPE_STEP_AUTO;
  o->stop_rule = GPE_STOP_RESID;
  o->monotone = 0;
  o->eps0 = 1e-6;
  o->crit2_tol = 1e-8;
  o->switch_window = 100;
  o->reserved1 = 0;
  o->switch_resid = 1e-4;
}

// ---------------------------------------------------------------------------
// apply_h / hess_vec
// ---------------------------------------------------------------------------
// Geometry of the stand-alone passes (no allocation): the descriptor's grid
// fields and tiles, each pass's launch shape, the number of last-pass
// partial sums (one per wavefront) and of residual blocks.
struct ApplyShape {
  Geom g[3];
  int nsum, nr;
};
int apply_shape(const gpe_problem* prob, int fp64, ProbDev* d, double* vaxis, ApplyShape* sh) {
  CHK(build_prob(prob, d, vaxis));
  const size_t elem = fp64 ? 16 : 8;
  // wider strided tiles (more columns per row segment) once the grid is large
  const int th = d->m >= ((int64_t)1 << 20) ? 256 : kApplyThreads;
  for (int ax = 0; ax < d->dim; ++ax) {
    sh->g[ax] = pass_geom(*d, ax, ax > 0, th, elem);
    if (d->dim == 1) sh->g[ax] = pass_geom(*d, 0, false, 64, elem);
    d->tiles[ax] = sh->g[ax].tiles;
    d->lanes[ax] = sh->g[ax].lanes;
  }
  const Geom& gl = sh->g[d->dim - 1];
  sh->nsum = gl.tiles * ((gl.threads + 63) / 64);
  sh->nr = (int)std::min<int64_t>((d->m + 255) / 256, fp64 ? 1024 : 2048);   // residual blocks
  return GPE_OK;
}

// Enqueue the passes (and, for H(phi)phi, the residual and scalar kernels)
// with the descriptor `P` already in device memory; `out` receives the ten
// scalars of gpe_apply_h (device), `tot` the chunk totals, `rpart` the
// residual partials.
int enqueue_apply(gpe_ctx* c, const ProbDev& d, const ApplyShape& sh, const ProbDev* P, int fp64,
                  const ApplyArgs& a, double* tot, double* rpart, double* out) {
  const void* tw = fp64 ? c->twd : c->twf;
  const Geom* g = sh.g;
  if (d.dim == 1) {
    launch_apply_pass(c->s, R_SOLO, fp64, g[0].tiles, g[0].threads, g[0].smem, P, a, tw);
  } else {
    launch_apply_pass(c->s, R_FIRST, fp64, g[0].tiles, g[0].threads, g[0].smem, P, a, tw);
    if (d.dim == 3) launch_apply_pass(c->s, R_MID, fp64, g[1].tiles, g[1].threads, g[1].smem, P, a, tw);
    launch_apply_pass(c->s, R_FINAL, fp64, g[d.dim - 1].tiles, g[d.dim - 1].threads, g[d.dim - 1].smem, P, a, tw);
  }
  HIPCHK(hipGetLastError());
  if (a.kind == 0) {
    launch_apply_resid(c->s, sh.nr, P, sh.nsum, a.in, a.out, rpart, tot, fp64);
    launch_apply_finalize(c->s, P, tot, rpart, sh.nr, out);
    HIPCHK(hipGetLastError());
  }
  return GPE_OK;
}

int run_apply(gpe_ctx* c, const gpe_problem* prob, int fp64, const ApplyArgs& a, double* scalars) {
  ProbDev d;
  std::vector<double> vaxis(3 * kMaxN);
  ApplyShape sh;
  CHK(apply_shape(prob, fp64, &d, vaxis.data(), &sh));
  const size_t elem = fp64 ? 16 : 8;
  void *t, *part, *vax, *pd, *rpart, *out;
  CHK(ws_get(c, WS_APPLY_T, (size_t)d.m * elem, &t));
  CHK(ws_get(c, WS_APPLY_PART, (size_t)sh.nsum * SA_COUNT * sizeof(double), &part));
  CHK(ws_get(c, WS_APPLY_VAXIS, vaxis.size() * sizeof(double), &vax));
  CHK(ws_get(c, WS_APPLY_PROB, sizeof(ProbDev), &pd));
  CHK(ws_get(c, WS_APPLY_RPART, (size_t)sh.nr * SR_COUNT * sizeof(double), &rpart));
  CHK(ws_get(c, WS_APPLY_OUT, (16 + SA_COUNT * 16) * sizeof(double), &out));   // scalars, then chunk totals
  d.t = t;
  d.partF = (double*)part;
  d.part1 = (double*)part;
  d.v_axis = (const double*)vax;
  // upload the descriptor and tables only when they differ from the last ones
  // (both workspaces have fixed sizes, so their contents persist)
  const size_t vb = vaxis.size() * sizeof(double);
  std::vector<unsigned char> key(sizeof(d) + vb);
  std::memcpy(key.data(), &d, sizeof(d));
  std::memcpy(key.data() + sizeof(d), vaxis.data(), vb);
  if (key != c->apply_key) {
    c->apply_key.clear();
    CHK(upload(c, vax, vaxis.data(), vb, 0));
    CHK(upload(c, pd, &d, sizeof(d), vb));
    c->apply_key.swap(key);
  }
  CHK(enqueue_apply(c, d, sh, (const ProbDev*)pd, fp64, a, (double*)out + 16, (double*)rpart, (double*)out));
  if (a.kind == 0 && scalars) {
    void* pin;
    CHK(pinned_get(c, 16 * sizeof(double), &pin));
    HIPCHK(hipMemcpyAsync(pin, out, 10 * sizeof(double), hipMemcpyDeviceToHost, c->s));
    HIPCHK(hipStreamSynchronize(c->s));
    std::memcpy(scalars, pin, 10 * sizeof(double));
  }
  return GPE_OK;
}

// ---------------------------------------------------------------------------
// solver
// ---------------------------------------------------------------------------
struct ProbLayout {
  size_t off_xf[2], off_gf[2], off_s[2], off_d[2], off_xk, off_gk, off_t, off_p1, off_p1x, off_pf, off_ticket;
};

void init_state(SolverState& S, const gpe_options& o) {
  std::memset(&S, 0, sizeof(S));
  S.mode = M_F;
  S.phase = PH_INIT;
  S.cur = 0;
  S.force_norm = 1;
  S.alg = o.algorithm;
  S.p = 1.0; S.q = 0.0; S.pm1 = 0.0;
  S.a_b = 0.0; S.n_b = 1.0; S.ng_b = 0.0;
  S.delta = o.delta0;
  S.tol = o.tol; S.tau0 = o.tau0; S.rho1 = o.rho1; S.sigma = o.sigma;
  S.eta = o.monotone ? 0.0 : o.eta;      // monotone Armijo: C = F(X_k)
  S.stop_rule = o.stop_rule; S.eps0 = o.eps0; S.crit2_tol = o.crit2_tol;
  S.switch_window = o.switch_window; S.since_best = 0; S.best_r = INFINITY;
  S.switch_r = o.switch_resid;
  S.renorm_tol = o.renorm_tol;
  S.eta1 = o.eta1; S.eta2 = o.eta2; S.gshrink = o.gamma_shrink; S.ggrow = o.gamma_grow;
  S.delta_min = o.delta_min; S.delta_max = o.delta_max;
  S.k_init = o.k_init; S.k_sub = o.k_sub; S.m_max = o.m_max; S.max_iter = o.max_iter;
  S.max_outer = o.max_outer;
}

int check_options(const gpe_options* o) {
  if (!o) return GPE_EINVAL;
  if (o->precision != GPE_PREC_FP64 && o->precision != GPE_PREC_MIXED) return GPE_EINVAL;
  if (o->algorithm != GPE_ALG1 && o->algorithm != GPE_ALG2) return GPE_EINVAL;
  if (!(o->tol >= 0.0) || o->k_sub < 1 || o->k_init < 0 || o->max_outer < 0 || o->max_iter < 0 || o->m_max < 0)
    return GPE_EINVAL;
  if (!(o->sigma > 0.0 && o->sigma < 1.0) || !(o->eta >= 0.0 && o->eta < 1.0) || !(o->tau0 > 0.0))
    return GPE_EINVAL;
  if (o->chunk < 1 || o->chunk > 4096) return GPE_EINVAL;
  if (o->step_at < GPE_STEP_AUTO || o->step_at > GPE_STEP_FUSED) return GPE_EINVAL;
  if (o->real_field < -1 || o->real_field > 1) return GPE_EINVAL;
  for (int a = 0; a < 3; ++a)
    if (o->elems[a] != 0 && o->elems[a] != 4 && o->elems[a] != 8) return GPE_EINVAL;
  if (o->stop_rule < GPE_STOP_RESID || o->stop_rule > GPE_STOP_CRIT2) return GPE_EINVAL;
  if (o->monotone != 0 && o->monotone != 1) return GPE_EINVAL;
  if (!(o->eps0 >= 0.0) || !(o->crit2_tol >= 0.0) || o->switch_window < 0 ||
      !(o->switch_resid >= 0.0)) return GPE_EINVAL;
  return GPE_OK;
}

// Upper bound on the evaluations the device state machine can take before
// its own caps end every problem (a host-side guard only).
int64_t eval_cap(const gpe_options& o) {
  const int64_t per = o.m_max + 2;
  if (o.algorithm == GPE_ALG1) return (int64_t)(o.max_iter + 2) * per + 16;
  return (int64_t)(o.k_init + 2) * per + (int64_t)(o.max_outer + 2) * ((int64_t)o.k_sub * per + 4) + 16;
}

// The context's tuned plan for a grid and precision, or null.
const TunedPlan* find_plan(const gpe_ctx* c, const gpe_problem& p, int prec) {
  for (const TunedPlan& t : c->plans) {
    bool same = t.dim == p.dim && t.bc == p.bc && t.prec == prec;
    for (int a = 0; a < p.dim && same; ++a) same = t.n[a] == p.n[a];
    if (same) return &t;
  }
  return nullptr;
}

// Keep plan `tp` for the grid of `p` (and tp.prec), replacing an earlier one.
void keep_plan(gpe_ctx* c, const gpe_problem& p, const TunedPlan& tp) {
  for (TunedPlan& t : c->plans)
    if (find_plan(c, p, tp.prec) == &t) { t = tp; return; }
  c->plans.push_back(tp);
}

// The launch plan (workgroup size and points per thread of each pass, step
// placement) a solve of `probs` in precision `prec` uses, where the options
// leave it open: a batch whose problems all share one tuned plan takes it
// whole; otherwise the sizes of the largest problem with a plan (a batch's
// slowest problems are usually its largest) when they suit every problem's
// lines.  `thr`, `ept` in/out (the options' values, 0 = open); `step_at` out
// (the plan's placement, or the options').
void pick_plan(const gpe_ctx* c, int count, const gpe_problem* probs, int prec, const gpe_options& o, int* thr,
               int* ept, int* step_at) {
  for (int a = 0; a < 3; ++a) {
    thr[a] = o.threads[a];
    ept[a] = o.elems[a];
  }
  *step_at = o.step_at;
  const TunedPlan* tp = find_plan(c, probs[0], prec);
  bool all = tp != nullptr;
  for (int i = 1; i < count && all; ++i) all = find_plan(c, probs[i], prec) == tp;
  if (!all) {
    tp = nullptr;
    int64_t best = -1;
    for (int i = 0; i < count; ++i) {
      const TunedPlan* t = find_plan(c, probs[i], prec);
      int64_t m = 1;
      for (int a = 0; a < probs[i].dim; ++a) m *= probs[i].n[a];
      if (t && m > best) { best = m; tp = t; }
    }
    for (int i = 0; i < count && tp; ++i)
      for (int a = 0; a < probs[i].dim; ++a) {
        const int tl = (probs[i].bc == GPE_BC_SINE ? 2 * probs[i].n[a] : probs[i].n[a]) / tp->elems[a];
        if (tl < 1 || tp->threads[a] < tl || tp->threads[a] % tl != 0) tp = nullptr;
        if (!tp) break;
      }
  }
  if (tp && o.threads[0] == 0 && o.threads[1] == 0 && o.threads[2] == 0 && o.elems[0] == 0 && o.elems[1] == 0 &&
      o.elems[2] == 0)
    for (int a = 0; a < 3; ++a) {
      thr[a] = tp->threads[a];
      ept[a] = tp->elems[a];
    }
  if (tp && all && o.step_at == GPE_STEP_AUTO) *step_at = tp->step_at;
}

// Trigonometric prolongation (Algorithm 3) of the complex128 grid function
// `src` of problem `dc` to the grid with every n doubled, axis by axis (the
// intermediate shapes in the context's prolongation buffers), into `dst`.
int enqueue_prolong(gpe_ctx* c, const ProbDev& dc, const void* src, void* dst) {
  int n[3] = {dc.n[0], dc.n[1], dc.n[2]};
  for (int ax = 0; ax < dc.dim; ++ax) {
    void* out = dst;
    if (ax < dc.dim - 1) {
      int nn[3] = {n[0], n[1], n[2]};
      nn[ax] *= 2;
      CHK(ws_get(c, ax == 0 ? WS_PROLONG0 : WS_PROLONG1, (size_t)nn[0] * nn[1] * nn[2] * 16, &out));
    }
    if (launch_prolong_axis(c->s, src, out, n[0], n[1], n[2], ax, c->twd) != 0) return GPE_EUNSUPPORTED;
    HIPCHK(hipGetLastError());
    n[ax] *= 2;
    src = out;
  }
  return GPE_OK;
}

// One precision's share of a solve: the launch shape of its passes and the
// block maps of its unfinished problems.  A mixed-precision solve has an
// FP32 group, from which problems move to the FP64 group when they hand over
// (reading: Algorithm 1 at the FP32 floor, Algorithm 2 below switch_resid);
// the groups run side by side, every evaluation launching each non-empty
// group's passes, so a problem's FP64 continuation starts at the host check
// after its hand-over whatever the other problems do.
struct Group {
  int prec64 = 1;
  int level = 0;                 // cascade level (grid of the coarse problem doubled `level` times)
  int pair = 0;                  // pair storage (real problems on Fourier grids, two or three dimensions)
  int thr[3] = {0, 0, 0}, ept[3] = {kE, kE, kE};
  size_t smem[3] = {0, 0, 0};
  std::vector<ProbDev> pd;       // each problem's descriptor in this precision
  std::vector<int2> bm[3];
  void* dbm[3] = {nullptr, nullptr, nullptr};
};

// Solve `count` problems (one launch sequence for all): Algorithm 1 or 2 in
// the options' precision; in mixed precision each problem that hands over
// continues in FP64 from its iterate (written to its phi buffer and read
// back as an FP64 initial point, the regularisation delta kept, the rest of
// its step or Newton-step budget), and its counters add up over both runs.
// With nlevels > 1 the solve is Algorithm 3 over grids that double per
// level: a problem that ends a coarse level (at level_tol) is prolonged and
// starts the next level at the following host check while the others go on
// with theirs; phi0s[i] holds the coarse initial data (phis[i] when
// nlevels == 1), phis[i] receives the finest level's result.
int solve_impl(gpe_ctx* c, int count, const gpe_problem* probs, const gpe_options* opts, void* const* phi0s,
               void* const* phis, gpe_result* results, int nlevels = 1, double level_tol = 0.0) {
  if (!c || count < 1 || !probs || !phi0s || !phis || !results || nlevels < 1) return GPE_EINVAL;
  CHK(check_options(opts));
  const gpe_options o = *opts;
  const bool mixed = o.precision == GPE_PREC_MIXED;
  // group index: level-major over precision slots (slot 0: the options'
  // precision; slot 1: the FP64 continuation of a mixed solve) over the
  // storage (0: complex elements; 1: pair storage of a real problem)
  const int np = mixed ? 2 : 1;
  const int ng = np * nlevels * 2;
  const int last_lv = nlevels - 1;
  auto gid = [&](int lv, int ps, int pr) { return (lv * np + ps) * 2 + pr; };
  // every level's problems: the coarse grid doubled per level
  std::vector<gpe_problem> lp((size_t)nlevels * count);
  for (int l = 0; l < nlevels; ++l)
    for (int i = 0; i < count; ++i) {
      gpe_problem q = probs[i];
      for (int a = 0; a < 3; ++a) q.n[a] = a < q.dim ? q.n[a] << l : q.n[a];
      lp[(size_t)l * count + i] = q;
    }
  std::vector<Group> grp(ng);
  for (int l = 0; l < nlevels; ++l)
    for (int ps = 0; ps < np; ++ps)
      for (int pr = 0; pr < 2; ++pr) {
        Group& g = grp[gid(l, ps, pr)];
        g.level = l;
        g.prec64 = (mixed && ps == 0) ? 0 : 1;
        g.pair = pr;
      }
  int plan_step = o.step_at;
  for (int gi = 0; gi < ng; ++gi) {
    int sa;
    pick_plan(c, count, &lp[(size_t)grp[gi].level * count], grp[gi].prec64 ? GPE_PREC_FP64 : GPE_PREC_MIXED, o,
              grp[gi].thr, grp[gi].ept, &sa);
    if (gi == gid(last_lv, 0, 0)) plan_step = sa;   // the finest level's plan places the step
  }
  std::vector<std::vector<ProbDev>> pdl(nlevels, std::vector<ProbDev>(count));
  std::vector<double> vaxis((size_t)nlevels * count * 3 * kMaxN);
  const int dim = probs[0].dim;
  for (int i = 0; i < count; ++i)
    if (!phis[i] || !phi0s[i]) return GPE_EINVAL;
  for (int l = 0; l < nlevels; ++l)
    for (int i = 0; i < count; ++i) {
      CHK(build_prob(&lp[(size_t)l * count + i], &pdl[l][i], &vaxis[((size_t)l * count + i) * 3 * kMaxN]));
      if (pdl[l][i].dim != dim) return GPE_EINVAL;
    }
  const std::vector<ProbDev>& pd0 = pdl[0];
  const std::vector<ProbDev>& pdf = pdl[last_lv];
  // real arithmetic forced: Omega = 0 required of every problem
  bool no_rotation = true;
  for (int i = 0; i < count; ++i) no_rotation = no_rotation && probs[i].omega == 0.0;
  if (o.real_field == 1 && !no_rotation) return GPE_EINVAL;
  CHK(begin_call(c));
  // per problem: real arithmetic (forced, or automatic at Omega = 0 when its
  // phi0 has a zero imaginary part), and pair storage for real problems on
  // Fourier grids in two or three dimensions, which halves the arrays' bytes
  // and the transform work; each problem's arithmetic depends on its own
  // data only, so a batched problem keeps the bits it has alone
  std::vector<int> realv(count, o.real_field == 1 ? 1 : 0), pairv(count, 0);
  if (o.real_field < 0) {
    std::vector<int> nb(count, 0);
    size_t tot = 0;
    for (int i = 0; i < count; ++i) {
      if (probs[i].omega != 0.0) continue;
      nb[i] = (int)std::min<int64_t>((pd0[i].m + 255) / 256, 256);   // level-0 data
      tot += nb[i];
    }
    if (tot > 0) {
      void *part, *hp;
      CHK(ws_get(c, WS_IMAG, tot * sizeof(double), &part));
      size_t at = 0;
      for (int i = 0; i < count; ++i) {
        if (nb[i] == 0) continue;
        launch_max_imag(c->s, nb[i], phi0s[i], pd0[i].m, (double*)part + at);
        at += nb[i];
      }
      HIPCHK(hipGetLastError());
      CHK(pinned_get(c, tot * sizeof(double), &hp));
      HIPCHK(hipMemcpyAsync(hp, part, tot * sizeof(double), hipMemcpyDeviceToHost, c->s));
      HIPCHK(hipStreamSynchronize(c->s));
      at = 0;
      for (int i = 0; i < count; ++i) {
        if (nb[i] == 0) continue;
        double mx = 0.0;
        for (int k = 0; k < nb[i]; ++k) mx = std::max(mx, ((const double*)hp)[at + k]);
        realv[i] = mx == 0.0 ? 1 : 0;
        at += nb[i];
      }
    }
  }
  for (int i = 0; i < count; ++i) pairv[i] = realv[i] && dim >= 2 && probs[i].bc == GPE_BC_FOURIER ? 1 : 0;

  // geometry of each pass for each problem and group: points per thread
  // (8, or 4 for latency-bound problems by default) and workgroup size
  // (a group's descriptors are those of its members: the problems whose
  // storage matches it; the others' are left empty)
  auto member = [&](const Group& g, int i) { return pairv[i] == g.pair; };
  for (Group& g : grp) {
    g.pd = pdl[g.level];
    std::vector<ProbDev> pdg;
    for (int i = 0; i < count; ++i) {
      ProbDev& d = g.pd[i];
      if (!member(g, i)) continue;
      if (g.pair) {   // the complex view of the pair storage
        d.pair = 1;
        d.n[0] /= 2;
        d.stride[1] = d.n[0];
        d.stride[2] = (int64_t)d.n[0] * d.n[1];
        d.m /= 2;
      }
      pdg.push_back(d);
    }
    if (pdg.empty()) continue;
    for (int ax = 0; ax < 3; ++ax) {
      if (g.ept[ax] == 0) g.ept[ax] = default_elems(pdg);
      const int th = g.thr[ax];
      if (th != 0 && (th < 64 || th > 256 || th % 64 != 0)) return GPE_EINVAL;   // whole wavefronts
      for (size_t k = 0; k < pdg.size() && ax < dim; ++k) {
        const int tl = pdg[k].nl[ax] / g.ept[ax];
        if (tl > 256 || (th != 0 && th % tl != 0)) return GPE_EINVAL;
      }
    }
    for (int ax = 0; ax < dim; ++ax) {
      int thr_ax = 0;
      for (int i = 0; i < count; ++i) {
        if (!member(g, i)) continue;
        const int th = g.thr[ax] ? g.thr[ax] : default_threads(pdg, dim);
        Geom ge = pass_geom(g.pd[i], ax, ax > 0, th, 16, g.ept[ax]);
        g.pd[i].tiles[ax] = ge.tiles;
        g.pd[i].lanes[ax] = ge.lanes;
        g.smem[ax] = std::max(g.smem[ax], ge.smem);
        if (thr_ax == 0) thr_ax = ge.threads;
        else if (ge.threads != thr_ax) return GPE_EUNSUPPORTED;   // one workgroup size per pass
      }
      g.thr[ax] = thr_ax;
    }
  }
  // placement of the scalar step: in the last workgroup of the final pass
  // while that pass is small (a 1D problem is one workgroup, no fence needed),
  // else a launch of its own (a device-scope fence per workgroup costs more
  // than a launch once there are many workgroups)
  int step_at = plan_step;
  if (step_at < 0) {
    int maxt = 0;
    for (int i = 0; i < count; ++i) maxt = std::max(maxt, grp[gid(last_lv, 0, pairv[i])].pd[i].tiles[dim - 1]);
    step_at = (dim == 1 || maxt <= 128) ? STEP_LAST_GROUP : STEP_KERNEL;
  }
  // a 1D problem is one pass of one workgroup: its step ends that pass
  if (dim == 1) step_at = STEP_LAST_GROUP;
  const bool fused = step_at == STEP_FUSED;
  for (Group& g : grp)
    for (int i = 0; i < count; ++i) {
      g.pd[i].step_at = step_at;
      g.pd[i].prec64 = g.prec64;
    }
  // cascade: each problem's prolonged initial data of its next level (the
  // finest grid's size), and room for the prolongation's intermediate axes
  void* lvbuf = nullptr;
  size_t lv_stride = 0;
  if (nlevels > 1) {
    for (int i = 0; i < count; ++i) lv_stride = std::max<size_t>(lv_stride, (size_t)pdf[i].m * 16);
    void *t0, *t1;
    CHK(ws_get(c, WS_PROLONG0, lv_stride, &t0));
    CHK(ws_get(c, WS_PROLONG1, lv_stride, &t1));
    CHK(ws_get(c, WS_LEVEL0, lv_stride * count, &lvbuf));
  }
  auto level_buf = [&](int i) { return (void*)((char*)lvbuf + (size_t)i * lv_stride); };
  // STEP_FUSED alternates two state arrays and two first-pass partials
  // buffers by evaluation parity; an even chunk leaves the latest state in
  // the first array at every host check
  const int chunk = fused ? (o.chunk + 1) & ~1 : o.chunk;
  // arena: every problem's arrays in every group's precision
  std::vector<ProbLayout> lay((size_t)ng * count);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t r = off;
    off += (bytes + 255) & ~(size_t)255;
    return r;
  };
  for (int gi = 0; gi < ng; ++gi)
    for (int i = 0; i < count; ++i) {
      if (!member(grp[gi], i)) continue;
      const ProbDev& d = grp[gi].pd[i];
      const size_t m = (size_t)d.m, es = grp[gi].prec64 ? 16 : 8;   // element size of the F / W arrays
      ProbLayout& L = lay[(size_t)gi * count + i];
      for (int k = 0; k < 2; ++k) {
        L.off_xf[k] = take(m * es);
        L.off_gf[k] = take(m * es);
        L.off_s[k] = take(m * es);
        L.off_d[k] = take(m * es);
      }
      L.off_xk = take(m * 16);
      L.off_gk = take(m * 16);
      L.off_t = take(m * 16);
      L.off_p1 = take((size_t)d.tiles[0] * S1_COUNT * sizeof(double));
      L.off_p1x = take((size_t)d.tiles[0] * S1_COUNT * sizeof(double));
      L.off_pf = take((size_t)std::max(d.tiles[dim - 1], 1) * SF_COUNT * sizeof(double));
      L.off_ticket = take(64);
    }
  void *arena, *dprob, *dstate, *dvax;
  CHK(ws_get(c, WS_ARENA, off, &arena));
  CHK(ws_get(c, WS_PROB, sizeof(ProbDev) * count, &dprob));
  CHK(ws_get(c, WS_STATE, 2 * sizeof(SolverState) * count, &dstate));
  CHK(ws_get(c, WS_VAXIS, vaxis.size() * sizeof(double), &dvax));
  char* A = (char*)arena;
  for (int gi = 0; gi < ng; ++gi)
    for (int i = 0; i < count; ++i) {
      if (!member(grp[gi], i)) continue;
      const ProbLayout& L = lay[(size_t)gi * count + i];
      ProbDev& d = grp[gi].pd[i];
      d.real = grp[gi].pair ? 0 : realv[i];   // pair storage holds both points' values, no imaginary parts
      for (int k = 0; k < 2; ++k) {
        d.xf[k] = A + L.off_xf[k];
        d.gf[k] = A + L.off_gf[k];
        d.s[k] = A + L.off_s[k];
        d.d[k] = A + L.off_d[k];
      }
      d.xk = A + L.off_xk;
      d.gk = A + L.off_gk;
      d.t = A + L.off_t;
      d.part1 = (double*)(A + L.off_p1);
      d.part1x = (double*)(A + L.off_p1x);
      d.partF = (double*)(A + L.off_pf);
      d.ticket = (int32_t*)(A + L.off_ticket);
      d.v_axis = (const double*)dvax + ((size_t)grp[gi].level * count + i) * 3 * kMaxN;
    }
  // every problem starts in group 0 (level 0, the options' precision); the
  // device descriptor array holds each problem's current one
  auto level_opts = [&](int lv) {
    gpe_options ol = o;
    if (lv < last_lv) ol.tol = level_tol;
    return ol;
  };
  std::vector<int> lev(count, 0);
  std::vector<int> gof(count, 0);
  std::vector<ProbDev> cur(count);
  for (int i = 0; i < count; ++i) {
    gof[i] = gid(0, 0, pairv[i]);
    cur[i] = grp[gof[i]].pd[i];
  }
  std::vector<char> done_host(count, 0);
  // block maps of every group: (problem, tile) of its unfinished problems
  auto build_maps = [&]() {
    for (int gi = 0; gi < ng; ++gi)
      for (int ax = 0; ax < dim; ++ax) {
        grp[gi].bm[ax].clear();
        for (int i = 0; i < count; ++i)
          if (gof[i] == gi && !done_host[i])
            for (int t = 0; t < grp[gi].pd[i].tiles[ax]; ++t) grp[gi].bm[ax].push_back(make_int2(i, t));
      }
  };
  build_maps();
  {
    // one buffer, a region per group and pass with room for every problem
    std::vector<size_t> at((size_t)ng * 3, 0);
    size_t tot = 0;
    for (int gi = 0; gi < ng; ++gi)
      for (int ax = 0; ax < dim; ++ax) {
        size_t cap = 0;
        for (int i = 0; i < count; ++i) cap += (size_t)grp[gi].pd[i].tiles[ax];
        at[(size_t)gi * 3 + ax] = tot;
        tot += (cap * sizeof(int2) + 255) / 256 * 256;
      }
    void* bmb;
    CHK(ws_get(c, WS_BMAP, tot, &bmb));
    for (int gi = 0; gi < ng; ++gi)
      for (int ax = 0; ax < dim; ++ax) grp[gi].dbm[ax] = (char*)bmb + at[(size_t)gi * 3 + ax];
  }
  std::vector<SolverState> st(count);
  for (int i = 0; i < count; ++i) init_state(st[i], level_opts(0));
  // uploads (staging offsets keep the pieces apart)
  size_t so = 0;
  CHK(upload(c, dvax, vaxis.data(), vaxis.size() * sizeof(double), so));
  so += vaxis.size() * sizeof(double);
  CHK(upload(c, dprob, cur.data(), sizeof(ProbDev) * count, so));
  so += sizeof(ProbDev) * count;
  CHK(upload(c, dstate, st.data(), sizeof(SolverState) * count, so));
  CHK(upload(c, (SolverState*)dstate + count, st.data(), sizeof(SolverState) * count, so));
  so += sizeof(SolverState) * count;
  for (int gi = 0; gi < ng; ++gi)
    for (int ax = 0; ax < dim; ++ax) {
      const std::vector<int2>& v = grp[gi].bm[ax];
      if (!v.empty()) CHK(upload(c, grp[gi].dbm[ax], v.data(), v.size() * sizeof(int2), so));
      so += v.size() * sizeof(int2);
    }
  const ProbDev* P = (const ProbDev*)dprob;
  SolverState* S = (SolverState*)dstate;
  for (int i = 0; i < count; ++i) launch_init(c->s, P, i, cur[i].m, phi0s[i], grp[gof[i]].prec64);
  HIPCHK(hipGetLastError());

  // profile: an event pair around the last-axis pass of every k-th
  // evaluation (while one group runs): stamped by the dispatch itself with
  // plain launches, event record nodes inside a graph (these also count the
  // event packets' own time, a few microseconds)
  std::vector<hipEvent_t> pev;
  if (o.profile) {
    pev.resize(2 * (size_t)chunk, nullptr);
    for (auto& e : pev) HIPCHK(hipEventCreate(&e));
  }
  int64_t eval_index = 0;   // evaluations enqueued so far (profile sampling)
  auto sampled = [&](int64_t e) { return o.profile > 0 && e % o.profile == 0; };
  hipError_t enq_err = hipSuccess;
  // an event record on the stream, or, while capturing, an event-record node
  // appended to the captured graph after the stream's current frontier
  auto record = [&](hipEvent_t e) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    hipGraph_t cg = nullptr;
    const hipGraphNode_t* deps = nullptr;
    size_t ndeps = 0;
    hipError_t r = hipStreamGetCaptureInfo_v2(c->s, &cs, nullptr, &cg, &deps, &ndeps);
    if (r == hipSuccess && cs == hipStreamCaptureStatusActive) {
      hipGraphNode_t node;
      r = hipGraphAddEventRecordNode(&node, cg, deps, ndeps, e);
      if (r == hipSuccess) r = hipStreamUpdateCaptureDependencies(c->s, &node, 1, hipStreamSetCaptureDependencies);
    } else if (r == hipSuccess) {
      r = hipEventRecord(e, c->s);
    }
    if (r != hipSuccess && enq_err == hipSuccess) enq_err = r;
  };
  bool capturing = false;
  auto enqueue_eval = [&](int k) {
    const bool prof = sampled(eval_index++);
    int busy = 0;
    for (const Group& g : grp) busy += g.bm[dim - 1].empty() ? 0 : 1;
    const bool timed = prof && busy == 1;
    const bool nodes = timed && capturing;                   // event record nodes around the pass
    hipEvent_t e0 = timed && !capturing ? pev[2 * k] : nullptr, e1 = timed && !capturing ? pev[2 * k + 1] : nullptr;
    const int last = dim == 1 ? R_SOLO : R_FINAL;
    // STEP_FUSED: the first pass reads the state of parity `par` and stores
    // the stepped state in the other array, which the later passes read
    const int par = fused ? (k & 1) : 0;
    SolverState* s_in = S + (size_t)par * count;
    SolverState* s_new = fused ? S + (size_t)(par ^ 1) * count : S;
    // block maps are only needed for batches (workgroup b is tile b of a single problem)
    auto bmap = [&](const Group& g, int ax) { return count == 1 ? nullptr : (const int2*)g.dbm[ax]; };
    if (dim > 1) {
      for (const Group& g : grp)
        if (!g.bm[0].empty())
          launch_solver_pass(c->s, R_FIRST, g.prec64, (int)g.bm[0].size(), g.thr[0], g.smem[0], P, s_in, s_new,
                             bmap(g, 0), c->twd, c->twf, par, nullptr, nullptr, 0, fused ? 1 : 0, g.ept[0],
                             g.pair);
      if (dim == 3)
        for (const Group& g : grp)
          if (!g.bm[1].empty())
            launch_solver_pass(c->s, R_MID, g.prec64, (int)g.bm[1].size(), g.thr[1], g.smem[1], P, s_new, s_new,
                               bmap(g, 1), c->twd, c->twf, par, nullptr, nullptr, 0, 0, g.ept[1], g.pair);
    }
    if (nodes) record(pev[2 * k]);
    for (const Group& g : grp) {
      if (g.bm[dim - 1].empty()) continue;
      // final pass: the epilogue re-reads its inputs once the launch has
      // enough tiles to be bandwidth bound (four workgroups per compute unit)
      // and the tiles are two wavefronts or more (measured: 128^3 with
      // 128-thread tiles 68 -> 49 us per launch; a batch of 64-thread tiles
      // 129 -> 146 us), at 8 points per thread only: with 4 the inputs held
      // through the transforms fit the registers of two waves per SIMD
      const int reread = ((int64_t)g.bm[dim - 1].size() >= kRereadTiles && g.thr[dim - 1] >= 128 &&
                          g.ept[dim - 1] == kE) ? 1 : 0;
      launch_solver_pass(c->s, last, g.prec64, (int)g.bm[dim - 1].size(), g.thr[dim - 1], g.smem[dim - 1], P,
                         s_new, s_new, bmap(g, dim - 1), c->twd, c->twf, par, e0, e1, reread, 0, g.ept[dim - 1],
                         g.pair);
    }
    if (nodes) record(pev[2 * k + 1]);
    if (step_at == STEP_KERNEL) launch_step(c->s, count, P, S);
  };
  auto free_events = [&]() {
    for (auto& e : pev)
      if (e) (void)hipEventDestroy(e);
  };
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  auto capture = [&]() -> int {
    if (exec) {
      (void)hipGraphExecDestroy(exec);
      (void)hipGraphDestroy(graph);
      exec = nullptr;
      graph = nullptr;
    }
    HIPCHK(hipStreamBeginCapture(c->s, hipStreamCaptureModeThreadLocal));
    capturing = true;
    for (int k = 0; k < chunk; ++k) enqueue_eval(k);
    capturing = false;
    HIPCHK(hipStreamEndCapture(c->s, &graph));
    if (enq_err != hipSuccess) {
      (void)hipGraphDestroy(graph);
      graph = nullptr;
      g_last_error = std::string("graph capture: ") + hipGetErrorString(enq_err);
      return GPE_EDEVICE;
    }
    HIPCHK(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
    return GPE_OK;
  };
  if (o.use_graph) {
    const int r = capture();
    if (r != GPE_OK) {
      free_events();
      return r;
    }
  }
  // new block maps on the device (after a hand-over, or to drop finished
  // problems' tiles: once a group's unfinished problems hold at most three
  // quarters of its launched last-pass tiles) and a new graph
  auto remap = [&](size_t so2) -> int {
    build_maps();
    for (int gi = 0; gi < ng; ++gi)
      for (int ax = 0; ax < dim; ++ax) {
        const std::vector<int2>& v = grp[gi].bm[ax];
        if (!v.empty()) CHK(upload(c, grp[gi].dbm[ax], v.data(), v.size() * sizeof(int2), so2));
        so2 += (v.size() * sizeof(int2) + 255) / 256 * 256;
      }
    if (o.use_graph) CHK(capture());
    return GPE_OK;
  };
  // counters of each problem's finished runs (an FP32 run that handed over,
  // earlier cascade levels), added to its last run's at the end
  struct Bank {
    int32_t outer = 0, inner = 0, nfe = 0, nfe64 = 0, bt = 0, rej = 0, nf = 0, nw = 0, no = 0, sw = 0;
    int32_t mx[3] = {0, 0, 0};
    bool capped = false;   // a cascade level stopped at its cap
  };
  std::vector<Bank> bank(count);
  auto deposit = [&](int i, const SolverState& s, bool fp32) {
    Bank& b = bank[i];
    b.outer += s.outer; b.inner += s.inner_total; b.nfe += s.nfe; b.nfe64 += s.nfe64;
    b.bt += s.backtracks; b.rej += s.rejections; b.nf += s.nfe_f; b.nw += s.nfe_w; b.no += s.nfe_o;
    if (fp32) { b.mx[0] += s.nfe_f; b.mx[1] += s.nfe_w; b.mx[2] += s.nfe_o; }
  };
  double pass_ms = 0.0;
  int64_t pass_n = 0;
  // host checks: each chunk's states are copied to one of two pinned slots
  // and an event marks the copy.  Without profiling the next chunk is
  // launched before the host reads the states of the one before, so the
  // GPU does not wait for the host: a problem that finished (or handed
  // over, or ended a coarse level) in chunk k only idles through chunk k + 1,
  // and the host's uploads for it follow chunk k + 1 in stream order.  The
  // pinned buffer is sized once for the two slots and every upload a check
  // can make (descriptors, states, block maps), so it never moves meanwhile.
  const bool pipe = o.profile == 0;
  const size_t st_bytes = (sizeof(SolverState) * count + 255) / 256 * 256;
  size_t bm_bytes = 0;
  for (int gi = 0; gi < ng; ++gi)
    for (int ax = 0; ax < dim; ++ax) {
      size_t cap_t = 0;
      for (int i = 0; i < count; ++i) cap_t += (size_t)grp[gi].pd[i].tiles[ax];
      bm_bytes += (cap_t * sizeof(int2) + 255) / 256 * 256;
    }
  const size_t stage_at = 2 * st_bytes;   // uploads of a check start here
  const size_t pin_bytes = stage_at + (size_t)count * ((sizeof(ProbDev) + 255) / 256 * 256 +
                                                       2 * ((sizeof(SolverState) + 255) / 256 * 256)) + bm_bytes;
  void* pinbase;
  CHK(pinned_get(c, pin_bytes, &pinbase));
  hipEvent_t chk_ev[2] = {nullptr, nullptr}, up_ev = nullptr;
  for (auto& e : chk_ev) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  HIPCHK(hipEventCreateWithFlags(&up_ev, hipEventDisableTiming));
  bool up_pending = false;   // a check's uploads may still read the staging area (up_ev marks their end)
  // a problem restarted at a check (hand-over, next level) has its old state
  // in the next check's copy, taken after the chunk launched ahead: skip it
  std::vector<char> stale(count, 0);
  auto slot_ptr = [&](int k) { return (SolverState*)((char*)c->pinned + (size_t)k * st_bytes); };
  const int64_t cap = eval_cap(o) * ng;
  int64_t evals = 0;
  int rc = GPE_OK;
  // GPE_PROGRESS=<seconds>: a line on stderr at host checks at least that
  // far apart (evaluations so far, problems finished), for long solves
  const char* prog_env = std::getenv("GPE_PROGRESS");
  const double prog_every = prog_env ? std::atof(prog_env) : 0.0;
  auto prog_last = std::chrono::steady_clock::now();
  // one chunk of evaluations and the copy of its states to slot k
  auto launch_chunk = [&](int k) -> bool {
    if (exec) {
      if (hipGraphLaunch(exec, c->s) != hipSuccess) return false;
    } else {
      for (int e = 0; e < chunk; ++e) enqueue_eval(e);
      if (enq_err != hipSuccess) return false;
    }
    evals += chunk;
    return hipMemcpyAsync(slot_ptr(k), dstate, sizeof(SolverState) * count, hipMemcpyDeviceToHost, c->s) ==
               hipSuccess &&
           hipEventRecord(chk_ev[k], c->s) == hipSuccess;
  };
  HIPCHK(hipEventRecord(c->t0, c->s));
  int slot = 0;
  if (!launch_chunk(slot)) rc = GPE_EDEVICE;
  std::vector<SolverState> hs;
  for (; rc == GPE_OK;) {
    if (pipe && !launch_chunk(slot ^ 1)) { rc = GPE_EDEVICE; break; }
    if (hipEventSynchronize(chk_ev[slot]) != hipSuccess) { rc = GPE_EDEVICE; break; }
    const int64_t evals_done = pipe ? evals - chunk : evals;   // evaluations up to the chunk read here
    hs.assign(slot_ptr(slot), slot_ptr(slot) + count);
    bool all = true;
    int64_t maxnfe = 0;
    std::vector<int> hand, adv;
    for (int i = 0; i < count; ++i) {
      if (stale[i]) {
        stale[i] = 0;
        all = false;
        continue;
      }
      maxnfe = std::max<int64_t>(maxnfe, hs[i].nfe);
      if (!done_host[i] && hs[i].done) {
        if (hs[i].status == kStatusStalled && mixed && grp[gof[i]].prec64 == 0) hand.push_back(i);
        else if (lev[i] < last_lv && (hs[i].status == GPE_OK || hs[i].status == GPE_NOT_CONVERGED)) adv.push_back(i);
        else done_host[i] = 1;
      }
      all = all && done_host[i];
    }
    if (o.profile) {
      // launches of this chunk during which some problem was still active
      const int64_t act = std::min<int64_t>(chunk, std::max<int64_t>(0, maxnfe - (evals_done - chunk)));
      for (int64_t k = 0; k < act; ++k) {
        if (!sampled(evals_done - chunk + k)) continue;
        float e = 0.0f;
        if (hipEventElapsedTime(&e, pev[2 * k], pev[2 * k + 1]) == hipSuccess) {
          pass_ms += e;
          ++pass_n;
        }
      }
    }
    if (prog_every > 0.0) {
      const auto now = std::chrono::steady_clock::now();
      if (std::chrono::duration<double>(now - prog_last).count() >= prog_every) {
        int fin = 0;
        for (int i = 0; i < count; ++i) fin += done_host[i] ? 1 : 0;
        std::fprintf(stderr, "gpe: %lld evaluations, %d of %d problems finished\n", (long long)evals_done, fin, count);
        std::fflush(stderr);
        prog_last = now;
      }
    }
    if (all) break;
    if (evals_done > cap) { rc = GPE_NOT_CONVERGED; break; }
    size_t so2 = stage_at;   // staging past the two state slots
    if (up_pending && (!hand.empty() || !adv.empty() || count > 1)) {
      // the previous check's uploads have left the staging area
      if (hipEventSynchronize(up_ev) != hipSuccess) { rc = GPE_EDEVICE; break; }
      up_pending = false;
    }
    // a problem's new run: its descriptor in group `to`, a fresh state on
    // both state arrays, and its initial data `phi0` (complex128)
    auto restart = [&](int i, int to, const SolverState& s2, const void* phi0) -> int {
      gof[i] = to;
      stale[i] = pipe ? 1 : 0;
      cur[i] = grp[to].pd[i];
      CHK(upload(c, (ProbDev*)dprob + i, &cur[i], sizeof(ProbDev), so2));
      so2 += (sizeof(ProbDev) + 255) / 256 * 256;
      CHK(upload(c, S + i, &s2, sizeof(SolverState), so2));
      CHK(upload(c, S + count + i, &s2, sizeof(SolverState), so2));
      so2 += (sizeof(SolverState) + 255) / 256 * 256;
      launch_init(c->s, P, i, grp[to].pd[i].m, phi0, grp[to].prec64);
      return GPE_OK;
    };
    // hand-overs: the FP32 iterate goes to the problem's phi buffer, comes
    // back as the initial point of an FP64 run of the same level with the
    // delta it reached and the rest of its budget
    int step_err = GPE_OK;   // an error of this check's uploads or launches ends the loop below
    for (int i : hand) {
      deposit(i, hs[i], true);
      bank[i].sw += std::max(1, hs[i].inner_total);
      launch_write_phi(c->s, P, S, i, grp[gof[i]].pd[i].m, phis[i], 0);
      const gpe_options ol = level_opts(lev[i]);
      gpe_options o2 = ol;
      o2.precision = GPE_PREC_FP64;
      if (o.algorithm == GPE_ALG1) o2.max_iter = std::max(0, ol.max_iter - hs[i].inner_total);
      else o2.max_outer = std::max(0, ol.max_outer - hs[i].outer);
      SolverState s2;
      init_state(s2, o2);
      if (o.algorithm != GPE_ALG1) s2.delta = std::min(std::max(hs[i].delta, o.delta_min), o.delta_max);
      step_err = restart(i, gid(lev[i], 1, pairv[i]), s2, phis[i]);
      if (step_err != GPE_OK) break;
    }
    // cascade (Algorithm 3): a finished coarse level's iterate goes to the
    // phi buffer, is prolonged to the next grid and starts that level's
    // solve in the options' precision with a fresh state
    for (int i : adv) {
      if (step_err != GPE_OK) break;
      deposit(i, hs[i], grp[gof[i]].prec64 == 0);
      if (hs[i].status == GPE_NOT_CONVERGED) bank[i].capped = true;
      launch_write_phi(c->s, P, S, i, grp[gof[i]].pd[i].m, phis[i], grp[gof[i]].prec64);
      step_err = enqueue_prolong(c, pdl[lev[i]][i], phis[i], level_buf(i));
      if (step_err != GPE_OK) break;
      ++lev[i];
      SolverState s2;
      init_state(s2, level_opts(lev[i]));
      step_err = restart(i, gid(lev[i], 0, pairv[i]), s2, level_buf(i));
    }
    if (step_err == GPE_OK && hipGetLastError() != hipSuccess) step_err = GPE_EDEVICE;
    if (step_err != GPE_OK) { rc = step_err; break; }
    bool rebuild = !hand.empty() || !adv.empty();
    for (int gi = 0; gi < ng && !rebuild; ++gi) {
      size_t act = 0;
      for (int i = 0; i < count; ++i)
        if (gof[i] == gi && !done_host[i]) act += (size_t)grp[gi].pd[i].tiles[dim - 1];
      rebuild = count > 1 && act * 4 <= grp[gi].bm[dim - 1].size() * 3;
    }
    if (rebuild) {
      // (the chunk launched ahead may still run from the graph being
      // replaced: let it finish first)
      if (pipe && hipStreamSynchronize(c->s) != hipSuccess) { rc = GPE_EDEVICE; break; }
      const int r = remap(so2);
      if (r != GPE_OK) { rc = r; break; }
    }
    if (rebuild) {   // (every hand-over or level change rebuilds the maps too)
      if (hipEventRecord(up_ev, c->s) != hipSuccess) { rc = GPE_EDEVICE; break; }
      up_pending = true;
    }
    if (pipe) slot ^= 1;
    else if (!launch_chunk(slot)) { rc = GPE_EDEVICE; break; }
  }
  // the chunk launched ahead has finished before the graph goes
  const hipError_t fin_err = hipStreamSynchronize(c->s);
  if (fin_err != hipSuccess && rc >= 0) rc = GPE_EDEVICE;
  if (exec) (void)hipGraphExecDestroy(exec);
  if (graph) (void)hipGraphDestroy(graph);
  free_events();
  for (auto& e : chk_ev)
    if (e) (void)hipEventDestroy(e);
  (void)hipEventDestroy(up_ev);
  if (rc == GPE_EDEVICE) {
    g_last_error = std::string("solver loop: ") + hipGetErrorString(hipGetLastError());
    return rc;
  }
  if (rc < 0) return rc;
  HIPCHK(hipEventRecord(c->t1, c->s));
  // the final states (a chunk launched ahead of the last check may have
  // stepped a problem the evaluation cap stopped)
  HIPCHK(hipMemcpyAsync(slot_ptr(0), dstate, sizeof(SolverState) * count, hipMemcpyDeviceToHost, c->s));
  HIPCHK(hipStreamSynchronize(c->s));
  std::memcpy(st.data(), slot_ptr(0), sizeof(SolverState) * count);
  for (int i = 0; i < count; ++i) {
    launch_write_phi(c->s, P, S, i, grp[gof[i]].pd[i].m, phis[i], grp[gof[i]].prec64);
    // a problem stopped on a coarse level (the solve's evaluation cap, an
    // error) still returns a finest-grid function: its iterate prolonged
    const void* src = phis[i];
    for (int l = lev[i]; l < last_lv; ++l) {
      void* dst = (src == phis[i]) ? level_buf(i) : phis[i];
      CHK(enqueue_prolong(c, pdl[l][i], src, dst));
      src = dst;
    }
    if (src != phis[i]) HIPCHK(hipMemcpyAsync(phis[i], src, (size_t)pdf[i].m * 16, hipMemcpyDeviceToDevice, c->s));
  }
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(c->s));
  float ms = 0.0f;
  HIPCHK(hipEventElapsedTime(&ms, c->t0, c->t1));
  int worst = GPE_OK;
  for (int i = 0; i < count; ++i) {
    gpe_result& r = results[i];
    std::memset(&r, 0, sizeof(r));
    const SolverState& s = st[i];
    const Bank& b = bank[i];
    r.status = s.done ? s.status : GPE_NOT_CONVERGED;
    if (lev[i] < last_lv && r.status == GPE_OK) r.status = GPE_NOT_CONVERGED;   // the cascade did not finish
    if (b.capped && r.status == GPE_OK) r.status = GPE_NOT_CONVERGED;
    // a run still in its FP32 phase at the cap, or stopped there, counts its
    // evaluations as mixed; earlier runs (FP32 before a hand-over, coarse
    // levels) add theirs
    const bool in32 = mixed && grp[gof[i]].prec64 == 0;
    r.outer_iters = s.outer + b.outer;
    r.inner_iters = s.inner_total + b.inner;
    r.nfe = s.nfe + b.nfe;
    r.nfe_fp64 = s.nfe64 + b.nfe64;
    r.backtracks = s.backtracks + b.bt;
    r.rejections = s.rejections + b.rej;
    r.delta = s.delta;
    r.time_ms = ms;
    r.nfe_f = s.nfe_f + b.nf;
    r.nfe_w = s.nfe_w + b.nw;
    r.nfe_outer = s.nfe_o + b.no;
    r.pass_launches = (int32_t)pass_n;
    r.pass_ms = pass_ms;
    r.switch_iter = b.sw;
    r.storage = pairv[i] ? 2 : (realv[i] ? 1 : 0);
    r.nfe_mixed[0] = b.mx[0] + (in32 ? s.nfe_f : 0);
    r.nfe_mixed[1] = b.mx[1] + (in32 ? s.nfe_w : 0);
    r.nfe_mixed[2] = b.mx[2] + (in32 ? s.nfe_o : 0);
    if (r.status == kStatusStalled) r.status = GPE_NOT_CONVERGED;   // stopped before its continuation ran
    if (r.status >= 0) {
      // outputs recomputed in float64 from the returned phi
      double sc[10];
      ApplyArgs a{0, 0.0, phis[i], nullptr, nullptr};
      void* hout;
      CHK(ws_get(c, WS_SCRATCH_OUT, (size_t)pdf[i].m * 16, &hout));
      a.out = hout;
      CHK(run_apply(c, &lp[(size_t)last_lv * count + i], 1, a, sc));
      r.energy = sc[0];
      r.mu = sc[1];
      r.resid = sc[2];
      r.norm_err = sc[3] - 1.0;
      r.rms[0] = sc[4]; r.rms[1] = sc[5]; r.rms[2] = sc[6];
      r.max_dens = sc[7];
      if (!std::isfinite(r.energy) || !std::isfinite(r.resid)) r.status = GPE_ENONFINITE;
    }
    if (r.status < 0 && worst >= 0) worst = r.status;
    else if (r.status == GPE_NOT_CONVERGED && worst == GPE_OK) worst = GPE_NOT_CONVERGED;
  }
  if (rc == GPE_NOT_CONVERGED && worst == GPE_OK) worst = GPE_NOT_CONVERGED;
  CHK(end_call(c));
  return worst;
}

// Statuses a caller may see: GPE_OK, GPE_NOT_CONVERGED or a documented
// negative code.  The internal hand-over status never leaves the library
// (the solver's FP64 continuation replaces it); anything else unexpected reads as not
// converged.
int public_status(int st) {
  if (st == GPE_OK || st == GPE_NOT_CONVERGED) return st;
  if (st <= GPE_EINVAL && st >= GPE_ENONFINITE) return st;
  return GPE_NOT_CONVERGED;
}

int solve_public(gpe_ctx* c, int count, const gpe_problem* probs, const gpe_options* opts, void* const* phis,
                 gpe_result* results) {
  if (!c || count < 1 || !probs || !phis || !results) return GPE_EINVAL;
  const int rc = solve_impl(c, count, probs, opts, phis, phis, results);
  for (int i = 0; i < count; ++i) results[i].status = public_status(results[i].status);
  return public_status(rc);
}

}  // namespace

// ===========================================================================
// exported
// ===========================================================================
extern "C" {

void gpe_options_default(gpe_options* o) {
  if (o) set_default(o);
}

const char* gpe_strerror(int status) {
  switch (status) {
    case GPE_OK: return "ok";
    case GPE_NOT_CONVERGED: return "not converged (iteration cap)";
    case GPE_EINVAL: return "invalid argument";
    case GPE_EUNSUPPORTED: return "unsupported size or combination";
    case GPE_ENOMEM: return "device allocation failed";
    case GPE_EDEVICE: return "HIP runtime error";
    case GPE_ENONFINITE: return "non-finite value";
    default: return "unknown status";
  }
}

const char* gpe_last_error(void) { return g_last_error.c_str(); }

int gpe_ctx_create(gpe_ctx** out, int device, void* stream) {
  if (!out) return GPE_EINVAL;
  *out = nullptr;
  int ndev = 0;
  HIPCHK(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev) return GPE_EINVAL;
  HIPCHK(hipSetDevice(device));
  gpe_ctx* c = new gpe_ctx();
  c->device = device;
  c->user = (hipStream_t)stream;
  int rc = GPE_OK;
  do {
    if (hipStreamCreateWithFlags(&c->s, hipStreamNonBlocking) != hipSuccess) { rc = GPE_EDEVICE; break; }
    if (hipEventCreateWithFlags(&c->ev_in, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_out, hipEventDisableTiming) != hipSuccess ||
        hipEventCreate(&c->t0) != hipSuccess || hipEventCreate(&c->t1) != hipSuccess) { rc = GPE_EDEVICE; break; }
    // twiddle tables exp(-2 pi i m / 1024), float64 and float32
    std::vector<double> twd(2 * kTwN);
    std::vector<float> twf(2 * kTwN);
    for (int m = 0; m < kTwN; ++m) {
      const long double ang = -2.0L * 3.14159265358979323846264338327950288L * (long double)m / (long double)kTwN;
      const double cr = (double)std::cos(ang), ci = (double)std::sin(ang);
      twd[2 * m] = cr; twd[2 * m + 1] = ci;
      twf[2 * m] = (float)cr; twf[2 * m + 1] = (float)ci;
    }
    // the device's copy of the no-allocation scratch (this device is current)
    if (noalloc_init(device) != 0) { rc = GPE_EDEVICE; break; }
    if (hipMalloc(&c->twd, twd.size() * sizeof(double)) != hipSuccess ||
        hipMalloc(&c->twf, twf.size() * sizeof(float)) != hipSuccess) { rc = GPE_ENOMEM; break; }
    if (hipMemcpy(c->twd, twd.data(), twd.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(c->twf, twf.data(), twf.size() * sizeof(float), hipMemcpyHostToDevice) != hipSuccess) {
      rc = GPE_EDEVICE;
      break;
    }
  } while (false);
  if (rc != GPE_OK) {
    g_last_error = std::string("context creation: ") + hipGetErrorString(hipGetLastError());
    gpe_ctx_destroy(c);
    return rc;
  }
  *out = c;
  return GPE_OK;
}

int gpe_ctx_destroy(gpe_ctx* c) {
  if (!c) return GPE_OK;
  (void)hipSetDevice(c->device);
  if (c->s) (void)hipStreamSynchronize(c->s);
  for (int i = 0; i < WS_COUNT; ++i)
    if (c->ws[i]) (void)hipFree(c->ws[i]);
  if (c->twd) (void)hipFree(c->twd);
  if (c->twf) (void)hipFree(c->twf);
  if (c->pinned) (void)hipHostFree(c->pinned);
  if (c->ev_in) (void)hipEventDestroy(c->ev_in);
  if (c->ev_out) (void)hipEventDestroy(c->ev_out);
  if (c->t0) (void)hipEventDestroy(c->t0);
  if (c->t1) (void)hipEventDestroy(c->t1);
  if (c->s) (void)hipStreamDestroy(c->s);
  delete c;
  return GPE_OK;
}

int gpe_apply_h(gpe_ctx* c, const gpe_problem* prob, int32_t precision, const void* phi, void* h_phi,
                double* scalars) {
  if (!c || !prob || !phi || !h_phi || phi == h_phi) return GPE_EINVAL;
  if (precision != GPE_PREC_FP64 && precision != GPE_PREC_MIXED) return GPE_EINVAL;
  CHK(begin_call(c));
  ApplyArgs a{0, 0.0, phi, nullptr, h_phi};
  CHK(run_apply(c, prob, precision == GPE_PREC_FP64, a, scalars));
  return end_call(c);
}

int gpe_apply_h_noalloc(gpe_ctx* c, const gpe_problem* prob, int32_t precision, const void* phi, void* h_phi,
                        double* scalars_dev) {
  if (!c || !prob || !phi || !h_phi || phi == h_phi) return GPE_EINVAL;
  if (precision != GPE_PREC_FP64 && precision != GPE_PREC_MIXED) return GPE_EINVAL;
  const int fp64 = precision == GPE_PREC_FP64;
  ProbDev d;
  ApplyShape sh;
  CHK(apply_shape(prob, fp64, &d, nullptr, &sh));
  // the fixed scratch: descriptor, tables, scalars, partial sums, accumulator
  const size_t part_b = kNoAllocAlign((size_t)sh.nsum * SA_COUNT * sizeof(double));
  const size_t rpart_b = kNoAllocAlign((size_t)sh.nr * SR_COUNT * sizeof(double));
  const size_t t_b = kNoAllocAlign((size_t)d.m * (fp64 ? 16 : 8));
  if (d.m > kNoAllocMaxPoints || part_b > kNoAllocPart || rpart_b > kNoAllocRpart || t_b > kNoAllocT) {
    g_last_error = "gpe_apply_h_noalloc: " + std::to_string(d.m) + " grid points exceed the fixed scratch (at most " +
                   std::to_string(kNoAllocMaxPoints) + ")";
    return GPE_EUNSUPPORTED;
  }
  HIPCHK(hipSetDevice(c->device));
  char* base = noalloc_scratch(c->device);
  if (!base) {
    g_last_error = "gpe_apply_h_noalloc: the device's scratch was not set up";
    return GPE_EDEVICE;
  }
  const size_t o_v = kNoAllocDesc, o_out = o_v + kNoAllocVaxis, o_part = o_out + kNoAllocOut,
               o_rpart = o_part + kNoAllocPart, o_t = o_rpart + kNoAllocRpart;
  d.t = base + o_t;
  d.part1 = d.partF = (double*)(base + o_part);
  d.v_axis = (const double*)(base + o_v);
  VAxisParams vp;
  for (int i = 0; i < 3; ++i) vp.gamma[i] = prob->gamma[i];
  vp.amp = prob->lattice_amp;
  vp.k = prob->lattice_k;
  // stream order as in every entry point (no staging buffer is involved)
  HIPCHK(hipEventRecord(c->ev_in, c->user));
  HIPCHK(hipStreamWaitEvent(c->s, c->ev_in, 0));
  launch_setup_desc(c->s, d, vp, (ProbDev*)base, (double*)(base + o_v));
  HIPCHK(hipGetLastError());
  double* out = (double*)(base + o_out);
  ApplyArgs a{0, 0.0, phi, nullptr, h_phi};
  CHK(enqueue_apply(c, d, sh, (const ProbDev*)base, fp64, a, out + 16, (double*)(base + o_rpart),
                    scalars_dev ? scalars_dev : out));
  return end_call(c);
}

int gpe_hess_vec(gpe_ctx* c, const gpe_problem* prob, int32_t precision, const void* x_k, const void* s,
                 double delta, void* out) {
  if (!c || !prob || !x_k || !s || !out || out == s || out == x_k) return GPE_EINVAL;
  if (precision != GPE_PREC_FP64 && precision != GPE_PREC_MIXED) return GPE_EINVAL;
  CHK(begin_call(c));
  ApplyArgs a{1, delta, s, x_k, out};
  CHK(run_apply(c, prob, precision == GPE_PREC_FP64, a, nullptr));
  return end_call(c);
}

int gpe_retract(gpe_ctx* c, int64_t m, int32_t precision, const void* x, const void* g, double tau, void* y,
                double* coeffs) {
  if (!c || m < 1 || !x || !g || !y || y == x || y == g) return GPE_EINVAL;
  if (precision != GPE_PREC_FP64 && precision != GPE_PREC_MIXED) return GPE_EINVAL;
  CHK(begin_call(c));
  const int nblk = (int)std::min<int64_t>((m + 255) / 256, 1024);
  void* part;
  CHK(ws_get(c, WS_RETRACT, (size_t)nblk * 3 * sizeof(double) + 64, &part));
  double* coef_dev = (double*)part + (size_t)nblk * 3;
  launch_retract(c->s, nblk, x, g, y, m, tau, (double*)part, coef_dev, precision == GPE_PREC_FP64);
  HIPCHK(hipGetLastError());
  if (coeffs) {
    void* pin;
    CHK(pinned_get(c, 64, &pin));
    HIPCHK(hipMemcpyAsync(pin, coef_dev, 5 * sizeof(double), hipMemcpyDeviceToHost, c->s));
    HIPCHK(hipStreamSynchronize(c->s));
    std::memcpy(coeffs, pin, 5 * sizeof(double));
  }
  return end_call(c);
}

int gpe_solve(gpe_ctx* c, const gpe_problem* prob, const gpe_options* opts, void* phi, gpe_result* result) {
  void* phis[1] = {phi};
  return solve_public(c, 1, prob, opts, phis, result);
}

int gpe_solve_batched(gpe_ctx* c, int32_t count, const gpe_problem* probs, const gpe_options* opts,
                      void* const* phis, gpe_result* results) {
  return solve_public(c, count, probs, opts, phis, results);
}

int gpe_set_plan(gpe_ctx* c, const gpe_problem* prob, int32_t precision, const int32_t* threads,
                 const int32_t* elems, int32_t step_at) {
  if (!c || !prob || !threads) return GPE_EINVAL;
  if (precision != GPE_PREC_FP64 && precision != GPE_PREC_MIXED) return GPE_EINVAL;
  if (step_at != GPE_STEP_LAST_GROUP && step_at != GPE_STEP_KERNEL && step_at != GPE_STEP_FUSED) return GPE_EINVAL;
  ProbDev d;
  CHK(build_prob(prob, &d, nullptr));
  TunedPlan tp{};
  for (int a = 0; a < 3; ++a) {
    if (a >= d.dim) continue;
    const int e = elems ? elems[a] : kE;
    if (e != 4 && e != 8) return GPE_EINVAL;
    const int tl = d.nl[a] / e, t = threads[a];
    if ((t != 64 && t != 128 && t != 256) || t < tl || t % tl != 0) return GPE_EINVAL;
    tp.threads[a] = t;
    tp.elems[a] = e;
  }
  tp.step_at = step_at;
  tp.dim = prob->dim;
  tp.bc = prob->bc;
  tp.prec = precision;
  for (int a = 0; a < 3; ++a) tp.n[a] = a < prob->dim ? prob->n[a] : 0;
  keep_plan(c, *prob, tp);
  return GPE_OK;
}

int gpe_autotune(gpe_ctx* c, const gpe_problem* prob, int32_t precision, int32_t* threads_out,
                 int32_t* elems_out, int32_t* step_at_out, double* us_per_eval_out) {
  if (!c || !prob) return GPE_EINVAL;
  if (precision != GPE_PREC_FP64 && precision != GPE_PREC_MIXED) return GPE_EINVAL;
  ProbDev d;
  CHK(build_prob(prob, &d, nullptr));
  // synthetic state on the grid: a Gaussian (with a vortex-like phase when
  // rotating, so that the complex path is timed)
  const size_t m = (size_t)d.m;
  std::vector<double> h(2 * m);
  for (size_t g = 0; g < m; ++g) {
    size_t r = g;
    double q = 0.0, xy[3] = {0.0, 0.0, 0.0};
    for (int a = 0; a < d.dim; ++a) {
      const size_t i = r % (size_t)d.n[a];
      r /= (size_t)d.n[a];
      xy[a] = d.x0[a] + d.h[a] * (double)i;
      q += xy[a] * xy[a];
    }
    const double e = std::exp(-0.5 * q);
    h[2 * g] = e * (1.0 + 0.1 * xy[0]);
    h[2 * g + 1] = d.omega != 0.0 ? e * 0.1 * xy[1] : 0.0;
  }
  void* buf;
  CHK(ws_get(c, WS_TUNE, m * 16, &buf));
  // candidates: points per thread (the same in every pass), workgroup
  // sizes per pass, then the step placement
  auto cands = [&](int ept, std::vector<int>* cand) {
    for (int a = 0; a < 3; ++a) {
      cand[a].clear();
      if (a >= d.dim) { cand[a].push_back(0); continue; }
      const int tl = d.nl[a] / ept;
      for (int t : {64, 128, 256})
        if (t >= tl && t % tl == 0) cand[a].push_back(t);
    }
  };
  gpe_options o;
  set_default(&o);
  o.precision = precision;
  o.algorithm = GPE_ALG2;
  o.k_init = 48;            // about 100 evaluations of each mode, no convergence test
  o.k_sub = 48;
  o.max_outer = 1;
  o.tol = 0.0;
  o.chunk = 32;
  o.switch_window = 0;
  o.switch_resid = 0.0;
  double best = INFINITY;
  TunedPlan bp{};
  std::vector<int> cand[3];
  for (int ept : {kE, 4}) {
    cands(ept, cand);
    for (int a = 0; a < 3; ++a) o.elems[a] = a < d.dim ? ept : 0;
  for (int t0 : cand[0])
    for (int t1 : cand[1])
      for (int t2 : cand[2])
        for (int sa : {GPE_STEP_LAST_GROUP, GPE_STEP_KERNEL, GPE_STEP_FUSED}) {
          if (sa == GPE_STEP_FUSED && (d.dim == 1 || d.m / d.n[0] / (t0 / (d.nl[0] / ept)) > kFusedMaxTiles)) continue;
          if (sa != GPE_STEP_LAST_GROUP && d.dim == 1) continue;     // a 1D solve always steps in its pass
          o.threads[0] = t0; o.threads[1] = t1; o.threads[2] = t2;
          o.step_at = sa;
          double us = INFINITY;
          for (int rep = 0; rep < 2; ++rep) {
            CHK(begin_call(c));
            CHK(upload(c, buf, h.data(), m * 16, 0));
            CHK(end_call(c));
            gpe_result r;
            void* phis[1] = {buf};
            CHK(solve_impl(c, 1, prob, &o, phis, phis, &r));
            if (r.nfe > 0) us = std::min(us, 1e3 * r.time_ms / r.nfe);
          }
          if (us < best) {
            best = us;
            bp.threads[0] = t0; bp.threads[1] = t1; bp.threads[2] = t2;
            for (int a = 0; a < 3; ++a) bp.elems[a] = a < d.dim ? ept : kE;
            bp.step_at = sa;
          }
        }
  }
  bp.dim = prob->dim;
  bp.bc = prob->bc;
  bp.prec = precision;
  for (int a = 0; a < 3; ++a) bp.n[a] = a < prob->dim ? prob->n[a] : 0;
  keep_plan(c, *prob, bp);
  if (threads_out)
    for (int a = 0; a < 3; ++a) threads_out[a] = bp.threads[a];
  if (elems_out)
    for (int a = 0; a < 3; ++a) elems_out[a] = bp.elems[a];
  if (step_at_out) *step_at_out = bp.step_at;
  if (us_per_eval_out) *us_per_eval_out = best;
  return GPE_OK;
}

int gpe_prolong(gpe_ctx* c, const gpe_problem* coarse, const gpe_problem* fine, const void* phi_c, void* phi_f) {
  if (!c || !coarse || !fine || !phi_c || !phi_f || phi_c == phi_f) return GPE_EINVAL;
  ProbDev dc, df;
  CHK(build_prob(coarse, &dc, nullptr));
  CHK(build_prob(fine, &df, nullptr));
  if (dc.dim != df.dim) return GPE_EINVAL;
  if (dc.bc != BC_FOURIER || df.bc != BC_FOURIER) return GPE_EUNSUPPORTED;   // trigonometric prolongation
  for (int i = 0; i < dc.dim; ++i)
    if (df.n[i] != 2 * dc.n[i] || coarse->lo[i] != fine->lo[i] || coarse->hi[i] != fine->hi[i]) return GPE_EINVAL;
  CHK(begin_call(c));
  CHK(enqueue_prolong(c, dc, phi_c, phi_f));
  return end_call(c);
}

int gpe_solve_cascadic(gpe_ctx* c, int32_t count, const gpe_problem* coarse, int32_t nlevels, double level_tol,
                       const gpe_options* opts, void* const* phi0s, void* const* phis, gpe_result* results) {
  if (!c || count < 1 || !coarse || nlevels < 1 || !opts || !phi0s || !phis || !results) return GPE_EINVAL;
  for (int i = 0; i < count; ++i)
    if (coarse[i].bc != GPE_BC_FOURIER) return GPE_EUNSUPPORTED;   // trigonometric prolongation
  const int rc = solve_impl(c, count, coarse, opts, phi0s, phis, results, nlevels, level_tol);
  for (int i = 0; i < count; ++i) results[i].status = public_status(results[i].status);
  return public_status(rc);
}

}  // extern "C"
