// Directional spectral passes of one function+gradient evaluation of the
// ground-state solver.  One evaluation of a d-dimensional problem is d
// launches: FIRST (x-lines, contiguous), MID (y-lines, 3D only), FINAL (last
// axis, strided).  A 1D problem is one SOLO launch.  Every pass loads the
// trial point's inputs once into registers, transforms each line, multiplies
// by the axis multiplier (lambda^2/2 + rotation term, §2.3) and transforms
// back; the final pass adds the other axes' results, V and the nonlinearity
// from the same registers, reduces the scalars of the evaluation, and its
// last workgroup runs the solver's scalar step.
#pragma once
#include <type_traits>
#include "gpe_device.h"
#include "step_impl.h"

namespace gpe {

__device__ __forceinline__ int role_axis(int role, int dim) {
  return role == R_FIRST || role == R_SOLO ? 0 : (role == R_MID ? 1 : dim - 1);
}
__device__ __forceinline__ int64_t pass_cols(const ProbDev& P, int ax) { return P.m / P.n[ax]; }

// Thread layout of a tile: `lanes` lines of N points, TL threads per line.
// The grid coordinates of a line (all but the one along the pass axis) are
// decoded once per tile with 32-bit arithmetic.
template <int N>
struct Tile {
  static constexpr int E = Plan<N>::E, TL = N / E;
  int lanes, lane, t, ax;
  int c[3];          // coordinates of the line's first point
  bool act;
  int64_t base, st;
  double vcol;       // potential of the fixed coordinates (separable V)
  LdsMap mp;
  __device__ __forceinline__ Tile(const ProbDev& P, int ax_, bool strided, int tile) {
    ax = ax_;
    lanes = blockDim.x / TL;
    if (strided) { lane = threadIdx.x % lanes; t = threadIdx.x / lanes; }
    else { lane = threadIdx.x / TL; t = threadIdx.x % TL; }
    const int col = tile * lanes + lane;
    act = col < (int)pass_cols(P, ax);
    const int cc = act ? col : 0;
    const int n0 = P.n[0], n1 = P.n[1];
    if (ax == 0) { c[0] = 0; c[1] = cc % n1; c[2] = cc / n1; }
    else if (ax == 1) { c[0] = cc % n0; c[1] = 0; c[2] = cc / n0; }
    else { c[0] = cc % n0; c[1] = cc / n0; c[2] = 0; }
    base = (int64_t)c[0] + (int64_t)c[1] * P.stride[1] + (int64_t)c[2] * P.stride[2];
    st = P.stride[ax];
    vcol = 0.0;
    if (!P.has_v)
      for (int a = 0; a < P.dim; ++a)
        if (a != ax) vcol += P.v_axis[a * kMaxN + c[a]];
    mp.lanes = lanes;
    mp.strided = strided;
  }
  __device__ __forceinline__ int pos(int e) const { return t + e * TL; }
  __device__ __forceinline__ int64_t g(int e) const { return base + (int64_t)(t + e * TL) * st; }
  __device__ __forceinline__ double pot(const ProbDev& P, int e) const {
    return P.has_v ? P.v_arr[g(e)] : vcol + P.v_axis[ax * kMaxN + pos(e)];
  }
  // Omega * (coordinate entering this axis' first-derivative multiplier)
  __device__ __forceinline__ double rot(const ProbDev& P) const {
    if (P.dim < 2 || P.omega == 0.0) return 0.0;
    if (ax == 0) return P.omega * (P.lo[1] + P.h[1] * (double)c[1]);    // + Omega y
    if (ax == 1) return -P.omega * (P.lo[0] + P.h[0] * (double)c[0]);   // - Omega x
    return 0.0;
  }
};

template <typename CT>
__device__ __forceinline__ CT axis_mult(int k, int n, CT two_pi_over_len, CT rc, CT inv_n) {
  const int p = k < (n >> 1) ? k : k - n;
  const CT lam = two_pi_over_len * (CT)p;
  return ((CT)0.5 * lam * lam + rc * lam) * inv_n;
}

// Forward transform, multiplier, inverse transform of the tile's lines.
// `lds` holds the twiddle table (N entries) followed by the line data.
template <int N, typename CT>
__device__ __forceinline__ void spectral_apply(const ProbDev& P, int ax, const Tile<N>& T, cx<CT>* v,
                                               cx<CT>* lds) {
  const cx<CT>* twl = lds;
  cx<CT>* data = lds + N;
  line_fft<N, false>(v, T.t, T.lane, T.mp, data, twl);
  const CT rc = (CT)T.rot(P);
  const CT tpl = (CT)(6.283185307179586477 / P.len[ax]);
  const CT inv_n = (CT)1 / (CT)N;
#pragma unroll
  for (int e = 0; e < Tile<N>::E; ++e) {
    const CT mlt = axis_mult<CT>(T.t + e * Tile<N>::TL, N, tpl, rc, inv_n);
    v[e] = mlt * v[e];
  }
  line_fft<N, true>(v, T.t, T.lane, T.mp, data, twl);
}

// Deterministic reduction of part[i*stride + s], i < count, for slots
// s < NSLOT (slot s is a max when bit s of `maxmask` is set, else a sum),
// done by the workgroup's first wavefront: lane l takes i = l, l+64, ... in
// order, then a butterfly.  All loads of a lane are independent (one memory
// round trip).  The final pass and the scalar step both use this order, so
// values derived from the same partials agree bitwise.  Every thread gets
// the result.
template <int NSLOT>
__device__ __forceinline__ void reduce_partials(const double* part, int count, int stride, unsigned maxmask,
                                                double* out, double* red) {
  if (threadIdx.x < 64) {
    double acc[NSLOT];
#pragma unroll
    for (int s = 0; s < NSLOT; ++s) acc[s] = 0.0;
    for (int i = threadIdx.x; i < count; i += 64) {
#pragma unroll
      for (int s = 0; s < NSLOT; ++s) {
        const double v = part[(int64_t)i * stride + s];
        acc[s] = ((maxmask >> s) & 1u) ? fmax(acc[s], v) : acc[s] + v;
      }
    }
#pragma unroll
    for (int s = 0; s < NSLOT; ++s) acc[s] = ((maxmask >> s) & 1u) ? wave_max(acc[s]) : wave_sum(acc[s]);
    if (threadIdx.x == 0)
#pragma unroll
      for (int s = 0; s < NSLOT; ++s) red[s] = acc[s];
  }
  __syncthreads();
#pragma unroll
  for (int s = 0; s < NSLOT; ++s) out[s] = red[s];
  __syncthreads();
}
// one slot with the same arithmetic (slots are reduced independently, so
// this equals slot `slot` of the multi-slot call bitwise)
__device__ __forceinline__ double fixed_reduce(const double* part, int count, int stride, int slot,
                                               bool is_max, double* red) {
  if (threadIdx.x < 64) {
    double a = 0.0;
    for (int i = threadIdx.x; i < count; i += 64) {
      const double v = part[(int64_t)i * stride + slot];
      a = is_max ? fmax(a, v) : a + v;
    }
    a = is_max ? wave_max(a) : wave_sum(a);
    if (threadIdx.x == 0) red[0] = a;
  }
  __syncthreads();
  const double r = red[0];
  __syncthreads();
  return r;
}
__device__ __forceinline__ double renorm_c(const SolverState& S, double ny) {
  return (S.force_norm || fabs(ny - 1.0) > S.renorm_tol) ? 1.0 / sqrt(ny) : 1.0;
}

template <typename T> __device__ __forceinline__ cx<T> ld(const void* p, int64_t g) {
  return reinterpret_cast<const cx<T>*>(p)[g];
}
template <typename T> __device__ __forceinline__ void stc(void* p, int64_t g, cx<T> v) {
  reinterpret_cast<cx<T>*>(p)[g] = v;
}

// ---------------------------------------------------------------------------
// Per-mode inputs (kept in registers for the whole pass), trial point and
// epilogue.
// ---------------------------------------------------------------------------
struct Acc1 { double ny = 0.0, np2 = 0.0, rmax = 0.0; };
struct AccF { double s[SF_COUNT_SUM] = {}; double smax = 0.0; };

// Algorithm 1 on F: Y = p X_b + q G_b.
template <typename TF>
struct FOps {
  struct In { cx<TF> x, g; };
  const ProbDev& P; const SolverState& S;
  const void *xb, *gb; void *xo, *go;
  __device__ FOps(const ProbDev& P_, const SolverState& S_) : P(P_), S(S_) {
    xb = P.xf[S.cur]; gb = P.gf[S.cur]; xo = P.xf[S.cur ^ 1]; go = P.gf[S.cur ^ 1];
  }
  __device__ __forceinline__ In load(int64_t g) const { return In{ld<TF>(xb, g), ld<TF>(gb, g)}; }
  __device__ __forceinline__ cx<double> trial(const In& in) const {
    return S.p * cvt<double>(in.x) + S.q * cvt<double>(in.g);
  }
  __device__ __forceinline__ void metrics1(const In& in, cx<double> y, Acc1& a) const {
    const cx<double> x = cvt<double>(in.x), gr = cvt<double>(in.g);
    a.np2 += abs2(S.n_b * gr - S.a_b * x);
    a.rmax = fmax(a.rmax, abs2(gr - (S.a_b / S.n_b) * x));
    a.ny += abs2(y);
  }
  // kin: kinetic(+rotation) part of H_lin applied to the unscaled trial
  __device__ __forceinline__ void final_(const In& in, int64_t g, double vg, cx<double> kin, double c,
                                         double n_hat, AccF& a) const {
    const cx<double> x = cvt<double>(in.x), gr = cvt<double>(in.g);
    const cx<TF> ys = cvt<TF>(c * trial(in));
    const cx<double> y = cvt<double>(ys);
    const double q = abs2(y);
    const cx<double> ay = 2.0 * (c * kin + vg * y);
    const cx<TF> gs = cvt<TF>(ay + (4.0 * P.alpha * q) * y);
    const cx<double> gy = cvt<double>(gs);
    stc<TF>(xo, g, ys);
    stc<TF>(go, g, gs);
    a.s[SF_F] += 0.5 * redot(y, ay) + P.alpha * q * q;
    const cx<double> s = y - x;
    const cx<double> w0 = n_hat * gy - S.n_b * gr - S.a_b * s;
    a.s[SF_A] += redot(y, gy);
    a.s[SF_NG] += abs2(gy);
    a.s[SF_NY] += q;
    a.s[SF_SS] += abs2(s);
    a.s[SF_SY] += redot(s, y);
    a.s[SF_SG] += redot(s, gy);
    a.s[SF_SW0] += redot(s, w0);
    a.s[SF_W0W0] += abs2(w0);
    a.s[SF_W0G] += redot(w0, gy);
    a.s[SF_W0Y] += redot(w0, y);
    a.smax = fmax(a.smax, abs2(s));
  }
};

// Newton subproblem, delta form: X = X_k + S, grad_W = G_k + D,
// S_new = (p-1) X_k + p S_b + q (G_k + D_b).
template <typename TW>
struct WOps {
  struct In { cx<double> xk, gk; cx<TW> s, d; };
  const ProbDev& P; const SolverState& S;
  const cx<double>*xk, *gk; const void *sb, *db; void *so, *dout;
  __device__ WOps(const ProbDev& P_, const SolverState& S_) : P(P_), S(S_) {
    xk = reinterpret_cast<const cx<double>*>(P.xk);
    gk = reinterpret_cast<const cx<double>*>(P.gk);
    sb = P.s[S.cur]; db = P.d[S.cur]; so = P.s[S.cur ^ 1]; dout = P.d[S.cur ^ 1];
  }
  __device__ __forceinline__ In load(int64_t g) const { return In{xk[g], gk[g], ld<TW>(sb, g), ld<TW>(db, g)}; }
  __device__ __forceinline__ cx<double> trial(const In& in) const {
    return S.pm1 * in.xk + S.p * cvt<double>(in.s) + S.q * (in.gk + cvt<double>(in.d));
  }
  __device__ __forceinline__ void metrics1(const In& in, cx<double> sn, Acc1& a) const {
    const cx<double> s = cvt<double>(in.s), d = cvt<double>(in.d);
    const cx<double> gb = in.gk + d, xb = in.xk + s;
    a.np2 += abs2((S.n_b * in.gk - S.a_b * in.xk) + (S.n_b * d - S.a_b * s));
    a.rmax = fmax(a.rmax, abs2(gb - (S.a_b / S.n_b) * xb));
    a.ny += abs2(in.xk + sn);
  }
  __device__ __forceinline__ void final_(const In& in, int64_t g, double vg, cx<double> kin, double c,
                                         double n_hat, AccF& a) const {
    const cx<double> x0 = in.xk, g0 = in.gk;
    const cx<double> s = cvt<double>(in.s), d = cvt<double>(in.d);
    const cx<double> sn = trial(in);
    const double qk = abs2(x0);
    const double al4 = 4.0 * P.alpha;
    const cx<double> axk = g0 - (al4 * qk) * x0;                     // A X_k
    const cx<TW> ss = cvt<TW>(c * sn + (c - 1.0) * x0);               // renormalised S
    const cx<double> sv = cvt<double>(ss);
    const cx<double> as = c * (2.0 * (kin + vg * sn)) + (c - 1.0) * axk;  // A S
    const cx<TW> ds = cvt<TW>(as + al4 * (qk * sv + (2.0 * redot(x0, sv)) * x0) + S.delta * sv);
    const cx<double> dv = cvt<double>(ds);
    stc<TW>(so, g, ss);
    stc<TW>(dout, g, ds);
    const cx<double> y = x0 + sv, gy = g0 + dv;
    const double ny = abs2(y);
    a.s[SF_F] += redot(sv, g0) + 0.5 * redot(sv, dv);
    a.s[SF_A] += redot(y, gy);
    a.s[SF_NG] += abs2(gy);
    a.s[SF_NY] += ny;
    const cx<double> sb_ = sv - s;
    const cx<double> w0 = (n_hat - S.n_b) * g0 + n_hat * dv - S.n_b * d - S.a_b * sb_;
    a.s[SF_SS] += abs2(sb_);
    a.s[SF_SY] += redot(sb_, y);
    a.s[SF_SG] += redot(sb_, gy);
    a.s[SF_SW0] += redot(sb_, w0);
    a.s[SF_W0W0] += abs2(w0);
    a.s[SF_W0G] += redot(w0, gy);
    a.s[SF_W0Y] += redot(w0, y);
    a.s[SF_ARED] += redot(sv, axk) + 0.5 * redot(sv, as)
                    + P.alpha * (2.0 * redot(x0, sv) + abs2(sv)) * (ny + qk);
    a.smax = fmax(a.smax, abs2(sb_));
  }
};

// Float64 evaluation at a new outer iterate; writes X_k, G_k and clears S/D.
template <typename TF, typename TW>
struct OOps {
  struct In { cx<double> y; };
  const ProbDev& P; const SolverState& S;
  cx<double>*xk, *gk;
  __device__ OOps(const ProbDev& P_, const SolverState& S_) : P(P_), S(S_) {
    xk = reinterpret_cast<cx<double>*>(P.xk);
    gk = reinterpret_cast<cx<double>*>(P.gk);
  }
  __device__ __forceinline__ In load(int64_t g) const {
    if (S.src == SRC_XF) return In{cvt<double>(ld<TF>(P.xf[S.cur], g))};
    if (S.src == SRC_XK_PLUS_S) return In{xk[g] + cvt<double>(ld<TW>(P.s[S.cur], g))};
    return In{xk[g]};
  }
  __device__ __forceinline__ cx<double> trial(const In& in) const { return in.y; }
  __device__ __forceinline__ void metrics1(const In&, cx<double> y, Acc1& a) const { a.ny += abs2(y); }
  __device__ __forceinline__ void final_(const In& in, int64_t g, double vg, cx<double> kin, double c, double,
                                         AccF& a) const {
    const cx<double> y = c * in.y;
    const double q = abs2(y);
    const cx<double> ay = 2.0 * (c * kin + vg * y);
    const cx<double> gy = ay + (4.0 * P.alpha * q) * y;
    xk[g] = y;
    gk[g] = gy;
    stc<TW>(P.s[0], g, cx<TW>{0, 0});
    stc<TW>(P.d[0], g, cx<TW>{0, 0});
    a.s[SF_F] += 0.5 * redot(y, ay) + P.alpha * q * q;
    a.s[SF_A] += redot(y, gy);
    a.s[SF_NG] += abs2(gy);
    a.s[SF_NY] += q;
  }
};

// ---------------------------------------------------------------------------
// One tile of one pass for a given mode.
// ---------------------------------------------------------------------------
template <int N, int ROLE, typename CT, class Ops>
__device__ __forceinline__ void solver_tile(const ProbDev& P, const SolverState& S, int tile, const Ops& ops,
                                            cx<CT>* lds, const cx<CT>* tw1024, double* red) {
  constexpr int E = Tile<N>::E;
  constexpr bool HAS_T = (ROLE == R_MID || ROLE == R_FINAL);
  const int ax = role_axis(ROLE, P.dim);
  const Tile<N> T(P, ax, HAS_T, tile);
  load_twiddles<N>(lds, tw1024);
  cx<CT>* tacc = reinterpret_cast<cx<CT>*>(P.t);
  // every input of the thread's elements in one batch of independent loads
  typename Ops::In in[E];
  cx<CT> tv[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    if (T.act) {
      in[e] = ops.load(T.g(e));
      if constexpr (HAS_T) tv[e] = tacc[T.g(e)];
    }
  }
  cx<CT> v[E];
  Acc1 a1;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    cx<double> y{0.0, 0.0};
    if (T.act) {
      y = ops.trial(in[e]);
      if constexpr (ROLE == R_FIRST || ROLE == R_SOLO) ops.metrics1(in[e], y, a1);
    }
    v[e] = cvt<CT>(y);
  }
  double c = 1.0, n_hat = 1.0;
  if constexpr (ROLE == R_SOLO) {
    double acc[3] = {a1.ny, a1.np2, a1.rmax};
    block_reduce<2, 1>(acc, red);
    __shared__ double bc;
    if (threadIdx.x == 0) {
      bc = acc[0];
      P.part1[S1_NY] = acc[0]; P.part1[S1_NP2] = acc[1]; P.part1[S1_RMAX] = acc[2];
    }
    __syncthreads();
    c = renorm_c(S, bc);
    n_hat = c * c * bc;
  } else if constexpr (ROLE == R_FINAL) {
    const double ny = fixed_reduce(P.part1, P.tiles[0], S1_COUNT, S1_NY, false, red);
    c = renorm_c(S, ny);
    n_hat = c * c * ny;
  }
  spectral_apply<N, CT>(P, ax, T, v, lds);
  if constexpr (ROLE == R_FIRST) {
    if (T.act)
#pragma unroll
      for (int e = 0; e < E; ++e) tacc[T.g(e)] = v[e];
    double acc[3] = {a1.ny, a1.np2, a1.rmax};
    block_reduce<2, 1>(acc, red);
    if (threadIdx.x == 0) {
      double* o = P.part1 + (int64_t)tile * S1_COUNT;
      o[S1_NY] = acc[0]; o[S1_NP2] = acc[1]; o[S1_RMAX] = acc[2];
    }
  } else if constexpr (ROLE == R_MID) {
    if (T.act)
#pragma unroll
      for (int e = 0; e < E; ++e) tacc[T.g(e)] = tv[e] + v[e];
  } else {
    AccF af;
    if (T.act)
#pragma unroll
      for (int e = 0; e < E; ++e) {
        cx<double> kin = cvt<double>(v[e]);
        if constexpr (HAS_T) kin = kin + cvt<double>(tv[e]);
        ops.final_(in[e], T.g(e), T.pot(P, e), kin, c, n_hat, af);
      }
    double acc[SF_COUNT];
#pragma unroll
    for (int i = 0; i < SF_COUNT_SUM; ++i) acc[i] = af.s[i];
    acc[SF_SMAX] = af.smax;
    block_reduce<SF_COUNT_SUM, 1>(acc, red);
    if (threadIdx.x == 0) {
      double* o = P.partF + (int64_t)tile * SF_COUNT;
#pragma unroll
      for (int i = 0; i < SF_COUNT; ++i) o[i] = acc[i];
    }
  }
}

// The last workgroup to finish a problem's final pass (ticket counter) runs
// the scalar step of the solver on the reduced partial sums.
__device__ __forceinline__ void step_if_last(const ProbDev& P, SolverState& S, int ntiles, int prec64,
                                             double* red) {
  __shared__ int is_last;
  if (threadIdx.x == 0) {
    int last = 1;
    if (ntiles > 1) {
      __threadfence();                       // publish this workgroup's partials
      last = atomicAdd(P.ticket, 1) == ntiles - 1;
      if (last) {
        __threadfence();                     // see every other workgroup's partials
        atomicExch(P.ticket, 0);
      }
    }
    is_last = last;
  }
  __syncthreads();
  if (!is_last) return;
  double r1[S1_COUNT], rf[SF_COUNT];
  reduce_partials<S1_COUNT>(P.part1, P.tiles[0], S1_COUNT, 1u << S1_RMAX, r1, red);
  reduce_partials<SF_COUNT>(P.partF, ntiles, SF_COUNT, 1u << SF_SMAX, rf, red);
  if (threadIdx.x == 0) step_logic(P, S, r1, rf, prec64);
}

// Dispatch on the problem's mode.  PREC64: every array float64.
template <int N, int ROLE, bool PREC64>
__device__ __forceinline__ void solver_dispatch(const ProbDev& P, SolverState& S, int tile, char* smem,
                                                const cx<double>* twd, const cx<float>* twf, double* red) {
  using TS = typename std::conditional<PREC64, double, float>::type;   // F/W storage and transforms
  const cx<TS>* tws = PREC64 ? reinterpret_cast<const cx<TS>*>(twd) : reinterpret_cast<const cx<TS>*>(twf);
  if (S.mode == M_F) {
    FOps<TS> ops(P, S);
    solver_tile<N, ROLE, TS>(P, S, tile, ops, reinterpret_cast<cx<TS>*>(smem), tws, red);
  } else if (S.mode == M_W) {
    WOps<TS> ops(P, S);
    solver_tile<N, ROLE, TS>(P, S, tile, ops, reinterpret_cast<cx<TS>*>(smem), tws, red);
  } else if (S.mode == M_OUTER) {
    OOps<TS, TS> ops(P, S);
    solver_tile<N, ROLE, double>(P, S, tile, ops, reinterpret_cast<cx<double>*>(smem), twd, red);
  }
}

template <int ROLE, bool PREC64>
__global__ void __launch_bounds__(256) k_solver_pass(const ProbDev* __restrict__ probs,
                                                     SolverState* __restrict__ states,
                                                     const int2* __restrict__ bmap,
                                                     const cx<double>* __restrict__ twd,
                                                     const cx<float>* __restrict__ twf) {
  extern __shared__ __align__(16) char smem[];
  __shared__ double red[SF_COUNT * 16];
  const int2 bm = bmap[blockIdx.x];
  const ProbDev& P = probs[bm.x];
  SolverState& S = states[bm.x];
  if (S.mode == M_IDLE) return;
  const int n = P.n[role_axis(ROLE, P.dim)];
  switch (n) {
    case 16: solver_dispatch<16, ROLE, PREC64>(P, S, bm.y, smem, twd, twf, red); break;
    case 32: solver_dispatch<32, ROLE, PREC64>(P, S, bm.y, smem, twd, twf, red); break;
    case 64: solver_dispatch<64, ROLE, PREC64>(P, S, bm.y, smem, twd, twf, red); break;
    case 128: solver_dispatch<128, ROLE, PREC64>(P, S, bm.y, smem, twd, twf, red); break;
    case 256: solver_dispatch<256, ROLE, PREC64>(P, S, bm.y, smem, twd, twf, red); break;
    case 512: solver_dispatch<512, ROLE, PREC64>(P, S, bm.y, smem, twd, twf, red); break;
    case 1024: solver_dispatch<1024, ROLE, PREC64>(P, S, bm.y, smem, twd, twf, red); break;
    default: break;
  }
  if constexpr (ROLE == R_FINAL || ROLE == R_SOLO)
    if (P.fuse_step) step_if_last(P, S, ROLE == R_SOLO ? 1 : P.tiles[P.dim - 1], PREC64 ? 1 : 0, red);
}

}  // namespace gpe
