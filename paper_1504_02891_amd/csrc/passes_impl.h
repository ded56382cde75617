// Directional spectral passes of one function+gradient evaluation of the
// ground-state solver.  One evaluation of a d-dimensional problem is d
// launches: FIRST (x-lines, contiguous), MID (y-lines, 3D only), FINAL (last
// axis, strided).  A 1D problem is one SOLO launch.  Every pass loads the
// trial point, transforms each line, multiplies by the axis multiplier
// (lambda^2/2 + rotation term, §2.3) and transforms back; the final pass adds
// the other axes' results, V and the nonlinearity, and reduces the scalars
// the step kernel needs.
#pragma once
#include <type_traits>
#include "gpe_device.h"

namespace gpe {

__device__ __forceinline__ int role_axis(int role, int dim) {
  return role == R_FIRST || role == R_SOLO ? 0 : (role == R_MID ? 1 : dim - 1);
}
__device__ __forceinline__ int64_t pass_cols(const ProbDev& P, int ax) { return P.m / P.n[ax]; }
__device__ __forceinline__ int64_t col_base(const ProbDev& P, int ax, int64_t col) {
  if (ax == 0) return col * P.n[0];
  if (ax == 1) {
    const int64_t x = col % P.n[0], z = col / P.n[0];
    return z * P.stride[2] + x;
  }
  return col;
}
// Omega * (coordinate entering the first-derivative multiplier of this axis)
__device__ __forceinline__ double rot_coef(const ProbDev& P, int ax, int64_t col) {
  if (P.dim < 2 || P.omega == 0.0) return 0.0;
  if (ax == 0) return P.omega * (P.lo[1] + P.h[1] * (double)(col % P.n[1]));   // + Omega y
  if (ax == 1) return -P.omega * (P.lo[0] + P.h[0] * (double)(col % P.n[0]));  // - Omega x
  return 0.0;
}
template <typename CT>
__device__ __forceinline__ CT axis_mult(int k, int n, CT two_pi_over_len, CT rc, CT inv_n) {
  const int p = k < (n >> 1) ? k : k - n;
  const CT lam = two_pi_over_len * (CT)p;
  return ((CT)0.5 * lam * lam + rc * lam) * inv_n;
}
__device__ __forceinline__ double potential_at(const ProbDev& P, int64_t g) {
  if (P.has_v) return P.v_arr[g];
  const int64_t ix = g % P.n[0];
  double v = P.v_axis[ix];
  if (P.dim > 1) v += P.v_axis[kMaxN + (g / P.n[0]) % P.n[1]];
  if (P.dim > 2) v += P.v_axis[2 * kMaxN + g / P.stride[2]];
  return v;
}

// Thread layout of a tile: `lanes` lines of N points, TL threads per line.
template <int N>
struct Tile {
  static constexpr int E = Plan<N>::E, TL = N / E;
  int lanes, lane, t;
  int64_t col;
  bool act;
  int64_t base, st;
  LdsMap mp;
  __device__ __forceinline__ Tile(const ProbDev& P, int ax, bool strided, int tile) {
    lanes = blockDim.x / TL;
    if (strided) { lane = threadIdx.x % lanes; t = threadIdx.x / lanes; }
    else { lane = threadIdx.x / TL; t = threadIdx.x % TL; }
    col = (int64_t)tile * lanes + lane;
    act = col < pass_cols(P, ax);
    base = act ? col_base(P, ax, col) : 0;
    st = P.stride[ax];
    mp.lanes = lanes;
    mp.strided = strided;
  }
  __device__ __forceinline__ int64_t g(int e) const { return base + (int64_t)(t + e * TL) * st; }
};

// Forward transform, multiplier, inverse transform of the tile's lines.
template <int N, typename CT>
__device__ __forceinline__ void spectral_apply(const ProbDev& P, int ax, const Tile<N>& T, cx<CT>* v,
                                               cx<CT>* lds, const cx<CT>* tw) {
  line_fft<N, false>(v, T.t, T.lane, T.mp, lds, tw);
  const CT rc = (CT)rot_coef(P, ax, T.col);
  const CT tpl = (CT)(6.283185307179586477 / P.len[ax]);
  const CT inv_n = (CT)1 / (CT)N;
#pragma unroll
  for (int e = 0; e < Tile<N>::E; ++e) {
    const CT mlt = axis_mult<CT>(T.t + e * Tile<N>::TL, N, tpl, rc, inv_n);
    v[e] = mlt * v[e];
  }
  line_fft<N, true>(v, T.t, T.lane, T.mp, lds, tw);
}

// Deterministic sum (or max) of part[i*stride + slot] over i < count, done by
// the block's first wavefront (lane l takes i = l, l+64, ...; then a
// butterfly).  The final pass and the step kernel both use it, so the
// renormalisation factor they derive from the first-pass sums agrees bitwise.
__device__ __forceinline__ double fixed_reduce(const double* part, int count, int stride, int slot,
                                               bool is_max, double* red) {
  if (threadIdx.x < 64) {
    double s = 0.0;
    for (int i = threadIdx.x; i < count; i += 64) {
      const double v = part[(int64_t)i * stride + slot];
      s = is_max ? fmax(s, v) : s + v;
    }
    s = is_max ? wave_max(s) : wave_sum(s);
    if (threadIdx.x == 0) red[0] = s;
  }
  __syncthreads();
  const double r = red[0];
  __syncthreads();
  return r;
}
__device__ __forceinline__ double sum_part1(const ProbDev& P, int slot, double* red) {
  return fixed_reduce(P.part1, P.tiles[0], S1_COUNT, slot, false, red);
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
template <typename T> __device__ __forceinline__ cx<double> rnd(cx<double> a) {  // round through storage type
  return cvt<double>(cvt<T>(a));
}

// ---------------------------------------------------------------------------
// Per-mode load (trial point) and epilogue.
// ---------------------------------------------------------------------------
struct Acc1 { double ny = 0.0, np2 = 0.0, rmax = 0.0; };
struct AccF { double s[SF_COUNT_SUM] = {}; double smax = 0.0; };

// Algorithm 1 on F: Y = p X_b + q G_b.
template <typename TF>
struct FOps {
  const ProbDev& P; const SolverState& S;
  const void *xb, *gb; void *xo, *go;
  __device__ FOps(const ProbDev& P_, const SolverState& S_) : P(P_), S(S_) {
    xb = P.xf[S.cur]; gb = P.gf[S.cur]; xo = P.xf[S.cur ^ 1]; go = P.gf[S.cur ^ 1];
  }
  __device__ __forceinline__ cx<double> trial(int64_t g) const {
    const cx<double> x = cvt<double>(ld<TF>(xb, g)), gr = cvt<double>(ld<TF>(gb, g));
    return S.p * x + S.q * gr;
  }
  __device__ __forceinline__ cx<double> load_first(int64_t g, Acc1& a) const {
    const cx<double> x = cvt<double>(ld<TF>(xb, g)), gr = cvt<double>(ld<TF>(gb, g));
    const cx<double> pb = S.n_b * gr - S.a_b * x;
    a.np2 += abs2(pb);
    a.rmax = fmax(a.rmax, sqrt(abs2(gr - (S.a_b / S.n_b) * x)));
    const cx<double> y = S.p * x + S.q * gr;
    a.ny += abs2(y);
    return y;
  }
  // kin: kinetic(+rotation) part of H_lin applied to the unscaled trial
  __device__ __forceinline__ void final_(int64_t g, cx<double> kin, double c, double n_hat, AccF& a) const {
    const cx<double> x = cvt<double>(ld<TF>(xb, g)), gr = cvt<double>(ld<TF>(gb, g));
    const cx<double> y0 = S.p * x + S.q * gr;
    const cx<TF> ys = cvt<TF>(c * y0);
    const cx<double> y = cvt<double>(ys);
    const double q = abs2(y);
    const cx<double> ay = 2.0 * (c * kin + potential_at(P, g) * y);
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
  const ProbDev& P; const SolverState& S;
  const cx<double>*xk, *gk; const void *sb, *db; void *so, *dout;
  __device__ WOps(const ProbDev& P_, const SolverState& S_) : P(P_), S(S_) {
    xk = reinterpret_cast<const cx<double>*>(P.xk);
    gk = reinterpret_cast<const cx<double>*>(P.gk);
    sb = P.s[S.cur]; db = P.d[S.cur]; so = P.s[S.cur ^ 1]; dout = P.d[S.cur ^ 1];
  }
  __device__ __forceinline__ cx<double> trial(int64_t g) const {
    const cx<double> s = cvt<double>(ld<TW>(sb, g)), d = cvt<double>(ld<TW>(db, g));
    return S.pm1 * xk[g] + S.p * s + S.q * (gk[g] + d);
  }
  __device__ __forceinline__ cx<double> load_first(int64_t g, Acc1& a) const {
    const cx<double> x0 = xk[g], g0 = gk[g];
    const cx<double> s = cvt<double>(ld<TW>(sb, g)), d = cvt<double>(ld<TW>(db, g));
    const cx<double> gb = g0 + d, xb = x0 + s;
    const cx<double> pb = (S.n_b * g0 - S.a_b * x0) + (S.n_b * d - S.a_b * s);
    a.np2 += abs2(pb);
    a.rmax = fmax(a.rmax, sqrt(abs2(gb - (S.a_b / S.n_b) * xb)));
    const cx<double> sn = S.pm1 * x0 + S.p * s + S.q * gb;
    a.ny += abs2(x0 + sn);
    return sn;
  }
  __device__ __forceinline__ void final_(int64_t g, cx<double> kin, double c, double n_hat, AccF& a) const {
    const cx<double> x0 = xk[g], g0 = gk[g];
    const cx<double> s = cvt<double>(ld<TW>(sb, g)), d = cvt<double>(ld<TW>(db, g));
    const cx<double> sn = S.pm1 * x0 + S.p * s + S.q * (g0 + d);
    const double vg = potential_at(P, g);
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
  const ProbDev& P; const SolverState& S;
  cx<double>*xk, *gk;
  __device__ OOps(const ProbDev& P_, const SolverState& S_) : P(P_), S(S_) {
    xk = reinterpret_cast<cx<double>*>(P.xk);
    gk = reinterpret_cast<cx<double>*>(P.gk);
  }
  __device__ __forceinline__ cx<double> trial(int64_t g) const {
    if (S.src == SRC_XF) return cvt<double>(ld<TF>(P.xf[S.cur], g));
    if (S.src == SRC_XK_PLUS_S) return xk[g] + cvt<double>(ld<TW>(P.s[S.cur], g));
    return xk[g];
  }
  __device__ __forceinline__ cx<double> load_first(int64_t g, Acc1& a) const {
    const cx<double> y = trial(g);
    a.ny += abs2(y);
    return y;
  }
  __device__ __forceinline__ void final_(int64_t g, cx<double> kin, double c, double, AccF& a) const {
    const cx<double> y = c * trial(g);
    const double q = abs2(y);
    const cx<double> ay = 2.0 * (c * kin + potential_at(P, g) * y);
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
__device__ __forceinline__ void solver_tile(const ProbDev& P, const SolverState& S, int tile,
                                            const Ops& ops, cx<CT>* lds, const cx<CT>* tw, double* red) {
  constexpr int E = Tile<N>::E;
  const int ax = role_axis(ROLE, P.dim);
  const Tile<N> T(P, ax, ROLE == R_MID || ROLE == R_FINAL, tile);
  cx<CT> v[E];
  Acc1 a1;
  // The trial point is formed element by element (a rolled loop keeps few
  // loads in flight per thread) and staged through the thread's own LDS
  // slots, then taken into registers for the transform.
#pragma unroll 1
  for (int e = 0; e < E; ++e) {
    cx<CT> val{0, 0};
    if (T.act) {
      if constexpr (ROLE == R_FIRST || ROLE == R_SOLO) val = cvt<CT>(ops.load_first(T.g(e), a1));
      else val = cvt<CT>(ops.trial(T.g(e)));
    }
    lds[T.mp.idx(T.lane, T.t + e * T.TL, N)] = val;
  }
#pragma unroll
  for (int e = 0; e < E; ++e) v[e] = lds[T.mp.idx(T.lane, T.t + e * T.TL, N)];
  double c = 1.0, n_hat = 1.0;
  if constexpr (ROLE == R_SOLO) {
    double acc[3] = {a1.ny, a1.np2, a1.rmax};
    block_reduce<2, 1>(acc, red);
    __shared__ double bc[3];
    if (threadIdx.x == 0) {
      bc[0] = acc[0]; bc[1] = acc[1]; bc[2] = acc[2];
      P.part1[S1_NY] = acc[0]; P.part1[S1_NP2] = acc[1]; P.part1[S1_RMAX] = acc[2];
    }
    __syncthreads();
    c = renorm_c(S, bc[0]);
    n_hat = c * c * bc[0];
  } else if constexpr (ROLE == R_FINAL) {
    const double ny = sum_part1(P, S1_NY, red);
    c = renorm_c(S, ny);
    n_hat = c * c * ny;
  }
  spectral_apply<N, CT>(P, ax, T, v, lds, tw);
  cx<CT>* tacc = reinterpret_cast<cx<CT>*>(P.t);
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
      for (int e = 0; e < E; ++e) {
        const int64_t g = T.g(e);
        tacc[g] = tacc[g] + v[e];
      }
  } else {
    AccF af;
    __syncthreads();  // every thread has finished reading LDS in the inverse transform
#pragma unroll
    for (int e = 0; e < E; ++e) lds[T.mp.idx(T.lane, T.t + e * T.TL, N)] = v[e];
    if (T.act)
#pragma unroll 1
      for (int e = 0; e < E; ++e) {
        const int64_t g = T.g(e);
        cx<double> kin = cvt<double>(lds[T.mp.idx(T.lane, T.t + e * T.TL, N)]);
        if constexpr (ROLE == R_FINAL) kin = kin + cvt<double>(tacc[g]);
        ops.final_(g, kin, c, n_hat, af);
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

// Dispatch on the problem's mode.  PREC64: every array float64.
template <int N, int ROLE, bool PREC64>
__device__ __forceinline__ void solver_dispatch(const ProbDev& P, const SolverState& S, int tile,
                                                char* smem, const cx<double>* twd, const cx<float>* twf,
                                                double* red) {
  using TS = typename std::conditional<PREC64, double, float>::type;   // F/W storage
  using CT = TS;                                                         // F/W transforms
  if (S.mode == M_F) {
    FOps<TS> ops(P, S);
    solver_tile<N, ROLE, CT>(P, S, tile, ops, reinterpret_cast<cx<CT>*>(smem),
                             PREC64 ? reinterpret_cast<const cx<CT>*>(twd) : reinterpret_cast<const cx<CT>*>(twf), red);
  } else if (S.mode == M_W) {
    WOps<TS> ops(P, S);
    solver_tile<N, ROLE, CT>(P, S, tile, ops, reinterpret_cast<cx<CT>*>(smem),
                             PREC64 ? reinterpret_cast<const cx<CT>*>(twd) : reinterpret_cast<const cx<CT>*>(twf), red);
  } else if (S.mode == M_OUTER) {
    OOps<TS, TS> ops(P, S);
    solver_tile<N, ROLE, double>(P, S, tile, ops, reinterpret_cast<cx<double>*>(smem), twd, red);
  }
}

template <int ROLE, bool PREC64>
__global__ void __launch_bounds__(256) k_solver_pass(const ProbDev* __restrict__ probs,
                                                     const SolverState* __restrict__ states,
                                                     const int2* __restrict__ bmap,
                                                     const cx<double>* __restrict__ twd,
                                                     const cx<float>* __restrict__ twf) {
  extern __shared__ __align__(16) char smem[];
  __shared__ double red[SF_COUNT * 16];
  const int2 bm = bmap[blockIdx.x];
  const ProbDev& P = probs[bm.x];
  const SolverState& S = states[bm.x];
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
}

}  // namespace gpe
