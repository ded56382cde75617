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

// Thread layout of a tile: `lanes` lines of N transform points, TL threads
// per line.  The grid coordinates of a line (all but the one along the pass
// axis) are decoded once per tile with 32-bit arithmetic.  Inactive threads
// of a partial last tile address line 0, so that every load is
// unconditional; only their stores are skipped.  For a sine problem,
// transform position p of the odd extension reads array index p-1 (p < N/2)
// or N-1-p (p > N/2) with sign +1 / -1, and is zero at p = 0 and p = N/2;
// only positions 1 .. N/2-1 ("inner") write results and enter reductions.
// For finite differences position p reads array index p-1 and position 0
// holds the boundary value 0; positions 1 .. N-1 are inner.
// `P` is a local copy of the descriptor.
// PAIR (real data, Fourier, Omega = 0, two or three dimensions): the arrays
// hold the real grid function two points to a complex element, (x = 2c,
// x = 2c + 1) at complex column c, and the descriptor describes that complex
// view (n[0] = nx/2 columns, m = M/2 elements; nl[0] = nx is the x lines'
// transform length).  The multipliers are real and even at Omega = 0, so a
// transform of u + i w gives the results for u and w in its real and
// imaginary parts: a strided pass transforms each complex column as the
// pair of real columns 2c, 2c + 1; the x pass takes rows y and y + 1 of one
// z slab as one complex line (tile lines are row pairs; the thread's first
// E/2 elements come from row y, the others from row y + 1).
template <int N, int EPT, bool PAIR = false>
struct Tile {
  static constexpr int E = EPT, TL = N / E;
  using VP = typename std::conditional<PAIR, cx<double>, double>::type;   // V at an element's point(s)
  int lanes, lane, t, ax;
  int c0, c1, c2;    // array coordinates of the line's first point (x, y, z)
  bool act, sine, fd;
  int64_t base, st, base2;   // base2: the second row of a PAIR x line
  double va[3];      // separable V tables at the line's fixed coordinates
  double va0b;       // PAIR strided passes: V_x at the column pair's second point
  LdsMap mp;
  __device__ __forceinline__ Tile(const ProbDev& P, int ax_, bool strided, int tile) {
    ax = ax_;
    sine = P.bc == BC_SINE;
    fd = P.bc == BC_FD;
    lanes = blockDim.x / TL;
    if (strided) { lane = threadIdx.x % lanes; t = threadIdx.x / lanes; }
    else { lane = threadIdx.x / TL; t = threadIdx.x % TL; }
    const int col = tile * lanes + lane;
    const int ncols = (PAIR && ax == 0) ? (int)(P.m / N) : (int)(P.m / pick3(P.n, ax));
    act = col < ncols;
    const int cc = act ? col : 0;
    const int n0 = P.n[0], n1 = P.n[1];
    if (ax == 0) {
      if constexpr (PAIR) { c0 = 0; c1 = 2 * (cc % (n1 >> 1)); c2 = cc / (n1 >> 1); }
      else { c0 = 0; c1 = cc % n1; c2 = cc / n1; }
    } else if (ax == 1) { c0 = cc % n0; c1 = 0; c2 = cc / n0; }
    else { c0 = cc % n0; c1 = cc / n0; c2 = 0; }
    base = (int64_t)c0 + (int64_t)c1 * P.stride[1] + (int64_t)c2 * P.stride[2];
    base2 = base + P.stride[1];
    st = pick3(P.stride, ax);
    // separable V: the tables at the line's fixed coordinates (unconditional
    // loads, in bounds of the [3][kMaxN] table; combined in pot_value)
    va[0] = gld<double>(P.v_axis, PAIR ? 2 * c0 : c0);
    va0b = PAIR ? gld<double>(P.v_axis, 2 * c0 + 1) : 0.0;
    va[1] = gld<double>(P.v_axis, kMaxN + c1);
    va[2] = gld<double>(P.v_axis, 2 * kMaxN + c2);
    mp.lanes = lanes;
    mp.strided = strided;
  }
  __device__ __forceinline__ int pos(int e) const { return t + e * TL; }
  // array index along the axis of transform position pos(e)
  __device__ __forceinline__ int idx(int e) const {
    const int p = pos(e);
    if (fd) return p > 0 ? p - 1 : 0;
    if (!sine) return p;
    const int h = N / 2;
    const int i = p < h ? p - 1 : N - 1 - p;
    return i < 0 ? 0 : (i > h - 2 ? h - 2 : i);
  }
  // sign of the odd extension at pos(e) (0 where it vanishes)
  __device__ __forceinline__ double sgn(int e) const {
    const int p = pos(e);
    if (fd) return p > 0 ? 1.0 : 0.0;
    if (!sine) return 1.0;
    return (p == 0 || p == N / 2) ? 0.0 : (p < N / 2 ? 1.0 : -1.0);
  }
  // pos(e) holds an array point of this line (not a mirror image)
  __device__ __forceinline__ bool inner(int e) const {
    const int p = pos(e);
    return act && (fd ? p > 0 : (!sine || (p > 0 && p < N / 2)));
  }
  __device__ __forceinline__ int64_t g(int e) const {
    if constexpr (PAIR)
      if (ax == 0) return (e < E / 2 ? base : base2) + (int64_t)(t + (e < E / 2 ? e : e - E / 2) * TL);
    return base + (int64_t)idx(e) * st;
  }
  // Potential at the thread's elements in two steps, so that the loads join
  // the tile's batch and the arithmetic waits until the values are used:
  // pot_load fetches the explicit V or this axis' table entries, pot_value
  // adds the other axes' entries.
  // (PAIR: V at both points of the element; an explicit V array is read as
  // its complex view too.  PAIR epilogues are strided passes, ax != 0.)
  __device__ __forceinline__ VP pot_one(const ProbDev& P, int e) const {
    if constexpr (PAIR) {
      if (P.has_v) return gld<cx<double>>(P.v_arr, g(e));
      const double v = gld<double>(P.v_axis, ax * kMaxN + idx(e));
      return cx<double>{v, v};
    } else {
      return P.has_v ? gld<double>(P.v_arr, g(e)) : gld<double>(P.v_axis, ax * kMaxN + idx(e));
    }
  }
  __device__ __forceinline__ void pot_load(const ProbDev& P, VP* vp) const {
#pragma unroll
    for (int e = 0; e < E; ++e) vp[e] = pot_one(P, e);
  }
  __device__ __forceinline__ VP pot_value(const ProbDev& P, VP vpe) const {
    if (P.has_v) return vpe;
    if constexpr (PAIR) {
      double v0 = va[0], v1 = va0b;
      if (ax != 1 && P.dim > 1) { v0 += va[1]; v1 += va[1]; }
      if (ax != 2 && P.dim > 2) { v0 += va[2]; v1 += va[2]; }
      return cx<double>{v0 + vpe.re, v1 + vpe.im};
    } else {
      double vcol = 0.0;
      if (ax != 0) vcol += va[0];
      if (ax != 1 && P.dim > 1) vcol += va[1];
      if (ax != 2 && P.dim > 2) vcol += va[2];
      return vcol + vpe;
    }
  }
  // Omega * (coordinate entering this axis' first-derivative multiplier);
  // rotation is Fourier only
  __device__ __forceinline__ double rot(const ProbDev& P) const {
    if (P.dim < 2 || P.omega == 0.0) return 0.0;
    if (ax == 0) return P.omega * (P.x0[1] + P.h[1] * (double)c1);    // + Omega y
    if (ax == 1) return -P.omega * (P.x0[0] + P.h[0] * (double)c0);   // - Omega x
    return 0.0;
  }
};

template <typename CT>
__device__ __forceinline__ CT axis_mult(int k, int n, CT two_pi_over_len, CT rc, CT inv_n) {
  const int p = k < (n >> 1) ? k : k - n;
  const CT lam = two_pi_over_len * (CT)p;
  return ((CT)0.5 * lam * lam + rc * lam) * inv_n;
}

// Finite differences (§2.1): -1/2 (u_{p+1} - 2 u_p + u_{p-1}) / h^2 along
// the line through the LDS line buffer; u at position 0 is the boundary
// value 0 (the caller's sign factor), the value past position N-1 the other.
template <int N, int E, typename CT, bool PR>
__device__ __forceinline__ void fd_stencil(const ProbDev& P, int ax, const Tile<N, E, PR>& T, cx<CT>* v,
                                           cx<CT>* lds) {
  cx<CT>* data = lds + N;
  __syncthreads();       // nobody still reads the LDS lines
#pragma unroll
  for (int e = 0; e < E; ++e) data[T.mp.idx(T.lane, T.pos(e), N)] = v[e];
  __syncthreads();
  const double h = pick3(P.h, ax);
  const CT c = (CT)(0.5 / (h * h));
  const cx<CT> zero{(CT)0, (CT)0};
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int p = T.pos(e);
    const cx<CT> lft = data[T.mp.idx(T.lane, p > 0 ? p - 1 : 0, N)];
    const cx<CT> rgt = data[T.mp.idx(T.lane, p < N - 1 ? p + 1 : N - 1, N)];
    const cx<CT> l = p > 0 ? lft : zero, r = p < N - 1 ? rgt : zero;
    // the neighbours' sum first: a line that is odd or even about its
    // centre keeps that parity to the last bit
    v[e] = c * ((CT)2 * v[e] - (l + r));
  }
}

// Mirror parity of sine lines about the box centre: interior positions
// p = 1 .. H-1 of the odd extension (H = N/2) mirror to H - p.  The FFT of
// the extension keeps a line's parity only up to rounding, and an excited
// state (§4.4) is a saddle point held by its parity alone, so a line that
// enters the transform exactly odd (or even) leaves it as the odd (even) part
// of the result, which equals the result up to that rounding; other lines are
// left as they are.  sine_parity_in records per line whether the input is
// exactly odd (bit 0) or even (bit 1); sine_parity_out applies it.  Every
// thread of the workgroup must call both (barriers); both use the LDS line
// area, sine_parity_in before the first transform stage (which starts with a
// barrier), sine_parity_out after the last.
__device__ __forceinline__ int* sine_flag_store() {
  __shared__ int f[64];   // lines per tile of a sine pass: at most 256 threads / 4
  return f;
}
template <int N, int E, typename CT, bool PR>
__device__ __forceinline__ void sine_parity_in(const Tile<N, E, PR>& T, const cx<CT>* v, cx<CT>* data) {
  constexpr int H = N / 2;
  int* flags = sine_flag_store();
  __syncthreads();       // nobody still reads the LDS lines
  if (T.t == 0) flags[T.lane] = 3;
#pragma unroll
  for (int e = 0; e < E; ++e) data[T.mp.idx(T.lane, T.pos(e), N)] = v[e];
  __syncthreads();
  int bad = 0;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int p = T.pos(e);
    if (p > 0 && p < H) {
      const cx<CT> q = data[T.mp.idx(T.lane, H - p, N)];
      if (!(v[e].re == -q.re && v[e].im == -q.im)) bad |= 1;
      if (!(v[e].re == q.re && v[e].im == q.im)) bad |= 2;
    }
  }
  if (bad) atomicAnd(&flags[T.lane], ~bad);
}
template <int N, int E, typename CT, bool PR>
__device__ __forceinline__ void sine_parity_out(const Tile<N, E, PR>& T, cx<CT>* v, cx<CT>* data) {
  constexpr int H = N / 2;
  const int* flags = sine_flag_store();
  __syncthreads();       // the last transform stage has read its LDS lines
#pragma unroll
  for (int e = 0; e < E; ++e) data[T.mp.idx(T.lane, T.pos(e), N)] = v[e];
  __syncthreads();
  const int f = flags[T.lane];
  if (f == 0) return;
  const CT half = (CT)0.5;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int p = T.pos(e);
    if (p > 0 && p < H) {
      const cx<CT> q = data[T.mp.idx(T.lane, H - p, N)];
      v[e] = (f & 1) ? half * (v[e] - q) : half * (v[e] + q);
    }
  }
}

// Forward transform and multiplier (spectral_forward), inverse transform
// (spectral_inverse) of the tile's lines; spectral_apply is both.  `lds`
// holds the twiddle table (N entries) followed by the line data.  Finite
// differences apply their stencil in the forward half.
template <int N, int E, typename CT, bool PR>
__device__ __forceinline__ void spectral_forward(const ProbDev& P, int ax, const Tile<N, E, PR>& T, cx<CT>* v,
                                                 cx<CT>* lds) {
  if (T.fd) {
    fd_stencil<N, E, CT>(P, ax, T, v, lds);
    return;
  }
  if (T.sine) sine_parity_in<N, E, CT>(T, v, lds + N);
  line_fft<N, E, false>(v, T.t, T.lane, T.mp, lds + N, lds);
  const CT rc = (CT)T.rot(P);
  const CT tpl = (CT)(6.283185307179586477 / pick3(P.len, ax));
  const CT inv_n = (CT)1 / (CT)N;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const CT mlt = axis_mult<CT>(T.t + e * (N / E), N, tpl, rc, inv_n);
    v[e] = mlt * v[e];
  }
}
template <int N, int E, typename CT, bool PR>
__device__ __forceinline__ void spectral_inverse(const Tile<N, E, PR>& T, cx<CT>* v, cx<CT>* lds) {
  if (!T.fd) line_fft<N, E, true>(v, T.t, T.lane, T.mp, lds + N, lds);
  if (T.sine) sine_parity_out<N, E, CT>(T, v, lds + N);
}
template <int N, int E, typename CT, bool PR>
__device__ __forceinline__ void spectral_apply(const ProbDev& P, int ax, const Tile<N, E, PR>& T, cx<CT>* v,
                                               cx<CT>* lds) {
  spectral_forward<N, E, CT>(P, ax, T, v, lds);
  spectral_inverse<N, E, CT>(T, v, lds);
}

// PAIR x pass: the thread's storage elements (E/2 complex elements q = t +
// j TL of row y, then of row y + 1, each the real points 2q, 2q + 1) to
// transform order (position p: row y's point p as the real part, row y + 1's
// as the imaginary part), through the LDS line area, and back.  Every thread
// of the workgroup must call them (barriers).
template <int N, int E, typename CT>
__device__ __forceinline__ void pair_to_line(const Tile<N, E, true>& T, cx<CT>* v, cx<CT>* data) {
  constexpr int H = E / 2, TL = N / E;
  __syncthreads();       // nobody still reads the LDS lines
#pragma unroll
  for (int j = 0; j < H; ++j) {
    const int q = T.t + j * TL;
    data[T.mp.idx(T.lane, 2 * q, N)] = cx<CT>{v[j].re, v[j + H].re};
    data[T.mp.idx(T.lane, 2 * q + 1, N)] = cx<CT>{v[j].im, v[j + H].im};
  }
  __syncthreads();
#pragma unroll
  for (int e = 0; e < E; ++e) v[e] = data[T.mp.idx(T.lane, T.t + e * TL, N)];
}
template <int N, int E, typename CT>
__device__ __forceinline__ void line_to_pair(const Tile<N, E, true>& T, cx<CT>* v, cx<CT>* data) {
  constexpr int H = E / 2, TL = N / E;
  __syncthreads();       // the last transform stage has read its LDS lines
#pragma unroll
  for (int e = 0; e < E; ++e) data[T.mp.idx(T.lane, T.t + e * TL, N)] = v[e];
  __syncthreads();
#pragma unroll
  for (int j = 0; j < H; ++j) {
    const int q = T.t + j * TL;
    const cx<CT> w0 = data[T.mp.idx(T.lane, 2 * q, N)], w1 = data[T.mp.idx(T.lane, 2 * q + 1, N)];
    v[j] = cx<CT>{w0.re, w1.re};
    v[j + H] = cx<CT>{w0.im, w1.im};
  }
}

// One slot of the fixed-order reduction (the same bits as that slot of the
// multi-slot call), computed by every wavefront of the caller on its own.
__device__ __forceinline__ double wave_reduce_slot(const double* part, int count, int slot, bool is_max) {
  double a[1];
  wave_reduce_partials<1>(part + (int64_t)slot * count, count, is_max ? 1u : 0u, a);
  return a[0];
}
// One slot's partials (count <= 64 B) loaded into registers by a wavefront,
// then summed in the order of wave_reduce_partials (the same bits).
constexpr int kNyLoads = 4;
template <int B>
struct SlotLoads {
  double v[B];
  __device__ __forceinline__ void load(const double* part, int count) {
    const int l = threadIdx.x & 63;
#pragma unroll
    for (int j = 0; j < B; ++j) v[j] = gld<double>(part, min(l + 64 * j, count - 1));
  }
  __device__ __forceinline__ double sum(int count) const {
    const int l = threadIdx.x & 63;
    double a[1] = {0.0};
#pragma unroll
    for (int j = 0; j < B; ++j)
      if (l + 64 * j < count) a[0] += v[j];
    wave_reduce_k<1>(a, 0u);
    return a[0];
  }
};

// Every wavefront reduces all first-pass (S1) slots of `part1` (n1 tiles)
// and final-pass (SF) slots of `partF` (nF tiles) on its own, with every
// load of every slot in one batch (B per lane) when the tiles allow it; each
// slot is summed in the order of wave_reduce_partials (lane l takes tiles l,
// l + 64, ... in turn), so the bits are those of the step kernel's.
template <int B>
__device__ __forceinline__ void wave_reduce_all_b(const double* part1, int n1, const double* partF, int nF,
                                                  double* r1, double* rf) {
  const int l = threadIdx.x & 63;
  double v1[B][S1_COUNT], vf[B][SF_COUNT];
#pragma unroll
  for (int j = 0; j < B; ++j) {
    const int64_t i1 = min(l + 64 * j, n1 - 1), iF = min(l + 64 * j, nF - 1);
#pragma unroll
    for (int s = 0; s < S1_COUNT; ++s) v1[j][s] = gld<double>(part1, (int64_t)s * n1 + i1);
#pragma unroll
    for (int s = 0; s < SF_COUNT; ++s) vf[j][s] = gld<double>(partF, (int64_t)s * nF + iF);
  }
#pragma unroll
  for (int s = 0; s < S1_COUNT; ++s) r1[s] = 0.0;
#pragma unroll
  for (int s = 0; s < SF_COUNT; ++s) rf[s] = 0.0;
#pragma unroll
  for (int j = 0; j < B; ++j) {
    if (l + 64 * j < n1)
#pragma unroll
      for (int s = 0; s < S1_COUNT; ++s) r1[s] = s == S1_RMAX ? fmax(r1[s], v1[j][s]) : r1[s] + v1[j][s];
    if (l + 64 * j < nF)
#pragma unroll
      for (int s = 0; s < SF_COUNT; ++s) rf[s] = s == SF_SMAX ? fmax(rf[s], vf[j][s]) : rf[s] + vf[j][s];
  }
  wave_reduce_k<S1_COUNT>(r1, 1u << S1_RMAX);
  wave_reduce_k<SF_COUNT>(rf, 1u << SF_SMAX);
}
// wave_reduce_all_b's per-lane sums (the same loads and order), combined over
// the lanes by wave_reduce_lds, one lane quad per slot (the same bits); lane
// 4k writes slot k (first-pass slots, then final-pass slots) to out[k].
// `tbuf` holds (S1_COUNT + SF_COUNT) * 65 doubles of LDS.
template <int B>
__device__ __forceinline__ void wave_reduce_all_lds(const double* part1, int n1, const double* partF, int nF,
                                                    double* tbuf, double* out) {
  constexpr int NS = S1_COUNT + SF_COUNT;
  static_assert(4 * NS <= 64, "one lane quad per slot");
  const int l = threadIdx.x & 63;
  double v1[B][S1_COUNT], vf[B][SF_COUNT];
#pragma unroll
  for (int j = 0; j < B; ++j) {
    const int64_t i1 = min(l + 64 * j, n1 - 1), iF = min(l + 64 * j, nF - 1);
#pragma unroll
    for (int s = 0; s < S1_COUNT; ++s) v1[j][s] = gld<double>(part1, (int64_t)s * n1 + i1);
#pragma unroll
    for (int s = 0; s < SF_COUNT; ++s) vf[j][s] = gld<double>(partF, (int64_t)s * nF + iF);
  }
  double acc[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) acc[s] = 0.0;
#pragma unroll
  for (int j = 0; j < B; ++j) {
    if (l + 64 * j < n1)
#pragma unroll
      for (int s = 0; s < S1_COUNT; ++s) acc[s] = s == S1_RMAX ? fmax(acc[s], v1[j][s]) : acc[s] + v1[j][s];
    if (l + 64 * j < nF)
#pragma unroll
      for (int s = 0; s < SF_COUNT; ++s)
        acc[S1_COUNT + s] = s == SF_SMAX ? fmax(acc[S1_COUNT + s], vf[j][s]) : acc[S1_COUNT + s] + vf[j][s];
  }
  const double r = wave_reduce_lds<NS>(acc, (1u << S1_RMAX) | (1u << (S1_COUNT + SF_SMAX)), tbuf);
  if ((l & 3) == 0) out[l >> 2] = r;
}

__device__ __forceinline__ void wave_reduce_all(const double* part1, int n1, const double* partF, int nF,
                                                double* r1, double* rf) {
  const int n = max(n1, nF);
  if (n <= 64) wave_reduce_all_b<1>(part1, n1, partF, nF, r1, rf);
  else if (n <= 128) wave_reduce_all_b<2>(part1, n1, partF, nF, r1, rf);
  else if (n <= 256) wave_reduce_all_b<4>(part1, n1, partF, nF, r1, rf);
  else {
    wave_reduce_partials<S1_COUNT>(part1, n1, 1u << S1_RMAX, r1);
    wave_reduce_partials<SF_COUNT>(partF, nF, 1u << SF_SMAX, rf);
  }
}

// The scalar step's reductions spread over the calling workgroup's
// wavefronts: wavefront w reduces slots w, w + nw, ... of the first-pass (S1)
// and final-pass (SF) partials, each slot in the fixed order of the
// one-wavefront reduction (the same bits), and thread 0 gets r1 and rf
// through `red` (at least S1_COUNT + SF_COUNT doubles).  With `tbuf`
// ((S1_COUNT + SF_COUNT) * 65 doubles of LDS) and at most 256 tiles the one
// wavefront combines its lanes through LDS (the same bits).  Every thread of
// the workgroup must call it (barrier).
__device__ __forceinline__ void step_reductions(const double* part1, int n1, const double* partF, int nF,
                                                double* r1, double* rf, double* red, double* tbuf = nullptr) {
  constexpr int NS = S1_COUNT + SF_COUNT, BS = 32;
  const int nw = blockDim.x >> 6, w = threadIdx.x >> 6;
  // rounds of dependent loads: one wavefront with every slot's loads in
  // flight together (B = 4 per slot), or slot by slot over the wavefronts
  // with BS loads per lane
  const int cnt = max(n1, nF);
  const bool spread = ((NS + nw - 1) / nw) * ((cnt + 64 * BS - 1) / (64 * BS)) < (cnt + 255) / 256;
  if (spread) {
    for (int k = w; k < NS; k += nw) {
      double r[1];
      if (k < S1_COUNT) wave_reduce_partials<1, BS>(part1 + (int64_t)k * n1, n1, k == S1_RMAX ? 1u : 0u, r);
      else wave_reduce_partials<1, BS>(partF + (int64_t)(k - S1_COUNT) * nF, nF, k - S1_COUNT == SF_SMAX ? 1u : 0u, r);
      if ((threadIdx.x & 63) == 0) red[k] = r[0];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
      for (int s = 0; s < S1_COUNT; ++s) r1[s] = red[s];
#pragma unroll
      for (int s = 0; s < SF_COUNT; ++s) rf[s] = red[S1_COUNT + s];
    }
  } else if (tbuf != nullptr && cnt <= 256) {
    if (threadIdx.x < 64) {
      if (cnt <= 64) wave_reduce_all_lds<1>(part1, n1, partF, nF, tbuf, red);
      else if (cnt <= 128) wave_reduce_all_lds<2>(part1, n1, partF, nF, tbuf, red);
      else wave_reduce_all_lds<4>(part1, n1, partF, nF, tbuf, red);
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      if (threadIdx.x == 0) {
#pragma unroll
        for (int s = 0; s < S1_COUNT; ++s) r1[s] = red[s];
#pragma unroll
        for (int s = 0; s < SF_COUNT; ++s) rf[s] = red[S1_COUNT + s];
      }
    }
  } else if (threadIdx.x < 64) {
    wave_reduce_all(part1, n1, partF, nF, r1, rf);   // both slot sets in one batch of loads
  }
}
// Fixed-order reduction for a whole workgroup: the first wavefront reduces,
// every thread gets the result through `red`.
template <int NSLOT>
__device__ __forceinline__ void reduce_partials(const double* part, int count, unsigned maxmask, double* out,
                                                double* red) {
  if (threadIdx.x < 64) {
    wave_reduce_partials<NSLOT>(part, count, maxmask, out);
    if (threadIdx.x == 0)
#pragma unroll
      for (int s = 0; s < NSLOT; ++s) red[s] = out[s];
  }
  __syncthreads();
#pragma unroll
  for (int s = 0; s < NSLOT; ++s) out[s] = red[s];
  __syncthreads();
}
__device__ __forceinline__ double fixed_reduce(const double* part, int count, int slot, bool is_max, double* red) {
  double r[1];
  reduce_partials<1>(part + (int64_t)slot * count, count, is_max ? 1u : 0u, r, red);
  return r[0];
}
__device__ __forceinline__ double renorm_c(const SolverState& S, double ny) {
  return (S.force_norm || fabs(ny - 1.0) > S.renorm_tol) ? 1.0 / sqrt(ny) : 1.0;
}

// real arithmetic: the stored values keep their real parts only
template <typename T> __device__ __forceinline__ cx<T> realify(const ProbDev& P, cx<T> v) {
  return P.real ? cx<T>{v.re, (T)0} : v;
}

template <typename T> __device__ __forceinline__ cx<T> ld(const void* p, int64_t g) { return gld<cx<T>>(p, g); }
template <typename T> __device__ __forceinline__ void stc(void* p, int64_t g, cx<T> v) { gst<cx<T>>(p, g, v); }

// ---------------------------------------------------------------------------
// Per-mode inputs (kept in registers for the whole pass), trial point and
// epilogue.
// ---------------------------------------------------------------------------
struct Acc1 { double ny = 0.0, np2 = 0.0, rmax = 0.0; };
struct AccF { double s[SF_COUNT_SUM] = {}; double smax = 0.0; };

// Point-wise arithmetic of the epilogues.  A complex element is one grid
// point (Pw<false>: its density |v|^2 and products Re(conj(a) b) are
// scalars), or under PAIR two real grid points (Pw<true>: densities and
// products are pairs, one per point).  Sums over the grid (abs2, redot of
// elements) are the same in both.
template <bool PAIR> struct Pw {
  using D = double;
  static __device__ __forceinline__ D dens(cx<double> v) { return abs2(v); }
  static __device__ __forceinline__ D pdot(cx<double> a, cx<double> b) { return redot(a, b); }
  static __device__ __forceinline__ D prod(D a, D b) { return a * b; }
  static __device__ __forceinline__ cx<double> mul(D s, cx<double> v) { return s * v; }
  static __device__ __forceinline__ double sum(D s) { return s; }
  static __device__ __forceinline__ double max2(cx<double> v) { return abs2(v); }   // largest |value|^2
  // al * a * b summed over the element's points (in this order)
  static __device__ __forceinline__ double asum(double al, D a, D b) { return al * a * b; }
};
template <> struct Pw<true> {
  using D = cx<double>;
  static __device__ __forceinline__ D dens(cx<double> v) { return {v.re * v.re, v.im * v.im}; }
  static __device__ __forceinline__ D pdot(cx<double> a, cx<double> b) { return {a.re * b.re, a.im * b.im}; }
  static __device__ __forceinline__ D prod(D a, D b) { return {a.re * b.re, a.im * b.im}; }
  static __device__ __forceinline__ cx<double> mul(D s, cx<double> v) { return {s.re * v.re, s.im * v.im}; }
  static __device__ __forceinline__ double sum(D s) { return s.re + s.im; }
  static __device__ __forceinline__ double max2(cx<double> v) { return fmax(v.re * v.re, v.im * v.im); }
  static __device__ __forceinline__ double asum(double al, D a, D b) { return al * a.re * b.re + al * a.im * b.im; }
};

// Algorithm 1 on F: Y = p X_b + q G_b.
template <typename TF, bool PAIR = false>
struct FOps {
  using W = Pw<PAIR>;
  using D = typename W::D;
  struct In { cx<TF> x, g; };
  const ProbDev& P; const SolverState& S;
  const void *xb, *gb; void *xo, *go;
  __device__ FOps(const ProbDev& P_, const SolverState& S_) : P(P_), S(S_) {
    xb = sel2(P.xf, S.cur); gb = sel2(P.gf, S.cur); xo = sel2(P.xf, S.cur ^ 1); go = sel2(P.gf, S.cur ^ 1);
  }
  __device__ __forceinline__ In load(int64_t g) const { return In{ld<TF>(xb, g), ld<TF>(gb, g)}; }
  __device__ __forceinline__ cx<double> trial(const In& in) const {
    return S.p * cvt<double>(in.x) + S.q * cvt<double>(in.g);
  }
  __device__ __forceinline__ void metrics1(const In& in, cx<double> y, Acc1& a) const {
    const cx<double> x = cvt<double>(in.x), gr = cvt<double>(in.g);
    a.np2 += abs2(S.n_b * gr - S.a_b * x);
    a.rmax = fmax(a.rmax, W::max2(gr - (S.a_b / S.n_b) * x));
    a.ny += abs2(y);
  }
  // kin: kinetic(+rotation) part of H_lin applied to the unscaled trial
  __device__ __forceinline__ void final_(const In& in, int64_t g, D vg, cx<double> kin, double c,
                                         double n_hat, AccF& a) const {
    const cx<double> x = cvt<double>(in.x), gr = cvt<double>(in.g);
    const cx<TF> ys = realify(P, cvt<TF>(c * trial(in)));
    const cx<double> y = cvt<double>(ys);
    const D q = W::dens(y);
    const cx<double> ay = 2.0 * (c * kin + W::mul(vg, y));
    const cx<TF> gs = realify(P, cvt<TF>(ay + W::mul(4.0 * P.alpha * q, y)));
    const cx<double> gy = cvt<double>(gs);
    stc<TF>(xo, g, ys);
    stc<TF>(go, g, gs);
    a.s[SF_F] += 0.5 * redot(y, ay) + W::asum(P.alpha, q, q);
    const cx<double> s = y - x;
    const cx<double> w0 = n_hat * gy - S.n_b * gr - S.a_b * s;
    a.s[SF_A] += redot(y, gy);
    a.s[SF_NG] += abs2(gy);
    a.s[SF_NY] += W::sum(q);
    a.s[SF_SS] += abs2(s);
    a.s[SF_SY] += redot(s, y);
    a.s[SF_SG] += redot(s, gy);
    a.s[SF_SW0] += redot(s, w0);
    a.s[SF_W0W0] += abs2(w0);
    a.s[SF_W0G] += redot(w0, gy);
    a.s[SF_W0Y] += redot(w0, y);
    a.smax = fmax(a.smax, W::max2(s));
  }
};

// Newton subproblem, delta form: X = X_k + S, grad_W = G_k + D,
// S_new = (p-1) X_k + p S_b + q (G_k + D_b).
template <typename TW, bool PAIR = false>
struct WOps {
  using W = Pw<PAIR>;
  using D = typename W::D;
  struct In { cx<double> xk, gk; cx<TW> s, d; };
  const ProbDev& P; const SolverState& S;
  const void *xk, *gk, *sb, *db; void *so, *dout;
  __device__ WOps(const ProbDev& P_, const SolverState& S_) : P(P_), S(S_) {
    xk = P.xk;
    gk = P.gk;
    sb = sel2(P.s, S.cur); db = sel2(P.d, S.cur); so = sel2(P.s, S.cur ^ 1); dout = sel2(P.d, S.cur ^ 1);
  }
  __device__ __forceinline__ In load(int64_t g) const {
    return In{ld<double>(xk, g), ld<double>(gk, g), ld<TW>(sb, g), ld<TW>(db, g)};
  }
  __device__ __forceinline__ cx<double> trial(const In& in) const {
    return S.pm1 * in.xk + S.p * cvt<double>(in.s) + S.q * (in.gk + cvt<double>(in.d));
  }
  __device__ __forceinline__ void metrics1(const In& in, cx<double> sn, Acc1& a) const {
    const cx<double> s = cvt<double>(in.s), d = cvt<double>(in.d);
    const cx<double> gb = in.gk + d, xb = in.xk + s;
    a.np2 += abs2((S.n_b * in.gk - S.a_b * in.xk) + (S.n_b * d - S.a_b * s));
    a.rmax = fmax(a.rmax, W::max2(gb - (S.a_b / S.n_b) * xb));
    a.ny += abs2(in.xk + sn);
  }
  __device__ __forceinline__ void final_(const In& in, int64_t g, D vg, cx<double> kin, double c,
                                         double n_hat, AccF& a) const {
    const cx<double> x0 = in.xk, g0 = in.gk;
    const cx<double> s = cvt<double>(in.s), d = cvt<double>(in.d);
    const cx<double> sn = trial(in);
    const D qk = W::dens(x0);
    const double al4 = 4.0 * P.alpha;
    const cx<double> axk = g0 - W::mul(al4 * qk, x0);                 // A X_k
    const cx<TW> ss = realify(P, cvt<TW>(c * sn + (c - 1.0) * x0));   // renormalised S
    const cx<double> sv = cvt<double>(ss);
    const cx<double> as = c * (2.0 * (kin + W::mul(vg, sn))) + (c - 1.0) * axk;  // A S
    const cx<TW> ds = realify(P, cvt<TW>(as + al4 * (W::mul(qk, sv) + W::mul(2.0 * W::pdot(x0, sv), x0)) +
                                         S.delta * sv));
    const cx<double> dv = cvt<double>(ds);
    stc<TW>(so, g, ss);
    stc<TW>(dout, g, ds);
    const cx<double> y = x0 + sv, gy = g0 + dv;
    const D ny = W::dens(y);
    a.s[SF_F] += redot(sv, g0) + 0.5 * redot(sv, dv);
    a.s[SF_A] += redot(y, gy);
    a.s[SF_NG] += abs2(gy);
    a.s[SF_NY] += W::sum(ny);
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
                    + W::asum(P.alpha, 2.0 * W::pdot(x0, sv) + W::dens(sv), ny + qk);
    a.smax = fmax(a.smax, W::max2(sb_));
  }
};

// Float64 evaluation at a new outer iterate; writes X_k, G_k and clears S/D.
template <typename TF, typename TW, bool PAIR = false>
struct OOps {
  using W = Pw<PAIR>;
  using D = typename W::D;
  struct In { cx<double> y, x0; };     // the point before renormalisation, and the old X_k
  const ProbDev& P; const SolverState& S;
  void *xk, *gk; const void *xf, *sc;
  __device__ OOps(const ProbDev& P_, const SolverState& S_) : P(P_), S(S_) {
    xk = P.xk;
    gk = P.gk;
    xf = sel2(P.xf, S.cur);
    sc = sel2(P.s, S.cur);
  }
  __device__ __forceinline__ In load(int64_t g) const {
    if (S.src == SRC_XF) {
      const cx<double> y = cvt<double>(ld<TF>(xf, g));
      return In{y, y};
    }
    const cx<double> x0 = ld<double>(xk, g);
    if (S.src == SRC_XK_PLUS_S) return In{x0 + cvt<double>(ld<TW>(sc, g)), x0};
    return In{x0, x0};
  }
  __device__ __forceinline__ cx<double> trial(const In& in) const { return in.y; }
  __device__ __forceinline__ void metrics1(const In&, cx<double> y, Acc1& a) const { a.ny += abs2(y); }
  __device__ __forceinline__ void final_(const In& in, int64_t g, D vg, cx<double> kin, double c, double,
                                         AccF& a) const {
    const cx<double> y = realify(P, c * in.y);
    const D q = W::dens(y);
    const cx<double> ay = 2.0 * (c * kin + W::mul(vg, y));
    const cx<double> gy = realify(P, ay + W::mul(4.0 * P.alpha * q, y));
    stc<double>(xk, g, y);
    stc<double>(gk, g, gy);
    stc<TW>(P.s[0], g, cx<TW>{0, 0});
    stc<TW>(P.d[0], g, cx<TW>{0, 0});
    a.s[SF_F] += 0.5 * redot(y, ay) + W::asum(P.alpha, q, q);
    a.s[SF_A] += redot(y, gy);
    a.s[SF_NG] += abs2(gy);
    a.s[SF_NY] += W::sum(q);
    a.smax = fmax(a.smax, W::max2(y - in.x0));   // |X_{k+1} - X_k|^2 (Newton step lengths)
  }
};

// ---------------------------------------------------------------------------
// One tile of one pass for a given mode.  P and S are local copies (read once
// at kernel entry, before any store).  Every input of the tile goes out as
// one batch of loads: the trial point's arrays, the accumulator of the
// earlier passes, the potential, the twiddle table and (final pass) the
// first pass's norm partials.
// RR (epilogue roles): the epilogue reads the trial point's inputs again,
// half of the elements at a time, with the accumulator and the potential
// (cache hits: the workgroup read the inputs before its transforms), instead
// of holding them in registers through the transforms.  That takes the final
// pass from one wavefront per SIMD to two, which pays where the launch has
// enough tiles to be bandwidth bound and costs a little latency where not.
// ---------------------------------------------------------------------------
// PAIR: see Tile (the x pass regroups its row pairs into transform lines
// and back through LDS).
template <int N, int E, int ROLE, typename CT, class Ops, bool RR, bool PAIR>
__device__ __forceinline__ void solver_tile(const ProbDev& P, const SolverState& S, int tile, const Ops& ops,
                                            cx<CT>* lds, const cx<CT>* tw1024, double* red) {
  constexpr bool HAS_T = (ROLE == R_MID || ROLE == R_FINAL);
  constexpr bool EPI = (ROLE == R_FINAL || ROLE == R_SOLO);
  const int ax = role_axis(ROLE, P.dim);
  const Tile<N, E, PAIR> T(P, ax, HAS_T, tile);
  TwiddleFetch<N, CT> twf;
  twf.fetch(tw1024);
  typename Ops::In in[E];
  cx<CT> tv[E];
  typename Tile<N, E, PAIR>::VP vp[E];
  constexpr bool LATE = EPI && RR;
  // loads in the order of use: the trial point's inputs first, so that the
  // transforms wait for those alone (loads return in order), then what only
  // the end of the pass needs (t, V, the first pass's norm partials)
#pragma unroll
  for (int e = 0; e < E; ++e) in[e] = ops.load(T.g(e));
  if constexpr (HAS_T && !LATE)
#pragma unroll
    for (int e = 0; e < E; ++e) tv[e] = ld<CT>(P.t, T.g(e));
  if constexpr (EPI && !LATE) T.pot_load(P, vp);
  double c = 1.0, n_hat = 1.0;
  // every wavefront of the final pass reduces the first pass's norm partials
  // itself; with 4 points per thread, no re-read epilogue and at most 256
  // first-pass tiles their loads go out here and the sum is taken after the
  // transforms (elsewhere the registers are needed more)
  constexpr bool EARLY_NY = ROLE == R_FINAL && !LATE && E == 4;
  const bool early_ny = EARLY_NY && P.tiles[0] <= 64 * kNyLoads;
  SlotLoads<kNyLoads> nyl;
  if constexpr (EARLY_NY)
    if (early_ny) nyl.load(P.part1 + (int64_t)S1_NY * P.tiles[0], P.tiles[0]);
  auto renorm = [&](double ny) {
    c = renorm_c(S, ny);
    n_hat = c * c * ny;
  };
  if constexpr (ROLE == R_FINAL)
    if (!early_ny) renorm(wave_reduce_slot(P.part1, P.tiles[0], S1_NY, false));
  twf.store(lds);
  cx<CT> v[E];
  Acc1 a1;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const cx<double> y = ops.trial(in[e]);
    if constexpr (ROLE == R_FIRST || ROLE == R_SOLO)
      if (T.inner(e)) ops.metrics1(in[e], y, a1);
    v[e] = cvt<CT>(T.sgn(e) * y);
  }
  if constexpr (ROLE == R_SOLO) {
    double acc[3] = {a1.ny, a1.np2, a1.rmax};
    block_reduce<2, 1>(acc, red);
    __shared__ double bc;
    if (threadIdx.x == 0) {
      bc = acc[0];
      gst<double>(P.part1, S1_NY, acc[0]);
      gst<double>(P.part1, S1_NP2, acc[1]);
      gst<double>(P.part1, S1_RMAX, acc[2]);
    }
    __syncthreads();
    c = renorm_c(S, bc);
    n_hat = c * c * bc;
  }
  if constexpr (PAIR && ROLE == R_FIRST) pair_to_line<N, E, CT>(T, v, lds + N);
  spectral_apply<N, E, CT>(P, ax, T, v, lds);
  if constexpr (PAIR && ROLE == R_FIRST) line_to_pair<N, E, CT>(T, v, lds + N);
  if constexpr (EARLY_NY)
    if (early_ny) renorm(nyl.sum(P.tiles[0]));
  if constexpr (ROLE == R_FIRST) {
#pragma unroll
    for (int e = 0; e < E; ++e)
      if (T.inner(e)) stc<CT>(P.t, T.g(e), v[e]);
    double acc[3] = {a1.ny, a1.np2, a1.rmax};
    const int64_t nt = P.tiles[0];
    if (blockDim.x == 64) {
      // one wavefront: slot k's sum lands in lane 4k, which stores it
      const double r = wave_reduce_lds<S1_COUNT>(acc, 1u << S1_RMAX, red);
      if ((threadIdx.x & 3) == 0 && (threadIdx.x >> 2) < S1_COUNT)
        gst<double>(P.part1, (threadIdx.x >> 2) * nt + tile, r);
    } else {
      block_reduce<2, 1>(acc, red);
      if (threadIdx.x == 0) {
        gst<double>(P.part1, S1_NY * nt + tile, acc[0]);
        gst<double>(P.part1, S1_NP2 * nt + tile, acc[1]);
        gst<double>(P.part1, S1_RMAX * nt + tile, acc[2]);
      }
    }
  } else if constexpr (ROLE == R_MID) {
#pragma unroll
    for (int e = 0; e < E; ++e)
      if (T.inner(e)) stc<CT>(P.t, T.g(e), tv[e] + v[e]);
  } else {
    AccF af;
    constexpr int G = LATE ? 2 : 1;          // element groups of the epilogue
#pragma unroll
    for (int hh = 0; hh < G; ++hh) {
      if constexpr (LATE) {
        __builtin_amdgcn_sched_barrier(0);    // keep the groups' loads apart
#pragma unroll
        for (int e = hh * (E / G); e < (hh + 1) * (E / G); ++e) {
          in[e] = ops.load(T.g(e));
          if constexpr (HAS_T) tv[e] = ld<CT>(P.t, T.g(e));
          vp[e] = T.pot_one(P, e);
        }
      }
#pragma unroll
      for (int e = hh * (E / G); e < (hh + 1) * (E / G); ++e)
        if (T.inner(e)) {
          cx<double> kin = cvt<double>(v[e]);
          if constexpr (HAS_T) kin = kin + cvt<double>(tv[e]);
          ops.final_(in[e], T.g(e), T.pot_value(P, vp[e]), kin, c, n_hat, af);
        }
    }
    double acc[SF_COUNT];
#pragma unroll
    for (int i = 0; i < SF_COUNT_SUM; ++i) acc[i] = af.s[i];
    acc[SF_SMAX] = af.smax;
    const int64_t nt = pick3(P.tiles, P.dim - 1);
    if (blockDim.x == 64) {
      const double r = wave_reduce_lds<SF_COUNT>(acc, 1u << SF_SMAX, red);
      if ((threadIdx.x & 3) == 0 && (threadIdx.x >> 2) < SF_COUNT)
        gst<double>(P.partF, (threadIdx.x >> 2) * nt + tile, r);
    } else {
      block_reduce<SF_COUNT_SUM, 1>(acc, red);
      if (threadIdx.x == 0)
#pragma unroll
        for (int i = 0; i < SF_COUNT; ++i) gst<double>(P.partF, i * nt + tile, acc[i]);
    }
  }
}

// The last workgroup to finish a problem's final pass (ticket counter) runs
// the scalar step of the solver on the reduced partial sums.
__device__ __forceinline__ void step_if_last(const ProbDev& P, SolverState* Sg, int ntiles, int prec64,
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
  if (threadIdx.x < 64) touch_lines(Sg);
  double r1[S1_COUNT], rf[SF_COUNT];
  step_reductions(P.part1, P.tiles[0], P.partF, ntiles, r1, rf, red);
  if (threadIdx.x == 0) {
    SolverState L = *Sg;
    step_logic(P, L, r1, rf, prec64);
    *Sg = L;
  }
}

// STEP_FUSED: the scalar step of the previous evaluation, run by every
// wavefront of the first pass on its own (every lane on the same values, so
// each copy of the state gets the same bits without any exchange); the
// workgroup of tile 0 stores the new state for the later passes and the
// host.  `part1_prev` holds the previous evaluation's first-pass partials.
// The partial sums are read before the state is known to need them, so that
// their loads go out with the state's.
__device__ __forceinline__ void fused_step(const ProbDev& P, SolverState& S, const double* part1_prev,
                                           SolverState* out, bool writer, int prec64) {
  double r1[S1_COUNT], rf[SF_COUNT];
  wave_reduce_all(part1_prev, P.tiles[0], P.partF, pick3(P.tiles, P.dim - 1), r1, rf);
  if (S.pending && S.mode != M_IDLE) step_logic(P, S, r1, rf, prec64);
  S.pending = S.mode != M_IDLE ? 1 : 0;
  if (writer && threadIdx.x == 0) *out = S;
}

// The state fields the passes read.
#define GPE_PASS_STATE_FIELDS(F) \
  F(S.mode); F(S.cur); F(S.src); F(S.force_norm); F(S.p); F(S.q); F(S.pm1); F(S.n_b); F(S.a_b); \
  F(S.delta); F(S.renorm_tol)

// The descriptor fields the passes read, forced into registers at kernel
// entry.
__device__ __forceinline__ void pin_desc_fields(ProbDev& P) {
  pin_reg(P.dim); pin_reg(P.n[0]); pin_reg(P.n[1]); pin_reg(P.n[2]);
  pin_reg(P.nl[0]); pin_reg(P.nl[1]); pin_reg(P.nl[2]); pin_reg(P.bc);
  pin_reg(P.x0[0]); pin_reg(P.x0[1]);
  pin_reg(P.stride[1]); pin_reg(P.stride[2]); pin_reg(P.m);
  pin_reg(P.tiles[0]); pin_reg(P.tiles[1]); pin_reg(P.tiles[2]);
  pin_reg(P.has_v); pin_reg(P.step_at); pin_reg(P.real);
  pin_reg(P.h[0]); pin_reg(P.h[1]);
  pin_reg(P.len[0]); pin_reg(P.len[1]); pin_reg(P.len[2]);
  pin_reg(P.omega); pin_reg(P.alpha);
  pin_reg(P.v_arr); pin_reg(P.v_axis);
  pin_reg(P.xf[0]); pin_reg(P.xf[1]); pin_reg(P.gf[0]); pin_reg(P.gf[1]);
  pin_reg(P.s[0]); pin_reg(P.s[1]); pin_reg(P.d[0]); pin_reg(P.d[1]);
  pin_reg(P.xk); pin_reg(P.gk); pin_reg(P.t); pin_reg(P.part1); pin_reg(P.part1x); pin_reg(P.partF);
}

// Dispatch on the problem's mode.  PREC64: every array float64.
template <int N, int E, int ROLE, bool PREC64, bool RR, bool PAIR>
__device__ __forceinline__ void solver_dispatch(const ProbDev& P, const SolverState& S, int tile, char* smem,
                                                const cx<double>* twd, const cx<float>* twf, double* red) {
  using TS = typename std::conditional<PREC64, double, float>::type;   // F/W storage and transforms
  const cx<TS>* tws = PREC64 ? reinterpret_cast<const cx<TS>*>(twd) : reinterpret_cast<const cx<TS>*>(twf);
  if (S.mode == M_F) {
    using O = FOps<TS, PAIR>;
    O ops(P, S);
    solver_tile<N, E, ROLE, TS, O, RR, PAIR>(P, S, tile, ops, reinterpret_cast<cx<TS>*>(smem), tws, red);
  } else if (S.mode == M_W) {
    using O = WOps<TS, PAIR>;
    O ops(P, S);
    solver_tile<N, E, ROLE, TS, O, RR, PAIR>(P, S, tile, ops, reinterpret_cast<cx<TS>*>(smem), tws, red);
  } else if (S.mode == M_OUTER) {
    using O = OOps<TS, TS, PAIR>;
    O ops(P, S);
    solver_tile<N, E, ROLE, double, O, RR, PAIR>(P, S, tile, ops, reinterpret_cast<cx<double>*>(smem), twd, red);
  }
}

// `bmap` maps a workgroup to (problem, tile); null for a single problem
// (workgroup b is tile b of problem 0).  EPT: transform points per thread
// (8 or 4; the host launches the instance of its plan).  PAIR: real grid
// functions two points to an element (see Tile; every problem of the launch
// is so stored).  RR: see solver_tile.  FUSED (first
// pass only): the pass runs the previous evaluation's scalar step first
// (STEP_FUSED; an instance of its own, so that the other instances carry
// none of its code and registers).  The passes
// read the state from st_in; with STEP_FUSED the first pass stores the state
// after its step in st_out (the host alternates two state arrays and passes
// the evaluation's parity `par`, which also selects the first-pass partials
// buffer); otherwise st_out is st_in and par is 0.
template <int ROLE, bool PREC64, bool RR, bool FUSED, int EPT, bool PAIR>
__global__ void __launch_bounds__(256) k_solver_pass(const ProbDev* __restrict__ probs,
                                                     SolverState* __restrict__ st_in,
                                                     SolverState* __restrict__ st_out,
                                                     const int2* __restrict__ bmap,
                                                     const cx<double>* __restrict__ twd,
                                                     const cx<float>* __restrict__ twf, int par) {
  extern __shared__ __align__(16) char smem[];
  // the block reduction's scratch, or the one-wavefront transpose's
  __shared__ double red[SF_COUNT * 65 > SF_COUNT * 16 ? SF_COUNT * 65 : SF_COUNT * 16];
  const int b = xcd_tile((int)blockIdx.x, (int)gridDim.x);
  const int2 bm = bmap ? bmap[b] : make_int2(0, b);
  // local copies, read in one batch: the fields the pass needs pinned in
  // scalar registers
  ProbDev P = probs[bm.x];
  pin_desc_fields(P);
  SolverState S = st_in[bm.x];
  GPE_PASS_STATE_FIELDS(pin_reg);
  double* const part1_other = par ? P.part1 : P.part1x;
  if (par) P.part1 = P.part1x;
  if constexpr (ROLE == R_FIRST && FUSED) {
    fused_step(P, S, part1_other, st_out + bm.x, bm.y == 0, PREC64 ? 1 : 0);
    GPE_PASS_STATE_FIELDS(make_uniform);
  }
  if (S.mode == M_IDLE) return;
  // line length of this pass; EPT points per thread (an instance per count)
  const int n = pick3(P.nl, role_axis(ROLE, P.dim));
#define GPE_SOLVER_CASE(NN)                                                   \
  case NN:                                                                    \
    solver_dispatch<NN, EPT, ROLE, PREC64, RR, PAIR>(P, S, bm.y, smem, twd, twf, red); \
    break;
  switch (n) {
    GPE_SOLVER_CASE(16) GPE_SOLVER_CASE(32) GPE_SOLVER_CASE(64) GPE_SOLVER_CASE(128)
    GPE_SOLVER_CASE(256) GPE_SOLVER_CASE(512) GPE_SOLVER_CASE(1024)
    default: break;
  }
#undef GPE_SOLVER_CASE
  if constexpr (ROLE == R_FINAL || ROLE == R_SOLO)
    if (P.step_at == STEP_LAST_GROUP)
      step_if_last(P, st_in + bm.x, ROLE == R_SOLO ? 1 : pick3(P.tiles, P.dim - 1), PREC64 ? 1 : 0, red);
}

}  // namespace gpe
