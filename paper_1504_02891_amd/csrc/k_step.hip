// Small kernels around a solve: initial data, write-back, apply_h outputs,
// the stand-alone Cayley retraction and the trigonometric prolongation.
#include "gpe_launch.h"
#include "passes_impl.h"  // reductions and helpers

namespace gpe {

// Scalar step as its own launch (one workgroup per problem): the partial
// sums are reduced by the first wavefront (all wavefronts, slot by slot, when
// there are many tiles); the state is copied in with one batch of loads,
// advanced in registers by one thread and written back whole.
constexpr int kStepThreads = 512;
__global__ void __launch_bounds__(kStepThreads) k_step(const ProbDev* __restrict__ probs,
                                                       SolverState* __restrict__ states) {
  __shared__ double red[S1_COUNT + SF_COUNT];
  __shared__ double tbuf[(S1_COUNT + SF_COUNT) * 65];
  ProbDev P = probs[blockIdx.x];
  pin_reg(P.part1); pin_reg(P.partF); pin_reg(P.tiles[0]); pin_reg(P.tiles[1]); pin_reg(P.tiles[2]);
  pin_reg(P.dim); pin_reg(P.sqrt_hvol); pin_reg(P.prec64);
  // the partial sums are reduced before the state is known to need them, so
  // that their loads go out with the state's
  if (threadIdx.x < 64) touch_lines(states + blockIdx.x);
  double r1[S1_COUNT], rf[SF_COUNT];
  step_reductions(P.part1, P.tiles[0], P.partF, pick3(P.tiles, P.dim - 1), r1, rf, red, tbuf);
  if (states[blockIdx.x].mode == M_IDLE) return;
  if (threadIdx.x == 0) {
    SolverState L = states[blockIdx.x];
    step_logic(P, L, r1, rf, P.prec64);
    states[blockIdx.x] = L;
  }
}


// ---- initial data: X_0 = sqrt(h_vol) phi_0 in the F-mode arrays, G = 0 ----
// (pair storage: element g holds the real parts of points 2g and 2g + 1)
template <typename TF>
__global__ void k_init(const ProbDev* probs, int pi, const cx<double>* __restrict__ phi0) {
  const ProbDev& P = probs[pi];
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < P.m; g += (int64_t)gridDim.x * blockDim.x) {
    const cx<double> u = P.pair ? cx<double>{phi0[2 * g].re, phi0[2 * g + 1].re} : phi0[g];
    stc<TF>(P.xf[0], g, realify(P, cvt<TF>(P.sqrt_hvol * u)));
    stc<TF>(P.gf[0], g, cx<TF>{0, 0});
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) *P.ticket = 0;
}

// ---- write phi = X / sqrt(h_vol) of the final iterate ----
template <typename TF>
__global__ void k_write_phi(const ProbDev* probs, const SolverState* states, int pi, cx<double>* __restrict__ phi) {
  const ProbDev& P = probs[pi];
  const SolverState& S = states[pi];
  const double sc = 1.0 / P.sqrt_hvol;
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < P.m; g += (int64_t)gridDim.x * blockDim.x) {
    cx<double> x = (S.src == SRC_XF) ? cvt<double>(ld<TF>(P.xf[S.cur], g)) : reinterpret_cast<const cx<double>*>(P.xk)[g];
    if (P.pair) {
      phi[2 * g] = cx<double>{sc * x.re, 0.0};
      phi[2 * g + 1] = cx<double>{sc * x.im, 0.0};
    } else {
      phi[g] = sc * x;
    }
  }
}

// ---- apply_h outputs: residual max |H phi - mu phi| and the scalar summary ----
// Fixed-order reduction of slot-major partials part[s * count + i], i < count,
// s < NSLOT (the last NM slots maxima) by one workgroup of kSumThreads
// threads: thread j takes i = j, j + kSumThreads, ... in turn (loads in
// batches), then the block reduction.  Thread 0 gets the result.
constexpr int kSumThreads = 1024;
template <int NS, int NM>
__device__ __forceinline__ void block_sum_partials(const double* part, int count, double* acc, double* red) {
  constexpr int NSLOT = NS + NM;
  // loads in flight per slot per thread (at most 128 registers at 1024 threads)
  constexpr int B = NSLOT >= 4 ? 4 : 8;
#pragma unroll
  for (int s = 0; s < NSLOT; ++s) acc[s] = 0.0;
  for (int b0 = 0; b0 < count; b0 += B * kSumThreads) {
    double v[B][NSLOT];
#pragma unroll
    for (int j = 0; j < B; ++j) {
      const int64_t i = min(b0 + (int)threadIdx.x + j * kSumThreads, count - 1);
#pragma unroll
      for (int s = 0; s < NSLOT; ++s) v[j][s] = gld<double>(part, (int64_t)s * count + i);
    }
#pragma unroll
    for (int j = 0; j < B; ++j)
      if (b0 + (int)threadIdx.x + j * kSumThreads < count)
#pragma unroll
        for (int s = 0; s < NSLOT; ++s) acc[s] = s < NS ? acc[s] + v[j][s] : fmax(acc[s], v[j][s]);
  }
  block_reduce<NS, NM>(acc, red);
}

// Totals of the last pass's `count` partials per slot (one per wavefront),
// in two fixed-order stages: workgroup (s, c) sums chunk c of slot s into
// tot[s * kSumChunks + c]; slot_total adds the chunks in order.
constexpr int kSumChunks = 16;
__global__ void __launch_bounds__(256) k_apply_sums(const ProbDev* probs, int count, double* __restrict__ tot) {
  __shared__ double red[16];
  const ProbDev& P = probs[0];
  const int slot = blockIdx.x / kSumChunks, chunk = blockIdx.x % kSumChunks;
  const int len = (count + kSumChunks - 1) / kSumChunks;
  const int lo = chunk * len, hi = min(count, lo + len);
  const double* part = P.partF + (int64_t)slot * count;
  double acc[1] = {0.0};
  for (int b0 = lo; b0 < hi; b0 += 8 * 256) {   // thread j: i = lo + j, lo + j + 256, ...
    double v[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int i = b0 + (int)threadIdx.x + j * 256;
      v[j] = i < hi ? gld<double>(part, i) : 0.0;
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) acc[0] += v[j];
  }
  block_reduce<1, 0>(acc, red);
  if (threadIdx.x == 0) tot[blockIdx.x] = acc[0];
}
__device__ __forceinline__ double slot_total(const double* tot, int slot) {
  double s = 0.0;
#pragma unroll
  for (int c = 0; c < kSumChunks; ++c) s += tot[slot * kSumChunks + c];
  return s;
}

// E and mu from the last pass's totals: mu = h_vol sum Re(conj(phi) H phi),
// E = mu - beta/2 h_vol sum |phi|^4 (§1: mu = E + beta/2 int |phi|^4)
__device__ __forceinline__ double apply_mu(const ProbDev& P, const double* tot) {
  return P.hvol * slot_total(tot, SA_MU);
}
__device__ __forceinline__ double apply_energy(const ProbDev& P, const double* tot) {
  return apply_mu(P, tot) - 0.5 * P.beta * P.hvol * slot_total(tot, SA_QUART);
}

// q = a / d and a - q d for a < 2^31, d >= 1, rd = 1/d rounded: the FP64
// quotient a * rd is within 2^-21 of a / d, so one correction step suffices.
__device__ __forceinline__ uint32_t div_rcp(uint32_t a, uint32_t d, double rd, uint32_t& rem) {
  uint32_t q = (uint32_t)((double)a * rd);
  int32_t r = (int32_t)(a - q * d);
  if (r < 0) { q -= 1; r += (int32_t)d; }
  else if (r >= (int32_t)d) { q += 1; r -= (int32_t)d; }
  rem = (uint32_t)r;
  return q;
}

// Residual pass: per block, sums of |phi|^2 and x_a^2 |phi|^2 and the maxima
// of |phi|^2 and |H phi - mu phi|^2 (rpart slot-major, [SR_COUNT][gridDim]).
template <typename T>
__global__ void __launch_bounds__(256) k_apply_resid(const ProbDev* probs, const cx<T>* __restrict__ phi,
                                                     const cx<T>* __restrict__ hphi, const double* __restrict__ tot,
                                                     double* __restrict__ rpart) {
  __shared__ double red[SR_COUNT * 16];
  const ProbDev& P = probs[0];
  const double mu = apply_mu(P, tot);
  const uint32_t n0 = (uint32_t)P.n[0], n1 = (uint32_t)P.n[1];
  const double r0 = 1.0 / (double)n0, r1 = 1.0 / (double)n1;
  double acc[SR_COUNT] = {};
  auto point = [&](int64_t g, cx<T> pu, cx<T> ph) {
    const cx<double> u = cvt<double>(pu), h = cvt<double>(ph);
    const double q = abs2(u);
    uint32_t i0, i1;
    const uint32_t i2 = div_rcp(div_rcp((uint32_t)g, n0, r0, i0), n1, r1, i1);
    const double x = P.x0[0] + P.h[0] * (double)i0, y = P.x0[1] + P.h[1] * (double)i1,
                 z = P.x0[2] + P.h[2] * (double)i2;
    acc[SR_NORM] += q;
    acc[SR_X2] += x * x * q;
    acc[SR_Y2] += y * y * q;
    acc[SR_Z2] += z * z * q;
    acc[SR_MAXD] = fmax(acc[SR_MAXD], q);
    acc[SR_RES] = fmax(acc[SR_RES], abs2(h - mu * u));
  };
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  constexpr int U = sizeof(T) == 4 ? 4 : 1;     // points whose loads are in flight together
  for (; g + (U - 1) * stride < P.m; g += U * stride) {
    cx<T> u[U], h[U];
#pragma unroll
    for (int k = 0; k < U; ++k) {
      u[k] = phi[g + k * stride];
      h[k] = hphi[g + k * stride];
    }
#pragma unroll
    for (int k = 0; k < U; ++k) point(g + k * stride, u[k], h[k]);
  }
  for (; g < P.m; g += stride) point(g, phi[g], hphi[g]);
  block_reduce<SR_COUNT_SUM, 2>(acc, red);
  if (threadIdx.x == 0)
#pragma unroll
    for (int s = 0; s < SR_COUNT; ++s) rpart[(int64_t)s * gridDim.x + blockIdx.x] = acc[s];
}

// The scalars documented for gpe_apply_h: out[0] = E, out[1] = mu, out[2] the
// residual, out[3..9] norm, rms, max density, energy parts.
__global__ void __launch_bounds__(kSumThreads) k_apply_finalize(const ProbDev* probs, const double* __restrict__ tot,
                                                                const double* __restrict__ rpart, int nr,
                                                                double* __restrict__ out) {
  __shared__ double red[SR_COUNT * 16];
  __shared__ double tl[SA_COUNT * kSumChunks];
  const ProbDev& P = probs[0];
  // the chunk totals go out with the residual partials' loads (one each for
  // the first threads) and reach thread 0 through LDS
  constexpr int NT = SA_COUNT * kSumChunks;
  double tv = 0.0;
  if (threadIdx.x < NT) tv = tot[threadIdx.x];
  double acc[SR_COUNT];
  block_sum_partials<SR_COUNT_SUM, 2>(rpart, nr, acc, red);
  if (threadIdx.x < NT) tl[threadIdx.x] = tv;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double e = apply_energy(P, tl), epot = P.hvol * slot_total(tl, SA_POT);
    out[0] = e;
    out[1] = apply_mu(P, tl);
    out[2] = sqrt(acc[SR_RES]);
    out[3] = P.hvol * acc[SR_NORM];
    out[4] = sqrt(P.hvol * acc[SR_X2]);
    out[5] = sqrt(P.hvol * acc[SR_Y2]);
    out[6] = sqrt(P.hvol * acc[SR_Z2]);
    out[7] = acc[SR_MAXD];
    out[8] = e - epot - 0.5 * P.beta * P.hvol * slot_total(tl, SA_QUART);
    out[9] = epot;
  }
}

// ---- largest |Im| of the initial data (choice of real arithmetic) ----
__global__ void __launch_bounds__(256) k_max_imag(const cx<double>* __restrict__ x, int64_t m,
                                                  double* __restrict__ part) {
  __shared__ double red[16];
  double a[1] = {0.0};
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x)
    a[0] = fmax(a[0], fabs(x[i].im));
  block_reduce<0, 1>(a, red);
  if (threadIdx.x == 0) part[blockIdx.x] = a[0];
}

// ---- Cayley retraction (Theorem 3.3) on plain vectors ----
// T: element type of x, g, y (complex float64, or complex float32 with the
// products converted to and summed in float64)
template <typename T>
__global__ void __launch_bounds__(256) k_retract_reduce(const cx<T>* __restrict__ x, const cx<T>* __restrict__ g,
                                                        int64_t m, double* __restrict__ part) {
  __shared__ double red[3 * 16];
  double acc[3] = {0.0, 0.0, 0.0};
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
    const cx<double> a = cvt<double>(x[i]), b = cvt<double>(g[i]);
    acc[0] += redot(a, b);
    acc[1] += abs2(a);
    acc[2] += abs2(b);
  }
  block_reduce<3, 0>(acc, red);
  if (threadIdx.x == 0) {
    part[0 * gridDim.x + blockIdx.x] = acc[0];
    part[1 * gridDim.x + blockIdx.x] = acc[1];
    part[2 * gridDim.x + blockIdx.x] = acc[2];
  }
}

template <typename T>
__global__ void __launch_bounds__(256) k_retract_apply(const cx<T>* __restrict__ x, const cx<T>* __restrict__ g,
                                                       cx<T>* __restrict__ y, int64_t m, double tau,
                                                       const double* __restrict__ part, int np,
                                                       double* __restrict__ coeffs) {
  __shared__ double red[4];
  const double a = fixed_reduce(part, np, 0, false, red);
  const double nx = fixed_reduce(part, np, 1, false, red);
  const double ng = fixed_reduce(part, np, 2, false, red);
  const double den = 1.0 - tau * tau * a * a + tau * tau * nx * ng;
  const double p = ((1.0 + tau * a) * (1.0 + tau * a) - tau * tau * nx * ng) / den;
  const double q = -2.0 * tau * nx / den;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = cvt<T>(p * cvt<double>(x[i]) + q * cvt<double>(g[i]));
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    coeffs[0] = p; coeffs[1] = q; coeffs[2] = a; coeffs[3] = nx; coeffs[4] = ng;
  }
}

// ---- trigonometric prolongation along one axis (NC -> NF = 2 NC points) ----
// Algorithm 3's interpolation of a coarse line: forward transform (NC
// points, 4 per thread), the spectrum placed on the fine grid with the
// coarse Nyquist mode split evenly between +NC/2 and -NC/2 and zeros above,
// inverse transform (NF points, 8 per thread) scaled by 1/NC.  The two line
// lengths use the same threads per line (NC/4 = NF/8).  A tile holds `lanes`
// lines: consecutive rows along x (contiguous), else consecutive columns
// (lane-interleaved, coalesced).  Input shape (a0, a1, a2); the output has
// the axis doubled.  LDS: twiddles of NC and NF points, then the line data.
template <int NC>
__global__ void __launch_bounds__(256) k_prolong_fft(const cx<double>* __restrict__ in, cx<double>* __restrict__ out,
                                                     int a0, int a1, int a2, int ax, int lanes,
                                                     const cx<double>* __restrict__ tw) {
  constexpr int NF = 2 * NC, TL = NC / 4;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<double>* twc = reinterpret_cast<cx<double>*>(smem_raw);
  cx<double>* twf = twc + NC;
  cx<double>* data = twf + NF;
  const bool strided = ax > 0;
  LdsMap mp;
  mp.lanes = lanes;
  mp.strided = strided;
  const int lane = strided ? threadIdx.x % lanes : threadIdx.x / TL;
  const int t = strided ? threadIdx.x / lanes : threadIdx.x % TL;
  const int64_t lines = (int64_t)a0 * a1 * a2 / NC;
  const int64_t L0 = (int64_t)blockIdx.x * lanes + lane;
  const bool act = L0 < lines;
  const int64_t L = act ? L0 : 0;
  int64_t bi, bo, st;
  if (ax == 0) { bi = L * NC; bo = L * NF; st = 1; }
  else if (ax == 1) {
    const int64_t x = L % a0, z = L / a0;
    bi = z * (int64_t)a0 * a1 + x; bo = z * (int64_t)a0 * 2 * a1 + x; st = a0;
  } else { bi = L; bo = L; st = (int64_t)a0 * a1; }
  TwiddleFetch<NC, double> fc;
  TwiddleFetch<NF, double> ff;
  fc.fetch(tw);
  ff.fetch(tw);
  cx<double> v[8];
#pragma unroll
  for (int e = 0; e < 4; ++e) v[e] = in[bi + (int64_t)(t + e * TL) * st];
  fc.store(twc);
  ff.store(twf);
  line_fft<NC, 4, false>(v, t, lane, mp, data, twc);   // starts with a barrier
  __syncthreads();                                     // the last stage's LDS reads are done
#pragma unroll
  for (int e = 0; e < 4; ++e) data[mp.idx(lane, t + e * TL, NC)] = v[e];
  __syncthreads();
  const double inv = 1.0 / NC;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int kf = t + e * TL;                 // fine frequency index, signed p
    const int p = kf < NF / 2 ? kf : kf - NF;
    const int ap = p < 0 ? -p : p;
    cx<double> c{0.0, 0.0};
    if (ap < NC / 2) c = inv * data[mp.idx(lane, p < 0 ? p + NC : p, NC)];
    else if (ap == NC / 2) c = (0.5 * inv) * data[mp.idx(lane, NC / 2, NC)];
    v[e] = c;
  }
  line_fft<NF, 8, true>(v, t, lane, mp, data, twf);    // starts with a barrier
  if (act)
#pragma unroll
    for (int e = 0; e < 8; ++e) out[bo + (int64_t)(t + e * TL) * st] = v[e];
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
void launch_step(hipStream_t s, int nprob, const ProbDev* probs, SolverState* st) {
  hipLaunchKernelGGL(k_step, dim3(nprob), dim3(kStepThreads), 0, s, probs, st);
}
void launch_init(hipStream_t s, const ProbDev* probs, int pi, int64_t m, const void* phi0, int prec64) {
  const int blocks = (int)std::min<int64_t>((m + 255) / 256, 4096);
  if (prec64) hipLaunchKernelGGL(k_init<double>, dim3(blocks), dim3(256), 0, s, probs, pi, (const cx<double>*)phi0);
  else hipLaunchKernelGGL(k_init<float>, dim3(blocks), dim3(256), 0, s, probs, pi, (const cx<double>*)phi0);
}
void launch_write_phi(hipStream_t s, const ProbDev* probs, const SolverState* st, int pi, int64_t m, void* phi,
                      int prec64) {
  const int blocks = (int)std::min<int64_t>((m + 255) / 256, 4096);
  if (prec64) hipLaunchKernelGGL(k_write_phi<double>, dim3(blocks), dim3(256), 0, s, probs, st, pi, (cx<double>*)phi);
  else hipLaunchKernelGGL(k_write_phi<float>, dim3(blocks), dim3(256), 0, s, probs, st, pi, (cx<double>*)phi);
}
void launch_apply_resid(hipStream_t s, int nblk, const ProbDev* probs, int nsum, const void* phi,
                        const void* hphi, double* rpart, double* tot, int fp64) {
  hipLaunchKernelGGL(k_apply_sums, dim3(SA_COUNT * kSumChunks), dim3(256), 0, s, probs, nsum, tot);
  if (fp64) hipLaunchKernelGGL(k_apply_resid<double>, dim3(nblk), dim3(256), 0, s, probs,
                               (const cx<double>*)phi, (const cx<double>*)hphi, (const double*)tot, rpart);
  else hipLaunchKernelGGL(k_apply_resid<float>, dim3(nblk), dim3(256), 0, s, probs,
                          (const cx<float>*)phi, (const cx<float>*)hphi, (const double*)tot, rpart);
}
void launch_apply_finalize(hipStream_t s, const ProbDev* probs, const double* tot, const double* rpart, int nr,
                           double* out) {
  hipLaunchKernelGGL(k_apply_finalize, dim3(1), dim3(kSumThreads), 0, s, probs, tot, rpart, nr, out);
}
template <typename T>
static void retract_t(hipStream_t s, int nblk, const void* x, const void* g, void* y, int64_t m, double tau,
                      double* part, double* coeffs) {
  hipLaunchKernelGGL(k_retract_reduce<T>, dim3(nblk), dim3(256), 0, s, (const cx<T>*)x, (const cx<T>*)g, m, part);
  hipLaunchKernelGGL(k_retract_apply<T>, dim3(nblk), dim3(256), 0, s, (const cx<T>*)x, (const cx<T>*)g, (cx<T>*)y, m,
                     tau, part, nblk, coeffs);
}
void launch_retract(hipStream_t s, int nblk, const void* x, const void* g, void* y, int64_t m, double tau,
                    double* part, double* coeffs, int fp64) {
  if (fp64) retract_t<double>(s, nblk, x, g, y, m, tau, part, coeffs);
  else retract_t<float>(s, nblk, x, g, y, m, tau, part, coeffs);
}
void launch_max_imag(hipStream_t s, int nblk, const void* x, int64_t m, double* part) {
  hipLaunchKernelGGL(k_max_imag, dim3(nblk), dim3(256), 0, s, (const cx<double>*)x, m, part);
}
int launch_prolong_axis(hipStream_t s, const void* in, void* out, int n0, int n1, int n2, int ax,
                        const void* twd) {
  const int n = ax == 0 ? n0 : (ax == 1 ? n1 : n2);
  const int tl = n / 4;
  const int64_t lines = (int64_t)n0 * n1 * n2 / n;
  int lanes = (int)std::min<int64_t>(std::max(1, 256 / tl), lines);
  auto lds = [&](int ln) { return (size_t)(3 * n + lds_elems(2 * n, ln, ax > 0)) * sizeof(cx<double>); };
  while (lanes > 1 && lds(lanes) > 65536) lanes /= 2;   // within 64 KB of LDS
  const int64_t tiles = (lines + lanes - 1) / lanes;
  const size_t smem = lds(lanes);
  const dim3 g((unsigned)tiles), b((unsigned)(lanes * tl));
  const cx<double>* a = (const cx<double>*)in;
  cx<double>* o = (cx<double>*)out;
  const cx<double>* w = (const cx<double>*)twd;
  switch (n) {
    case 16: hipLaunchKernelGGL(k_prolong_fft<16>, g, b, smem, s, a, o, n0, n1, n2, ax, lanes, w); break;
    case 32: hipLaunchKernelGGL(k_prolong_fft<32>, g, b, smem, s, a, o, n0, n1, n2, ax, lanes, w); break;
    case 64: hipLaunchKernelGGL(k_prolong_fft<64>, g, b, smem, s, a, o, n0, n1, n2, ax, lanes, w); break;
    case 128: hipLaunchKernelGGL(k_prolong_fft<128>, g, b, smem, s, a, o, n0, n1, n2, ax, lanes, w); break;
    case 256: hipLaunchKernelGGL(k_prolong_fft<256>, g, b, smem, s, a, o, n0, n1, n2, ax, lanes, w); break;
    case 512: hipLaunchKernelGGL(k_prolong_fft<512>, g, b, smem, s, a, o, n0, n1, n2, ax, lanes, w); break;
    default: return -1;
  }
  return 0;
}

}  // namespace gpe
