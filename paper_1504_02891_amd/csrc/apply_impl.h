// H(phi) phi and the Newton-model Hessian-vector product as stand-alone
// launch sequences (x pass, [y pass], last pass), sharing the line transforms
// of the solver passes.
#pragma once
#include "passes_impl.h"


namespace gpe {

// KIND 0: H(phi) phi with the energy sums; KIND 1: Hessian-vector product.
// Only the epilogue roles (FINAL, SOLO) depend on KIND.
template <int N, int E, int ROLE, typename T, int KIND>
__device__ __forceinline__ void apply_tile(const ProbDev& P, const ApplyArgs& A, int tile, cx<T>* lds,
                                           const cx<T>* tw1024, double* red) {
  constexpr bool HAS_T = (ROLE == R_MID || ROLE == R_FINAL);
  const int ax = role_axis(ROLE, P.dim);
  constexpr bool EPI = (ROLE == R_FINAL || ROLE == R_SOLO);
  constexpr bool HESS = EPI && KIND == 1;
  const Tile<N, E> Tl(P, ax, HAS_T, tile);
  TwiddleFetch<N, T> twf;
  twf.fetch(tw1024);
  // loads: the input first; the accumulator, X_k (Hessian-vector) and the
  // potential of the epilogue roles after the inverse transform, which keeps
  // them out of the registers live through the transforms (256^3, last pass:
  // float32 four waves per SIMD, float64 three; measured 103 vs 164 us and
  // 182 vs 211 us against loading them with the input)
  constexpr int LOADS_AT = EPI ? 2 : 0;
  cx<T> u[E], tv[E], v[E];
  cx<double> xk[HESS ? E : 1];
  double vp[E];
  auto late_loads = [&]() {
#pragma unroll
    for (int e = 0; e < E; ++e) {
      if constexpr (HAS_T) tv[e] = ld<T>(P.t, Tl.g(e));
      if constexpr (HESS) xk[e] = ld<double>(A.xk, Tl.g(e));
    }
    if constexpr (EPI) Tl.pot_load(P, vp);
  };
#pragma unroll
  for (int e = 0; e < E; ++e) u[e] = ld<T>(A.in, Tl.g(e));
  if (Tl.sine || Tl.fd) {   // odd extension: signs +1, -1 and zeros; FD: the boundary zero
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = (T)Tl.sgn(e) * u[e];
  } else {
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = u[e];
  }
  if constexpr (LOADS_AT == 0) late_loads();
  twf.store(lds);
  spectral_forward<N, E, T>(P, ax, Tl, v, lds);
  spectral_inverse<N, E, T>(Tl, v, lds);
  if constexpr (LOADS_AT == 2) late_loads();
  if constexpr (ROLE == R_FIRST) {
#pragma unroll
    for (int e = 0; e < E; ++e)
      if (Tl.inner(e)) stc<T>(P.t, Tl.g(e), v[e]);
  } else if constexpr (ROLE == R_MID) {
#pragma unroll
    for (int e = 0; e < E; ++e)
      if (Tl.inner(e)) stc<T>(P.t, Tl.g(e), tv[e] + v[e]);
  } else if constexpr (HESS) {
#pragma unroll
    for (int e = 0; e < E; ++e)
      if (Tl.inner(e)) {
        cx<double> kin = cvt<double>(v[e]);
        if constexpr (HAS_T) kin = kin + cvt<double>(tv[e]);
        const cx<double> uu = cvt<double>(u[e]);
        const double vg = Tl.pot_value(P, vp[e]);
        const cx<double> x0 = xk[e];
        const cx<double> hs = 2.0 * (kin + vg * uu) +
                              (4.0 * P.alpha) * (abs2(x0) * uu + (2.0 * redot(x0, uu)) * x0) + A.delta * uu;
        stc<T>(A.out, Tl.g(e), cvt<T>(hs));
      }
  } else {
    // H(phi) phi pointwise in the pass precision; the products entering
    // mu = h_vol sum Re(conj(phi) H phi), sum |phi|^4 and sum V |phi|^2
    // accumulate in FP64 (the other scalars come from the residual pass)
    double acc[SA_COUNT] = {};
#pragma unroll
    for (int e = 0; e < E; ++e)
      if (Tl.inner(e)) {
        cx<T> kin = v[e];
        if constexpr (HAS_T) kin = kin + tv[e];
        const cx<T> uu = u[e];
        const T vg = (T)Tl.pot_value(P, vp[e]);
        const T q = uu.re * uu.re + uu.im * uu.im;
        const cx<T> h = kin + (vg + (T)P.beta * q) * uu;
        stc<T>(A.out, Tl.g(e), h);
        acc[SA_MU] += (double)(uu.re * h.re + uu.im * h.im);
        acc[SA_QUART] += (double)(q * q);
        acc[SA_POT] += (double)(vg * q);
      }
    // one partial per wavefront (no workgroup barrier): entry tile * nw + wave
    wave_reduce_k<SA_COUNT>(acc, 0u);
    if ((threadIdx.x & 63) == 0) {
      const int nw = blockDim.x >> 6;
      const int64_t cnt = (int64_t)pick3(P.tiles, P.dim - 1) * nw;
      const int64_t at = (int64_t)tile * nw + (threadIdx.x >> 6);
#pragma unroll
      for (int i = 0; i < SA_COUNT; ++i) gst<double>(P.partF, i * cnt + at, acc[i]);
    }
  }
}

template <int ROLE, typename T, int KIND>
__global__ void __launch_bounds__(256) k_apply_pass(const ProbDev* __restrict__ probs, ApplyArgs A,
                                                    const cx<T>* __restrict__ tw) {
  extern __shared__ __align__(16) char smem[];
  __shared__ double red[SA_COUNT * 16];
  const ProbDev P = probs[0];     // local copy: one batch of loads
  const int tile = xcd_tile((int)blockIdx.x, (int)gridDim.x);
  // the stand-alone passes take kE (8) points per thread
  const int n = pick3(P.nl, role_axis(ROLE, P.dim));
  cx<T>* lds = reinterpret_cast<cx<T>*>(smem);
#define GPE_APPLY_CASE(NN)                                                      \
  case NN:                                                                      \
    apply_tile<NN, kE, ROLE, T, KIND>(P, A, tile, lds, tw, red);                \
    break;
  switch (n) {
    GPE_APPLY_CASE(16) GPE_APPLY_CASE(32) GPE_APPLY_CASE(64) GPE_APPLY_CASE(128)
    GPE_APPLY_CASE(256) GPE_APPLY_CASE(512) GPE_APPLY_CASE(1024)
    default: break;
  }
#undef GPE_APPLY_CASE
}

}  // namespace gpe
