// H(phi) phi and the Newton-model Hessian-vector product as stand-alone
// launch sequences (x pass, [y pass], last pass), sharing the line transforms
// of the solver passes.
#pragma once
#include "passes_impl.h"

namespace gpe {

template <int N, int ROLE, typename T>
__device__ __forceinline__ void apply_tile(const ProbDev& P, const ApplyArgs& A, int tile, cx<T>* lds,
                                           const cx<T>* tw1024, double* red) {
  constexpr int E = Tile<N>::E;
  constexpr bool HAS_T = (ROLE == R_MID || ROLE == R_FINAL);
  const int ax = role_axis(ROLE, P.dim);
  constexpr bool EPI = (ROLE == R_FINAL || ROLE == R_SOLO);
  const Tile<N> Tl(P, ax, HAS_T, tile);
  TwiddleFetch<N, T> twf;
  twf.fetch(tw1024);
  // one batch of loads: input, accumulator, potential, X_k (Hessian-vector)
  cx<T> u[E], tv[E], v[E];
  cx<double> xk[E];
  double vp[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    u[e] = ld<T>(A.in, Tl.g(e));
    if constexpr (HAS_T) tv[e] = ld<T>(P.t, Tl.g(e));
    if constexpr (EPI) xk[e] = A.kind == 1 ? ld<double>(A.xk, Tl.g(e)) : cx<double>{0.0, 0.0};
    v[e] = cvt<T>(Tl.sgn(e) * cvt<double>(u[e]));
  }
  if constexpr (EPI) Tl.pot_load(P, vp);
  twf.store(lds);
  spectral_apply<N, T>(P, ax, Tl, v, lds);
  if constexpr (ROLE == R_FIRST) {
#pragma unroll
    for (int e = 0; e < E; ++e)
      if (Tl.inner(e)) stc<T>(P.t, Tl.g(e), v[e]);
  } else if constexpr (ROLE == R_MID) {
#pragma unroll
    for (int e = 0; e < E; ++e)
      if (Tl.inner(e)) stc<T>(P.t, Tl.g(e), tv[e] + v[e]);
  } else {
    double acc[SA_COUNT] = {};
#pragma unroll
    for (int e = 0; e < E; ++e)
      if (Tl.inner(e)) {
        const int64_t g = Tl.g(e);
        cx<double> kin = cvt<double>(v[e]);
        if constexpr (HAS_T) kin = kin + cvt<double>(tv[e]);
        const cx<double> uu = cvt<double>(u[e]);
        const double vg = Tl.pot_value(P, vp[e]);
        const double q = abs2(uu);
        if (A.kind == 0) {
          const cx<double> h = kin + vg * uu + (P.beta * q) * uu;
          stc<T>(A.out, g, cvt<T>(h));
          acc[SA_KIN] += redot(uu, kin);
          acc[SA_POT] += vg * q;
          acc[SA_QUART] += q * q;
          acc[SA_NORM] += q;
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            if (a >= P.dim) break;
            const int ca = a == 0 ? Tl.c0 : (a == 1 ? Tl.c1 : Tl.c2);
            const int ia = a == ax ? Tl.idx(e) : ca;
            const double xa = P.x0[a] + P.h[a] * (double)ia;   // a is a compile-time index here
            acc[SA_X2 + a] += xa * xa * q;
          }
          acc[SA_MAXD] = fmax(acc[SA_MAXD], q);
        } else {
          const cx<double> x0 = xk[e];
          const cx<double> hs = 2.0 * (kin + vg * uu) +
                                (4.0 * P.alpha) * (abs2(x0) * uu + (2.0 * redot(x0, uu)) * x0) + A.delta * uu;
          stc<T>(A.out, g, cvt<T>(hs));
        }
      }
    block_reduce<SA_COUNT_SUM, 1>(acc, red);
    if (threadIdx.x == 0) {
      const int64_t nt = pick3(P.tiles, P.dim - 1);
#pragma unroll
      for (int i = 0; i < SA_COUNT; ++i) gst<double>(P.partF, i * nt + tile, acc[i]);
    }
  }
}

template <int ROLE, typename T>
__global__ void __launch_bounds__(256) k_apply_pass(const ProbDev* __restrict__ probs, ApplyArgs A,
                                                    const cx<T>* __restrict__ tw) {
  extern __shared__ __align__(16) char smem[];
  __shared__ double red[SA_COUNT * 16];
  const ProbDev P = probs[0];     // local copy: one batch of loads
  const int tile = xcd_tile((int)blockIdx.x, (int)gridDim.x);
  const int n = pick3(P.nl, role_axis(ROLE, P.dim));
  cx<T>* lds = reinterpret_cast<cx<T>*>(smem);
  switch (n) {
    case 16: apply_tile<16, ROLE, T>(P, A, tile, lds, tw, red); break;
    case 32: apply_tile<32, ROLE, T>(P, A, tile, lds, tw, red); break;
    case 64: apply_tile<64, ROLE, T>(P, A, tile, lds, tw, red); break;
    case 128: apply_tile<128, ROLE, T>(P, A, tile, lds, tw, red); break;
    case 256: apply_tile<256, ROLE, T>(P, A, tile, lds, tw, red); break;
    case 512: apply_tile<512, ROLE, T>(P, A, tile, lds, tw, red); break;
    case 1024: apply_tile<1024, ROLE, T>(P, A, tile, lds, tw, red); break;
    default: break;
  }
}

}  // namespace gpe
