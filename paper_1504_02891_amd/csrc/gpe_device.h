// Device building blocks: complex arithmetic, in-register/LDS Stockham FFT
// for one line per group of threads, FP64 block reductions.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include "gpe_state.h"

namespace gpe {

template <typename T>
struct alignas(2 * sizeof(T)) cx {
  T re, im;
};

// Global-memory access through pointers read from descriptors.  Such
// pointers are generic to the compiler, and generic (flat) accesses wait on
// both the vector-memory and the LDS counters; the cast makes them plain
// global loads and stores that can be issued back to back.
// Complex values move as two-element vectors (one 8- or 16-byte access).
template <typename T> using gptr = __attribute__((address_space(1))) T*;
template <typename T> struct GAccess {
  static __device__ __forceinline__ T load(const void* p, int64_t i) { return ((gptr<const T>)p)[i]; }
  static __device__ __forceinline__ void store(void* p, int64_t i, T v) { ((gptr<T>)p)[i] = v; }
};
template <typename U> struct GAccess<cx<U>> {
  typedef U v2 __attribute__((ext_vector_type(2)));
  static __device__ __forceinline__ cx<U> load(const void* p, int64_t i) {
    const v2 r = ((gptr<const v2>)p)[i];
    return cx<U>{r.x, r.y};
  }
  static __device__ __forceinline__ void store(void* p, int64_t i, cx<U> v) {
    v2 r;
    r.x = v.re;
    r.y = v.im;
    ((gptr<v2>)p)[i] = r;
  }
};
template <typename T> __device__ __forceinline__ T gld(const void* p, int64_t i) { return GAccess<T>::load(p, i); }
template <typename T> __device__ __forceinline__ void gst(void* p, int64_t i, T v) { GAccess<T>::store(p, i, v); }

// Makes the value of `x` available in a scalar register at this point, so
// that the load behind it is issued here and later uses read the register.
// Applied to the descriptor fields a kernel needs, right after reading them,
// it turns a chain of lazily issued scalar loads (one wait per branch that
// first needs a field) into one batch with one wait.  Only for values that
// are uniform across the wavefront.
template <typename T> __device__ __forceinline__ void pin_reg(T& x) {
  static_assert(sizeof(T) == 4 || sizeof(T) == 8, "pin_reg: 32- or 64-bit values");
  if constexpr (sizeof(T) == 4) {
    uint32_t w = __builtin_bit_cast(uint32_t, x);
    asm volatile("" : "+s"(w));
    x = __builtin_bit_cast(T, w);
  } else {
    uint64_t w = __builtin_bit_cast(uint64_t, x);
    asm volatile("" : "+s"(w));
    x = __builtin_bit_cast(T, w);
  }
}

// The value of `x` in the wavefront's first active lane, in a scalar
// register: for values that are uniform but which the compiler cannot prove
// uniform (read from LDS, for instance).
template <typename T> __device__ __forceinline__ void make_uniform(T& x) {
  static_assert(sizeof(T) == 4 || sizeof(T) == 8, "make_uniform: 32- or 64-bit values");
  if constexpr (sizeof(T) == 4) {
    x = __builtin_bit_cast(T, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, x)));
  } else {
    const uint64_t w = __builtin_bit_cast(uint64_t, x);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)w);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(w >> 32));
    x = __builtin_bit_cast(T, ((uint64_t)hi << 32) | lo);
  }
}

// One load per 64-byte line of a struct, all issued together and completed
// here: later reads of any of its fields (issued lazily by the compiler, one
// branch at a time) then hit the cache instead of each waiting on memory.
template <typename T> __device__ __forceinline__ void touch_lines(const T* p) {
  constexpr int L = (int)((sizeof(T) + 63) / 64);
  uint32_t w[L];
#pragma unroll
  for (int i = 0; i < L; ++i) w[i] = ((gptr<const uint32_t>)p)[16 * i];
#pragma unroll
  for (int i = 0; i < L; ++i) asm volatile("" ::"v"(w[i]));
}

// Workgroups go to the chip's 8 XCDs round robin (workgroup b to XCD b % 8),
// each XCD with its own L2.  Renumbered by this bijection of [0, g), XCD x
// works on one contiguous range of tiles: neighbouring tiles of a strided
// pass read the same cache lines (a tile covers only part of a 128-byte
// row), which are then fetched once into that XCD's L2 instead of once into
// every XCD's.
constexpr int kXcd = 8;
__device__ __forceinline__ int xcd_tile(int b, int g) {
  const int x = b % kXcd, i = b / kXcd;
  const int q = g / kXcd, r = g % kXcd;
  return x * q + min(x, r) + i;
}

// Element i of a 2- or 3-array with i known only at run time, by selects, so
// that a local copy of a descriptor is never indexed dynamically (which would
// place it in scratch memory).
template <typename T> __device__ __forceinline__ T sel2(const T* a, int i) { return i ? a[1] : a[0]; }
template <typename T> __device__ __forceinline__ T pick3(const T* a, int i) {
  return i == 0 ? a[0] : (i == 1 ? a[1] : a[2]);
}

template <typename T> __device__ __forceinline__ cx<T> mk(T r, T i) { return cx<T>{r, i}; }
template <typename T> __device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T> __device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T> __device__ __forceinline__ cx<T> operator*(T s, cx<T> a) { return {s * a.re, s * a.im}; }
template <typename T> __device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T> __device__ __forceinline__ cx<T> cmulc(cx<T> a, cx<T> b) {  // a * conj(b)
  return {a.re * b.re + a.im * b.im, a.im * b.re - a.re * b.im};
}
template <typename T> __device__ __forceinline__ T abs2(cx<T> a) { return a.re * a.re + a.im * a.im; }
template <typename T> __device__ __forceinline__ T redot(cx<T> a, cx<T> b) { return a.re * b.re + a.im * b.im; }  // Re(conj(a) b)
template <typename To, typename Ti> __device__ __forceinline__ cx<To> cvt(cx<Ti> a) { return {(To)a.re, (To)a.im}; }

// multiply by -i (forward) or +i (inverse)
template <bool INV, typename T> __device__ __forceinline__ cx<T> rot90(cx<T> a) {
  return INV ? cx<T>{-a.im, a.re} : cx<T>{a.im, -a.re};
}

// ---------------------------------------------------------------------------
// Small DFTs in registers, y_k = sum_n x_n w^{nk}, w = exp(-+ 2 pi i / R).
// ---------------------------------------------------------------------------
template <bool INV, typename T>
__device__ __forceinline__ void dft2(cx<T>& a, cx<T>& b) {
  cx<T> t = a - b;
  a = a + b;
  b = t;
}

template <bool INV, typename T>
__device__ __forceinline__ void dft4(cx<T>& x0, cx<T>& x1, cx<T>& x2, cx<T>& x3) {
  cx<T> a0 = x0 + x2, a1 = x0 - x2, a2 = x1 + x3, a3 = rot90<INV>(x1 - x3);
  x0 = a0 + a2;
  x2 = a0 - a2;
  x1 = a1 + a3;
  x3 = a1 - a3;
}

// multiply by w8^j, w8 = exp(-+ i pi/4)
template <bool INV, typename T>
__device__ __forceinline__ cx<T> tw8(cx<T> a, int j) {
  const T s = (T)0.70710678118654752440;
  switch (j & 7) {
    case 0: return a;
    case 1: return INV ? cx<T>{s * (a.re - a.im), s * (a.re + a.im)} : cx<T>{s * (a.re + a.im), s * (a.im - a.re)};
    case 2: return rot90<INV>(a);
    case 3: return INV ? cx<T>{-s * (a.re + a.im), s * (a.re - a.im)} : cx<T>{s * (a.im - a.re), -s * (a.re + a.im)};
    default: return a;  // not used
  }
}

template <bool INV, typename T>
__device__ __forceinline__ void dft8(cx<T>* v) {
  cx<T> e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
  cx<T> o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
  dft4<INV>(e0, e1, e2, e3);
  dft4<INV>(o0, o1, o2, o3);
  o1 = tw8<INV>(o1, 1);
  o2 = tw8<INV>(o2, 2);
  o3 = tw8<INV>(o3, 3);
  v[0] = e0 + o0; v[4] = e0 - o0;
  v[1] = e1 + o1; v[5] = e1 - o1;
  v[2] = e2 + o2; v[6] = e2 - o2;
  v[3] = e3 + o3; v[7] = e3 - o3;
}

// multiply by w16^j for j in 0..9 (products n2*k1 of the 4x4 split)
template <bool INV, typename T>
__device__ __forceinline__ cx<T> tw16(cx<T> a, int j) {
  // cos/sin of 2 pi j / 16
  const T c1 = (T)0.92387953251128675613, s1 = (T)0.38268343236508977173;
  const T r2 = (T)0.70710678118654752440;
  T c, s;
  switch (j) {
    case 0: return a;
    case 1: c = c1; s = s1; break;
    case 2: c = r2; s = r2; break;
    case 3: c = s1; s = c1; break;
    case 4: return rot90<INV>(a);
    case 6: c = -r2; s = r2; break;
    case 9: c = -c1; s = -s1; break;
    default: c = 1; s = 0; break;  // not used
  }
  // forward: multiply by (c - i s); inverse: (c + i s)
  if (INV) return cx<T>{a.re * c - a.im * s, a.re * s + a.im * c};
  return cx<T>{a.re * c + a.im * s, a.im * c - a.re * s};
}

template <bool INV, typename T>
__device__ __forceinline__ void dft16(cx<T>* v) {
  // n = 4 n1 + n2, k = k1 + 4 k2
  cx<T> z[4][4];
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) {
    cx<T> a = v[n2], b = v[4 + n2], c = v[8 + n2], d = v[12 + n2];
    dft4<INV>(a, b, c, d);
    z[n2][0] = a; z[n2][1] = b; z[n2][2] = c; z[n2][3] = d;
  }
#pragma unroll
  for (int n2 = 1; n2 < 4; ++n2)
#pragma unroll
    for (int k1 = 1; k1 < 4; ++k1) z[n2][k1] = tw16<INV>(z[n2][k1], n2 * k1);
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    cx<T> a = z[0][k1], b = z[1][k1], c = z[2][k1], d = z[3][k1];
    dft4<INV>(a, b, c, d);
    v[k1] = a; v[k1 + 4] = b; v[k1 + 8] = c; v[k1 + 12] = d;
  }
}

template <int R, bool INV, typename T>
__device__ __forceinline__ void dftR(cx<T>* u) {
  if constexpr (R == 2) dft2<INV>(u[0], u[1]);
  else if constexpr (R == 4) dft4<INV>(u[0], u[1], u[2], u[3]);
  else if constexpr (R == 8) dft8<INV>(u);
  else dft16<INV>(u);
}

// ---------------------------------------------------------------------------
// Line FFT plan: N points handled by TL = N/E threads holding E values each
// (E = 8 or 4); thread t holds v[e] = line[t + e*TL] before and after a
// transform.  Radix-E stages, then one stage of the remaining factor; the
// inverse runs the stages in reverse order so that the forward output
// (natural frequency order, register e = frequency t + e*TL) stays in
// registers across the multiplier.  Twiddles come from a per-workgroup LDS
// table tw[m] = exp(-2 pi i m / N), m < N.  E = 4 gives a line twice the
// threads and each thread half the points: shorter per-thread chains where a
// pass is latency bound, one more LDS exchange per transform.
// ---------------------------------------------------------------------------
template <int N, int E> struct Plan;
template <> struct Plan<16, 8>   { static constexpr int NS = 2; static constexpr int R[2] = {8, 2}; };
template <> struct Plan<32, 8>   { static constexpr int NS = 2; static constexpr int R[2] = {8, 4}; };
template <> struct Plan<64, 8>   { static constexpr int NS = 2; static constexpr int R[2] = {8, 8}; };
template <> struct Plan<128, 8>  { static constexpr int NS = 3; static constexpr int R[3] = {8, 8, 2}; };
template <> struct Plan<256, 8>  { static constexpr int NS = 3; static constexpr int R[3] = {8, 8, 4}; };
template <> struct Plan<512, 8>  { static constexpr int NS = 3; static constexpr int R[3] = {8, 8, 8}; };
template <> struct Plan<1024, 8> { static constexpr int NS = 4; static constexpr int R[4] = {8, 8, 8, 2}; };
template <> struct Plan<16, 4>   { static constexpr int NS = 2; static constexpr int R[2] = {4, 4}; };
template <> struct Plan<32, 4>   { static constexpr int NS = 3; static constexpr int R[3] = {4, 4, 2}; };
template <> struct Plan<64, 4>   { static constexpr int NS = 3; static constexpr int R[3] = {4, 4, 4}; };
template <> struct Plan<128, 4>  { static constexpr int NS = 4; static constexpr int R[4] = {4, 4, 4, 2}; };
template <> struct Plan<256, 4>  { static constexpr int NS = 4; static constexpr int R[4] = {4, 4, 4, 4}; };
template <> struct Plan<512, 4>  { static constexpr int NS = 5; static constexpr int R[5] = {4, 4, 4, 4, 2}; };
template <> struct Plan<1024, 4> { static constexpr int NS = 5; static constexpr int R[5] = {4, 4, 4, 4, 4}; };

// LDS addressing of a line element: `lane` is the line inside the tile,
// `pos` the position on the line.  Contiguous tiles store lines one after
// the other (padded one element per 16); strided tiles interleave the lanes
// (lane fastest) to match the coalesced global layout.
struct LdsMap {
  int lanes;       // lines per tile
  bool strided;
  __device__ __forceinline__ int idx(int lane, int pos, int n) const {
    if (strided) return pos * (lanes + 1) + lane;
    int row = n + (n >> 4);
    return lane * row + pos + (pos >> 4);
  }
};
// elements of LDS a tile of `lanes` lines of n points needs (data region)
__host__ __device__ inline int lds_elems(int n, int lanes, bool strided) {
  return strided ? n * (lanes + 1) : lanes * (n + n / 16);
}

template <int N, int E, int R, bool INV, bool LAST, typename T>
__device__ __forceinline__ void stockham_stage(cx<T>* v, int t, int ns, int lane, const LdsMap& mp,
                                               cx<T>* lds, const cx<T>* twl) {
  constexpr int TL = N / E;
  constexpr int B = E / R;  // butterflies per thread
  cx<T> out[E];
#pragma unroll
  for (int i = 0; i < B; ++i) {
    const int j = t + i * TL;
    const int k = j & (ns - 1);
    cx<T> u[R];
#pragma unroll
    for (int r = 0; r < R; ++r) u[r] = v[i + r * B];
    if (ns > 1) {
      const int step = N / (ns * R);
#pragma unroll
      for (int r = 1; r < R; ++r) {
        const cx<T> w = twl[(r * k * step) & (N - 1)];
        u[r] = INV ? cmulc(u[r], w) : cmul(u[r], w);
      }
    }
    dftR<R, INV>(u);
    if constexpr (LAST) {
#pragma unroll
      for (int r = 0; r < R; ++r) out[i + r * B] = u[r];
    } else {
      const int base = (j - k) * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) lds[mp.idx(lane, base + r * ns, N)] = u[r];
    }
  }
  if constexpr (LAST) {
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = out[e];
  } else {
    __syncthreads();
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = lds[mp.idx(lane, t + e * TL, N)];
  }
}

template <int N, int E, bool INV, int S, typename T>
__device__ __forceinline__ void run_stages(cx<T>* v, int t, int ns, int lane, const LdsMap& mp, cx<T>* lds,
                                           const cx<T>* twl) {
  using P = Plan<N, E>;
  if constexpr (S < P::NS) {
    constexpr int R = INV ? P::R[P::NS - 1 - S] : P::R[S];
    constexpr bool LAST = (S == P::NS - 1);
    if constexpr (!LAST) __syncthreads();   // nobody still reads the LDS lines
    stockham_stage<N, E, R, INV, LAST>(v, t, ns, lane, mp, lds, twl);
    run_stages<N, E, INV, S + 1>(v, t, ns * R, lane, mp, lds, twl);
  }
}

// Full line transform; every thread of the workgroup must call it (barriers).
template <int N, int E, bool INV, typename T>
__device__ __forceinline__ void line_fft(cx<T>* v, int t, int lane, const LdsMap& mp, cx<T>* lds,
                                         const cx<T>* twl) {
  run_stages<N, E, INV, 0>(v, t, 1, lane, mp, lds, twl);
}

// Per-workgroup twiddle table exp(-2 pi i m / N) from the 1024-entry table.
// Callers issue it before a barrier that precedes the first stage using it.
// The workgroup has at least N/8 threads (lanes x N/E, E <= 8), so eight
// rounds cover the table.  fetch issues the loads, store writes the LDS table;
// callers put their other loads in between so that all go out together.
template <int N, typename T>
struct TwiddleFetch {
  cx<T> w[8];
  __device__ __forceinline__ void fetch(const cx<T>* tw1024) {
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int m = min((int)(threadIdx.x + k * blockDim.x), N - 1);
      w[k] = gld<cx<T>>(tw1024, m * (kTwN / N));
    }
  }
  __device__ __forceinline__ void store(cx<T>* twl) const {
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int m = threadIdx.x + k * blockDim.x;
      if (m < N) twl[m] = w[k];
    }
  }
};

// ---------------------------------------------------------------------------
// FP64 reductions: within a wavefront by DPP moves, then across the block's waves.
// ---------------------------------------------------------------------------
// Cross-lane move of a double with DPP: lanes of rows outside ROWMASK (and
// lanes whose source is outside the wavefront) receive 0.
template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp_d(double x) {
  return __builtin_amdgcn_update_dpp(0.0, x, CTRL, ROWMASK, 0xf, false);
}
// value of lane 63, in every lane
__device__ __forceinline__ double lane63(double x) {
  const uint64_t b = __builtin_bit_cast(uint64_t, x);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, 63);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), 63);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}
template <int CTRL, int ROWMASK, int K>
__device__ __forceinline__ void dpp_step(double* acc, unsigned maxmask) {
  double u[K];
#pragma unroll
  for (int i = 0; i < K; ++i) u[i] = dpp_d<CTRL, ROWMASK>(acc[i]);
#pragma unroll
  for (int i = 0; i < K; ++i) acc[i] = ((maxmask >> i) & 1u) ? fmax(acc[i], u[i]) : acc[i] + u[i];
}
// Reduction over the 64 lanes of a full wavefront of K values at once (sums,
// or maxima where bit i of `maxmask` is set; maxima of non-negative values).
// Fixed combining order: lane pairs, quads, half rows, rows (mirrored
// partners, so all lanes of a row agree bitwise), then row 0 into row 1 and
// row 2 into row 3, then rows 0-1 into row 3.  The result is broadcast from
// lane 63, so every lane, and every caller reducing the same values, gets
// the same bits.  The steps are VALU moves: no LDS round trip.
template <int K>
__device__ __forceinline__ void wave_reduce_k(double* acc, unsigned maxmask) {
  dpp_step<0xb1, 0xf, K>(acc, maxmask);    // quad_perm [1,0,3,2]
  dpp_step<0x4e, 0xf, K>(acc, maxmask);    // quad_perm [2,3,0,1]
  dpp_step<0x141, 0xf, K>(acc, maxmask);   // row_half_mirror
  dpp_step<0x140, 0xf, K>(acc, maxmask);   // row_mirror
  dpp_step<0x142, 0xa, K>(acc, maxmask);   // row_bcast:15 into rows 1, 3
  dpp_step<0x143, 0xc, K>(acc, maxmask);   // row_bcast:31 into rows 2, 3
#pragma unroll
  for (int i = 0; i < K; ++i) acc[i] = lane63(acc[i]);
}

// K values per lane reduced over one wavefront through LDS (a transpose),
// with the bits of wave_reduce_k: its butterfly is the balanced pairwise tree
// over the lanes in order (pairs, quads, eights, rows, then rows 2-3 and 0-1),
// and every step commutes.  The values are written slot-major, a row of 65
// doubles per slot; lane 4k + q (k < K) sums lanes 16q .. 16q + 15 of slot k
// as that tree, then the quad combines its four row sums (partner xor 1, then
// xor 2).  Lanes 4k .. 4k + 3 return slot k (a max where bit k of `maxmask`
// is set, of non-negative values), the other lanes 0.  `buf` holds K * 65
// doubles of LDS that only the calling wavefront touches.
template <int K>
__device__ __forceinline__ double wave_reduce_lds(const double* acc, unsigned maxmask, double* buf) {
  static_assert(4 * K <= 64, "one quad of lanes per slot");
  const int l = threadIdx.x & 63;
#pragma unroll
  for (int i = 0; i < K; ++i) buf[i * 65 + l] = acc[i];
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  const int k = l >> 2, q = l & 3;
  const bool mx = k < K && ((maxmask >> k) & 1u);
  const double* p = buf + min(k, K - 1) * 65 + 16 * q;
  double v[16];
#pragma unroll
  for (int m = 0; m < 16; ++m) v[m] = p[m];
#pragma unroll
  for (int w = 8; w >= 1; w >>= 1)
#pragma unroll
    for (int m = 0; m < w; ++m) v[m] = mx ? fmax(v[2 * m], v[2 * m + 1]) : v[2 * m] + v[2 * m + 1];
  double s = v[0];
  double u = dpp_d<0xb1, 0xf>(s);   // quad_perm [1,0,3,2]
  s = mx ? fmax(s, u) : s + u;
  u = dpp_d<0x4e, 0xf>(s);          // quad_perm [2,3,0,1]
  s = mx ? fmax(s, u) : s + u;
  return k < K ? s : 0.0;
}

// Partial sums are stored slot-major, part[s * count + i] for slot s of
// workgroup (tile) i, so that reading one slot of consecutive tiles is
// coalesced.
//
// Fixed-order reduction of part[s * count + i] over i < count, for slots
// s < NSLOT (a max where bit s of `maxmask` is set, else a sum), by one
// wavefront: lane l accumulates i = l, l+64, l+128, ... in turn, then the
// lanes are combined by wave_reduce_k.  Loads go out in batches of B per
// lane (indices clamped, the extra values discarded; BB > 0 sets B).  Every
// lane of the calling wavefront gets the result; every caller reducing the
// same partials gets the same bits, whatever B and NSLOT.
template <int NSLOT, int BB = 0>
__device__ __forceinline__ void wave_reduce_partials(const double* part, int count, unsigned maxmask,
                                                     double* acc) {
  constexpr int B = BB > 0 ? BB : (NSLOT <= 4 ? 8 : 4);
  const int l = threadIdx.x & 63;
#pragma unroll
  for (int s = 0; s < NSLOT; ++s) acc[s] = 0.0;
  for (int b0 = 0; b0 < count; b0 += 64 * B) {
    double v[B][NSLOT];
#pragma unroll
    for (int j = 0; j < B; ++j) {
      const int64_t i = min(b0 + l + 64 * j, count - 1);
#pragma unroll
      for (int s = 0; s < NSLOT; ++s) v[j][s] = gld<double>(part, (int64_t)s * count + i);
    }
#pragma unroll
    for (int j = 0; j < B; ++j)
      if (b0 + l + 64 * j < count)
#pragma unroll
        for (int s = 0; s < NSLOT; ++s)
          acc[s] = ((maxmask >> s) & 1u) ? fmax(acc[s], v[j][s]) : acc[s] + v[j][s];
  }
  wave_reduce_k<NSLOT>(acc, maxmask);
}

// Reduce NS sums followed by NM maxima over the block; thread 0 gets results
// in `acc`.  `red` is LDS scratch of at least (NS+NM)*16 doubles.
template <int NS, int NM>
__device__ __forceinline__ void block_reduce(double* acc, double* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  wave_reduce_k<NS + NM>(acc, ((1u << NM) - 1u) << NS);
  __syncthreads();
  if (lane == 0)
#pragma unroll
    for (int i = 0; i < NS + NM; ++i) red[i * 16 + wave] = acc[i];
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < NS + NM; ++i) {
      double s = red[i * 16];
      for (int w = 1; w < nw; ++w) s = (i < NS) ? s + red[i * 16 + w] : fmax(s, red[i * 16 + w]);
      acc[i] = s;
    }
  }
}

}  // namespace gpe
