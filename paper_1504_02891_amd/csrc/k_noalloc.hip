// Fixed scratch of gpe_apply_h_noalloc, the entry point for callers that
// cannot allocate device memory (code under stream capture, tight serving
// loops): a file-scope device array holds the descriptor, the potential
// tables, the partial sums and the pass accumulator of one H(phi)phi call.
// Each GPU keeps its own copy of the array until the process ends; every
// call on a GPU reuses it, so calls that overlap on one GPU race.
#include <hip/hip_runtime.h>
#include <cmath>
#include <mutex>
#include "gpe_launch.h"

namespace gpe {

static __device__ __align__(256) char scratch[kNoAllocBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
char* g_ptr[kMaxDevices] = {};   // device address of each device's copy of `scratch`
}  // namespace

int noalloc_init(int device) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (device < 0 || device >= kMaxDevices) return (int)hipErrorInvalidDevice;
  if (g_ptr[device]) return 0;
  // the caller made `device` current: the address is that device's copy
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) return e != hipSuccess ? (int)e : (int)hipErrorInvalidSymbol;
  g_ptr[device] = (char*)p;
  return 0;
}

char* noalloc_scratch(int device) {
  std::lock_guard<std::mutex> lk(g_mu);
  return (device >= 0 && device < kMaxDevices) ? g_ptr[device] : nullptr;
}

// The descriptor (passed by value) into device memory, and the separable
// potential tables V_i(x_j) = 1/2 gamma_i^2 x_j^2 + A sin^2(k x_j) for
// j < n_i on the problem's axes (zero elsewhere), computed on the device.
__global__ void __launch_bounds__(256) k_setup_desc(ProbDev d, VAxisParams vp, ProbDev* __restrict__ dst,
                                                    double* __restrict__ vaxis) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *dst = d;
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < 3 * kMaxN; idx += gridDim.x * blockDim.x) {
    const int i = idx / kMaxN, j = idx % kMaxN;
    double v = 0.0;
    if (i < d.dim && j < d.n[i]) {
      const double x = grid_coord(d, i, j);
      const double s = sin(vp.k * x);
      v = 0.5 * vp.gamma[i] * vp.gamma[i] * x * x + vp.amp * s * s;
    }
    vaxis[idx] = v;
  }
}

void launch_setup_desc(hipStream_t s, const ProbDev& d, const VAxisParams& vp, ProbDev* dst, double* vaxis) {
  hipLaunchKernelGGL(k_setup_desc, dim3(12), dim3(256), 0, s, d, vp, dst, vaxis);
}

}  // namespace gpe
