// One stand-alone apply pass (role GPE_ROLE, float64 if GPE_FP64) per object file.
#include "gpe_launch.h"
#include "apply_impl.h"

#ifndef GPE_ROLE
#error "GPE_ROLE must be defined"
#endif
#ifndef GPE_FP64
#error "GPE_FP64 must be defined"
#endif
#define GPE_CAT2(a, b, c) a##b##_##c
#define GPE_CAT(a, b, c) GPE_CAT2(a, b, c)

namespace gpe {
using T_ = std::conditional<GPE_FP64 != 0, double, float>::type;
void GPE_CAT(launch_apply_pass_r, GPE_ROLE, GPE_FP64)(hipStream_t s, int nblocks, int threads, size_t smem,
                                                      const ProbDev* probs, const ApplyArgs& a, const void* tw) {
  // the x and y passes do not depend on the kind
  constexpr bool epi = GPE_ROLE == R_FINAL || GPE_ROLE == R_SOLO;
  if (epi && a.kind == 1)
    hipLaunchKernelGGL((k_apply_pass<GPE_ROLE, T_, epi ? 1 : 0>), dim3(nblocks), dim3(threads), smem, s, probs,
                       a, (const cx<T_>*)tw);
  else
    hipLaunchKernelGGL((k_apply_pass<GPE_ROLE, T_, 0>), dim3(nblocks), dim3(threads), smem, s, probs, a,
                       (const cx<T_>*)tw);
}
}  // namespace gpe
