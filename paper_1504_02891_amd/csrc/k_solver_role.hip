// One solver pass (role GPE_ROLE, precision GPE_PREC64) per object file, so
// the build compiles the pass variants in parallel.
#include <hip/hip_ext.h>
#include "gpe_launch.h"
#include "passes_impl.h"

#ifndef GPE_ROLE
#error "GPE_ROLE must be defined (0 first, 1 mid, 2 final, 3 solo)"
#endif
#ifndef GPE_PREC64
#error "GPE_PREC64 must be defined (0 or 1)"
#endif
#define GPE_CAT2(a, b, c) a##b##_##c
#define GPE_CAT(a, b, c) GPE_CAT2(a, b, c)

namespace gpe {
template <bool RR, bool FUSED, int EPT, bool PAIR>
static void launch_e(hipStream_t s, int nblocks, int threads, size_t smem, const ProbDev* probs, SolverState* st_in,
                     SolverState* st_out, const int2* bmap, const void* twd, const void* twf, int par, hipEvent_t ev0,
                     hipEvent_t ev1) {
  if (ev0) {
    // events stamped by the dispatch itself (start and end of this kernel)
    hipExtLaunchKernelGGL((k_solver_pass<GPE_ROLE, (GPE_PREC64 != 0), RR, FUSED, EPT, PAIR>), dim3(nblocks),
                          dim3(threads), smem, s, ev0, ev1, 0, probs, st_in, st_out, bmap, (const cx<double>*)twd,
                          (const cx<float>*)twf, par);
  } else {
    hipLaunchKernelGGL((k_solver_pass<GPE_ROLE, (GPE_PREC64 != 0), RR, FUSED, EPT, PAIR>), dim3(nblocks),
                       dim3(threads), smem, s, probs, st_in, st_out, bmap, (const cx<double>*)twd,
                       (const cx<float>*)twf, par);
  }
}
// the 1D pass never pairs lines
template <bool RR, bool FUSED, int EPT>
static void launch_p(hipStream_t s, int nblocks, int threads, size_t smem, const ProbDev* probs, SolverState* st_in,
                     SolverState* st_out, const int2* bmap, const void* twd, const void* twf, int par, hipEvent_t ev0,
                     hipEvent_t ev1, int pair) {
  if (GPE_ROLE != R_SOLO && pair)
    launch_e<RR, FUSED, EPT, GPE_ROLE != R_SOLO>(s, nblocks, threads, smem, probs, st_in, st_out, bmap, twd, twf,
                                                 par, ev0, ev1);
  else launch_e<RR, FUSED, EPT, false>(s, nblocks, threads, smem, probs, st_in, st_out, bmap, twd, twf, par, ev0, ev1);
}
template <bool RR, bool FUSED>
static void launch(hipStream_t s, int nblocks, int threads, size_t smem, const ProbDev* probs, SolverState* st_in,
                   SolverState* st_out, const int2* bmap, const void* twd, const void* twf, int par, hipEvent_t ev0,
                   hipEvent_t ev1, int ept, int pair) {
  if (ept == 4)
    launch_p<RR, FUSED, 4>(s, nblocks, threads, smem, probs, st_in, st_out, bmap, twd, twf, par, ev0, ev1, pair);
  else launch_p<RR, FUSED, kE>(s, nblocks, threads, smem, probs, st_in, st_out, bmap, twd, twf, par, ev0, ev1, pair);
}
void GPE_CAT(launch_solver_pass_r, GPE_ROLE, GPE_PREC64)(hipStream_t s, int nblocks, int threads, size_t smem,
                                                         const ProbDev* probs, SolverState* st_in,
                                                         SolverState* st_out, const int2* bmap, const void* twd,
                                                         const void* twf, int par, hipEvent_t ev0, hipEvent_t ev1,
                                                         int reread, int fused, int ept, int pair) {
  constexpr bool epi = GPE_ROLE == R_FINAL || GPE_ROLE == R_SOLO;
  constexpr bool first = GPE_ROLE == R_FIRST;
  if (epi && reread)
    launch<epi, false>(s, nblocks, threads, smem, probs, st_in, st_out, bmap, twd, twf, par, ev0, ev1, ept, pair);
  else if (first && fused)
    launch<false, first>(s, nblocks, threads, smem, probs, st_in, st_out, bmap, twd, twf, par, ev0, ev1, ept, pair);
  else launch<false, false>(s, nblocks, threads, smem, probs, st_in, st_out, bmap, twd, twf, par, ev0, ev1, ept, pair);
}
}  // namespace gpe
