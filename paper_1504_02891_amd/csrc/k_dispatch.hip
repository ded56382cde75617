// Dispatch of the pass launchers by role and precision.
#include "gpe_launch.h"

namespace gpe {
#define GPE_DECL_SOLVER(r, p)                                                                              \
  void launch_solver_pass_r##r##_##p(hipStream_t, int, int, size_t, const ProbDev*, SolverState*, SolverState*, \
                                     const int2*, const void*, const void*, int, hipEvent_t, hipEvent_t, int, int, \
                                     int, int);
#define GPE_DECL_APPLY(r, p) \
  void launch_apply_pass_r##r##_##p(hipStream_t, int, int, size_t, const ProbDev*, const ApplyArgs&, const void*);
GPE_DECL_SOLVER(0, 0) GPE_DECL_SOLVER(1, 0) GPE_DECL_SOLVER(2, 0) GPE_DECL_SOLVER(3, 0)
GPE_DECL_SOLVER(0, 1) GPE_DECL_SOLVER(1, 1) GPE_DECL_SOLVER(2, 1) GPE_DECL_SOLVER(3, 1)
GPE_DECL_APPLY(0, 0) GPE_DECL_APPLY(1, 0) GPE_DECL_APPLY(2, 0) GPE_DECL_APPLY(3, 0)
GPE_DECL_APPLY(0, 1) GPE_DECL_APPLY(1, 1) GPE_DECL_APPLY(2, 1) GPE_DECL_APPLY(3, 1)

void launch_solver_pass(hipStream_t s, int role, int prec64, int nb, int th, size_t sm, const ProbDev* p,
                        SolverState* st_in, SolverState* st_out, const int2* bm, const void* twd, const void* twf,
                        int par, hipEvent_t ev0, hipEvent_t ev1, int reread, int fused, int ept, int pair) {
  typedef void (*F)(hipStream_t, int, int, size_t, const ProbDev*, SolverState*, SolverState*, const int2*,
                    const void*, const void*, int, hipEvent_t, hipEvent_t, int, int, int, int);
  static const F tab[2][4] = {
      {launch_solver_pass_r0_0, launch_solver_pass_r1_0, launch_solver_pass_r2_0, launch_solver_pass_r3_0},
      {launch_solver_pass_r0_1, launch_solver_pass_r1_1, launch_solver_pass_r2_1, launch_solver_pass_r3_1}};
  tab[prec64 ? 1 : 0][role & 3](s, nb, th, sm, p, st_in, st_out, bm, twd, twf, par, ev0, ev1, reread, fused, ept,
                                pair);
}
void launch_apply_pass(hipStream_t s, int role, int fp64, int nb, int th, size_t sm, const ProbDev* p,
                       const ApplyArgs& a, const void* tw) {
  typedef void (*F)(hipStream_t, int, int, size_t, const ProbDev*, const ApplyArgs&, const void*);
  static const F tab[2][4] = {
      {launch_apply_pass_r0_0, launch_apply_pass_r1_0, launch_apply_pass_r2_0, launch_apply_pass_r3_0},
      {launch_apply_pass_r0_1, launch_apply_pass_r1_1, launch_apply_pass_r2_1, launch_apply_pass_r3_1}};
  tab[fp64 ? 1 : 0][role & 3](s, nb, th, sm, p, a, tw);
}
}  // namespace gpe
