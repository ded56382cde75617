// Scalar control of the solver, run by one thread of the last workgroup of
// an evaluation's final pass (float64): the nonmonotone BB line search of
// Algorithm 1 (§3.1) and the trust-region ratio / regularisation update of
// Algorithm 2 (§3.2).
#pragma once
#include "gpe_device.h"

namespace gpe {

__device__ __forceinline__ void set_trial(SolverState& S) {
  // Theorem 3.3 coefficients for the curve through the base point.
  const double t = S.t, a = S.a_b, n = S.n_b, ng = S.ng_b;
  const double den = 1.0 - t * t * a * a + t * t * n * ng;
  S.p = ((1.0 + t * a) * (1.0 + t * a) - t * t * n * ng) / den;
  S.q = -2.0 * t * n / den;
  S.pm1 = 2.0 * t * (a + t * a * a - t * n * ng) / den;
  S.mode = (S.phase == PH_INNER) ? M_W : M_F;
}

__device__ __forceinline__ void finish(SolverState& S, int status, int src) {
  S.phase = PH_DONE;
  S.mode = M_IDLE;
  S.status = status;
  S.src = src;
  S.done = 1;
}

__device__ __forceinline__ void end_alg1(SolverState& S, bool stopped) {
  if (S.alg == 1) {
    finish(S, stopped ? 0 : 1, SRC_XF);
    return;
  }
  S.tau_last = S.tau_bb;
  S.phase = PH_OUTER;
  S.mode = M_OUTER;
  S.src = SRC_XF;
  S.force_norm = 0;
}

__device__ __forceinline__ void end_inner(SolverState& S) {
  const double pred = S.k > 0 ? S.pred_acc : 0.0;
  const double rho = pred < 0.0 ? S.ared_acc / pred : -INFINITY;
  const bool acc = rho >= S.eta1;
  if (!acc) S.rejections++;
  if (rho > S.eta2) S.delta *= S.gshrink;
  else if (rho < S.eta1) S.delta *= S.ggrow;
  S.delta = fmin(fmax(S.delta, S.delta_min), S.delta_max);
  S.outer++;
  S.tau_last = S.tau_bb;
  S.phase = PH_OUTER;
  S.mode = M_OUTER;
  S.src = acc ? SRC_XK_PLUS_S : SRC_XK;
  S.force_norm = acc ? 1 : 0;
}

__device__ __forceinline__ void step_logic(const ProbDev& P, SolverState& S, const double* r1, const double* rf,
                                  int prec64) {
  S.nfe++;
  if (prec64 || S.mode == M_OUTER) S.nfe64++;
  if (S.mode == M_F) S.nfe_f++;
  else if (S.mode == M_W) S.nfe_w++;
  else S.nfe_o++;
  const double ny_pre = r1[S1_NY];
  const double c = (S.force_norm || fabs(ny_pre - 1.0) > S.renorm_tol) ? 1.0 / sqrt(ny_pre) : 1.0;
  const double n_hat = c * c * ny_pre;
  if (S.phase == PH_INIT && ny_pre == 0.0) {   // zero initial data
    finish(S, -1, SRC_XF);
    return;
  }
  if (!isfinite(ny_pre) || !isfinite(rf[SF_F]) || !isfinite(rf[SF_NG]) || !isfinite(rf[SF_A]) ||
      !isfinite(r1[S1_NP2]) || !(ny_pre > 0.0)) {
    finish(S, -5, S.phase == PH_ALG1 || S.phase == PH_INIT ? SRC_XF : SRC_XK);
    return;
  }
  const double rscale = 1.0 / (2.0 * P.sqrt_hvol);

  if (S.phase == PH_INIT) {
    S.f_b = rf[SF_F]; S.a_b = rf[SF_A]; S.n_b = rf[SF_NY]; S.ng_b = rf[SF_NG];
    S.cur ^= 1;
    S.C = S.f_b; S.Q = 1.0;
    S.k = 0; S.m = 0;
    S.tau_bb = S.tau0;
    S.force_norm = 0;
    S.phase = PH_ALG1;
    S.maxit = (S.alg == 1) ? S.max_iter : S.k_init;
    if (S.maxit <= 0 && S.alg != 1) { end_alg1(S, false); return; }
    S.t = 0.5 * S.tau_bb;
    set_trial(S);
    return;
  }
  if (S.phase == PH_OUTER) {
    // crit2 on an accepted Newton step: max |X_{k+1} - X_k| from this evaluation
    if (S.stop_rule == STOP_CRIT2 && S.src == SRC_XK_PLUS_S && sqrt(rf[SF_SMAX]) <= S.crit2_tol) {
      finish(S, 0, SRC_XK);
      return;
    }
    S.f_outer = rf[SF_F];
    S.a_b = rf[SF_A]; S.n_b = rf[SF_NY]; S.ng_b = rf[SF_NG]; S.f_b = 0.0;
    S.k = 0; S.m = 0; S.C = 0.0; S.Q = 1.0;
    S.tau_bb = S.tau_last;
    S.cur = 0;
    S.force_norm = 0;
    S.phase = PH_INNER;
    S.maxit = S.k_sub;
    S.t = 0.5 * S.tau_bb;
    set_trial(S);
    return;
  }
  // PH_ALG1 / PH_INNER: a trial from the current base was evaluated.
  if (S.m == 0) {
    S.np2_b = r1[S1_NP2];
    const double rb = sqrt(r1[S1_RMAX]) * rscale;   // residual of the base point (phi units)
    if (S.phase == PH_ALG1) {
      const bool resid_rule = S.stop_rule == STOP_RESID || (S.alg == 2 && S.stop_rule == STOP_CRIT2);
      if (resid_rule && rb < S.tol) {
        // an FP32 residual carries the transforms' rounding: mixed-precision
        // Algorithm 1 hands its iterate to the FP64 continuation, which tests
        // (and if needed refines) it in FP64
        if (!prec64 && S.alg == 1 && S.switch_window > 0) { finish(S, kStatusStalled, SRC_XF); return; }
        end_alg1(S, true);
        return;
      }
      if (!prec64 && S.alg == 1 && S.switch_window > 0) {
        // FP32 floor: no halving of the best residual within the window
        if (rb < 0.5 * S.best_r) {
          S.best_r = rb;
          S.since_best = 0;
        } else if (++S.since_best >= S.switch_window) {
          finish(S, kStatusStalled, SRC_XF);
          return;
        }
      }
    } else {
      if (S.k == 0) {
        S.r_outer = rb;
        if (S.stop_rule != STOP_CRIT2 && rb < S.tol) { finish(S, 0, SRC_XK); return; }
        // mixed precision: X_k (FP64) continues in an FP64 run once its
        // residual reaches the handover level
        if (!prec64 && rb < S.switch_r) { finish(S, kStatusStalled, SRC_XK); return; }
        if (S.outer >= S.max_outer) { finish(S, 1, SRC_XK); return; }
        const double npk = sqrt(S.np2_b);
        S.forcing = fmin(0.1, npk) * npk;
      }
      if (sqrt(S.np2_b) <= S.forcing) { end_inner(S); return; }
    }
  }
  const bool pass = rf[SF_F] <= S.C - S.rho1 * S.t * S.np2_b;
  if (pass || S.m >= S.m_max) {
    const double ny = rf[SF_NY];
    const double dn = ny - n_hat, da = rf[SF_A] - S.a_b;
    S.ss = rf[SF_SS];
    S.sw = rf[SF_SW0] + dn * rf[SF_SG] - da * rf[SF_SY];
    S.ww = rf[SF_W0W0] + dn * dn * rf[SF_NG] + da * da * ny + 2.0 * dn * rf[SF_W0G] -
           2.0 * da * rf[SF_W0Y] - 2.0 * dn * da * rf[SF_A];
    S.f_b = rf[SF_F]; S.a_b = rf[SF_A]; S.n_b = ny; S.ng_b = rf[SF_NG];
    if (S.phase == PH_INNER) { S.pred_acc = rf[SF_F]; S.ared_acc = rf[SF_ARED]; }
    S.cur ^= 1;
    const double qn = S.eta * S.Q + 1.0;
    S.C = (S.eta * S.Q * S.C + S.f_b) / qn;
    S.Q = qn;
    S.k++; S.inner_total++; S.m = 0;
    if (S.phase == PH_ALG1 &&
        (S.stop_rule == STOP_CRIT1 || (S.alg == 1 && S.stop_rule == STOP_CRIT2))) {
      // step-length rules on the accepted step of length t (max |S_j|^2 of this trial)
      const double dx = sqrt(rf[SF_SMAX]);
      if (S.stop_rule == STOP_CRIT1 ? dx <= S.eps0 * S.t : dx <= S.crit2_tol) {
        end_alg1(S, true);
        return;
      }
    }
    if (S.k >= S.maxit) {
      if (S.phase == PH_ALG1) end_alg1(S, false);
      else end_inner(S);
      return;
    }
    const double sw = fabs(S.sw);
    if (sw > 0.0) S.tau_bb = (S.k & 1) ? S.ss / sw : sw / S.ww;
    S.tau_bb = fmin(fmax(S.tau_bb, 1e-20), 1e20);
    S.t = 0.5 * S.tau_bb;
  } else {
    S.m++;
    S.backtracks++;
    S.t *= S.sigma;
  }
  set_trial(S);
}

}  // namespace gpe
