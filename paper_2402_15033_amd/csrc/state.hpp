// Device-resident state of one solve: parameters, cycle control flags and every
// small dense matrix of the method, in one block of device memory (float64).
// Small matrices are column-major with leading dimension kLd = 64.
#pragma once

#include "common.hpp"

namespace tsg {

// Head: read back by the host once per restart cycle (keep it first and small).
struct StateHead {
  int32_t done;          // solve finished: every later kernel returns at entry
  int32_t status;        // 0 converged, 1 max_iters reached, 2 breakdown
  int32_t stop_panel;    // panels with a larger index are skipped in this cycle
  int32_t k_used;        // Krylov vectors kept in the current cycle
  int64_t iters;         // Krylov vectors generated so far (all cycles)
  int64_t cycles;        // restart cycles completed
  double relres;         // explicit relative residual at the last check
  double est;            // implicit relative residual estimate at the end of the last cycle
  int32_t truncated;     // cycles truncated by a Cholesky breakdown
  int32_t refine;        // panel + 1 of the panel whose stage-1 PIP needs the explicit pass
  int32_t fallbacks;     // stage-1 panels that took the explicit second pass (all cycles)
  int32_t newton_from;   // Leja-Ritz basis: cycles completed when it took over (0: not yet)
  int32_t refine2;       // panel + 1 of the panel whose explicit pass needs the shifted pass
  int32_t shifted;       // stage-1 panels that took the shifted Cholesky QR pass (all cycles)
  int32_t redo;          // a cycle run without the fallback passes met a panel that needs them:
                         // the rest of the cycle returned at entry, the host runs it again in full
  int32_t pad4;
};
static_assert(sizeof(StateHead) == 80, "the host reads an 80-byte status head per cycle");

struct SmallState {
  StateHead h;
  // parameters (written by the host at solve start)
  int32_t m, s, ortho, prec;
  int64_t max_iters;
  double tol, bnorm, pivot_tol;
  double pip_tol;        // two-stage stage 1: relative pivot below which the explicit pass runs
  // basis step i: w_{i+1} = ((A - theta_i I) w_i + tau_i w_{i-1}) / sigma_i
  double theta[kMaxS], sigma[kMaxS], tau[kMaxS];
  double glo, ghi;       // Gershgorin interval of the operator
  int32_t ritz_pending;  // Leja-Ritz basis: the next cycle end computes the Newton shifts
  int32_t pad3;
  // cycle scalars
  double beta, inv_beta;
  int32_t identity_t;    // the next update kernel uses T = I (no scaling)
  int32_t fail_col;      // stand-alone: panel column whose pivot failed (-1: none)
  // small matrices
  double Hh[kLd * kLd];    // Hessenberg of the basis, (m+1) x m
  double G2[kLd * kLd];    // stage-2 Gram of the pre-processed basis (upper triangle)
  double Wk[kLd * kLd];    // scratch matrix
  double Pcur[kLd * kMaxS];   // P read by the next update kernel (k x s)
  double Tcur[kMaxS * kMaxS]; // upper-triangular T read by the next update kernel
  double P1[kLd * kMaxS];     // first-pass projection coefficients
  double R1[kMaxS * kMaxS];   // first-pass triangular factor
  double Ra[kMaxS * kMaxS];   // accumulated CholQR factor (BCGS2 + CholQR2)
  double P2[kLd * kMaxS];     // second-pass projection coefficients
  double refW[kMaxS];         // raw Gram diagonal of the panel whose PIP pass failed
  double Rs[kMaxS * kMaxS];   // shifted Cholesky factor of that panel's explicit pass
  // two-stage with big panels (s_hat < m)
  double gscale;              // least-squares rhs: beta M(0,0) once the first big panel is final
  double Bs[kLd * kLd];       // q(:, big panel) = Y(:, :b1) Bs(:b1, big panel): [-P2 T2; T2]
  // Givens state of the one-stage variants and of standard GMRES
  double gc[kLd], gs[kLd], gg[kLd + 1];
  double Rg[kLd * kLd];       // Givens-triangularized Hessenberg
  double coef[kLd];           // x-update coefficients of the current cycle
};

}  // namespace tsg
