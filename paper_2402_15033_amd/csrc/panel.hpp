// Panel steps of every block orthogonalization scheme (Sec. IV-V): the arguments shared
// by the streaming kernels (GramBody, FusedBody, UpdateBody), and the
// one-block FP64 "tail" that follows a reduction.
//
// A streaming launch passes once over the rows of the column-major basis V and, per row r,
// forms some of
//     y  = W(r,:) - Q(r,:) P          (PF_HAS_P; else y = W(r,:))
//     q  = y T                        (PF_HAS_T, T upper triangular; else q = y)
//     W(r,:) <- q                     (PF_STORE, in place)
//     G += [Q(r,:), q]^T q            (PF_GRAM_Q: Q rows, PF_GRAM_W: q rows)
// where Q = V(:, 0:k) and W = V(:, wcol:wcol+sw).  Each block writes its partial Gram;
// PTailBody sums the partials in a fixed order and runs the tail (Cholesky of the
// Pythagorean Gram, Hessenberg block, Givens, ...).
#pragma once

#include "small.hpp"

namespace tsg {

enum PanelFlags : int {
  PF_HAS_P = 1,
  PF_HAS_T = 2,
  PF_STORE = 4,
  PF_GRAM_Q = 8,
  PF_GRAM_W = 16,
  PF_BMAT = 32,  // fused kernel: q = Y(:, staged) Bs(staged, wcol:wcol+sw) (big-panel stage 2)
};

enum TailOp : int {
  TAIL_NONE = 0,
  TAIL_NORM0,      // two-stage: G2(0,0) <- q0^T q0
  TAIL_SA_NORM,    // stand-alone: r00 = ||x0||, T = 1/r00
  TAIL_PIP,        // BCGS-PIP Cholesky; two-stage stage 1 (+ Hessenberg block)
  TAIL_PIP_FB,     // two-stage stage 1: explicit second pass after a failed PIP pivot
  TAIL_PIP_FB2,    // two-stage stage 1: pass after the shifted Cholesky QR
  TAIL_G2COL,      // two-stage: block column of the stage-2 Gram
  TAIL_PIP2_A,     // BCGS-PIP2 first pass
  TAIL_PIP2_B,     // BCGS-PIP2 second pass (+ Hessenberg block, Givens)
  TAIL_BC_P1,      // BCGS2 + CholQR2: P1 = Q^T W
  TAIL_BC_A1,      // ... Ra1 = Chol(Vhat^T Vhat)
  TAIL_BC_A2,      // ... Ra2 = Chol(Qt1^T Qt1), Ra = Ra2 Ra1
  TAIL_BC_P2,      // ... P2 = Q^T Qt
  TAIL_BC_C,       // ... Rc = Chol(Y^T Y) (+ Hessenberg block, Givens)
  TAIL_CGS_H1,     // standard GMRES, CGS2 first pass
  TAIL_CGS_H2,     // standard GMRES, CGS2 second pass (+ Hessenberg column, Givens)
  TAIL_GRAM_OUT,   // copy the reduced Gram into st->Wk (orthogonality check)
};

struct PanelArgs {
  void* V;
  int64_t ld;
  int64_t n;
  int64_t rows_per_block;
  int32_t k;         // Q = V(:, 0:k)
  int32_t wcol;      // W = V(:, wcol : wcol+sw)
  int32_t sw;        // panel width (<= template S)
  int32_t flags;
  int32_t tail;
  int32_t nblocks;
  int32_t gate;      // 1: return at entry when the solve is done or panel > stop_panel;
                     // 2: also unless this panel asked for the explicit second pass;
                     // 3: also unless it asked for the pass after the shifted Cholesky QR
  int32_t standalone;// 0: solver; 1: stand-alone (tails assemble an R factor in st->Hh
                     // instead of Hessenberg/Givens; any failed pivot is a breakdown);
                     // 2: stand-alone with stage 1's fallback chain (a failed PIP pivot
                     // takes the explicit pass, as in the solver)
  int32_t kkeep;     // Krylov vectors kept if this panel breaks down (solver mode)
  int32_t panel;     // index of the panel within the cycle (-1: cycle set-up)
  int32_t nz;        // reduced Gram has nz columns: nz - sw previous-panel columns, then W
  int32_t shifted;   // the cycle holds the gate-3 pass: a failed explicit pass shifts
  int32_t fast;      // the cycle holds no fallback pass: a failed PIP pivot asks for a redo
  SmallState* st;
  double* part1;     // per-block partial Grams, nblocks x (k+sw)*sw
};


__device__ __forceinline__ bool gated_off(const PanelArgs& a, const SmallState* st_) {
  if (!a.gate) return false;
  gbl<const SmallState>* st = G(st_);
  if (st->h.done || a.panel > st->h.stop_panel) return true;
  if (a.gate == 2) return st->h.refine != a.panel + 1;
  return a.gate == 3 && st->h.refine2 != a.panel + 1;
}
// gated_off in two halves: the flags' loads (issued early), then the decision.
struct GateFlags {
  int32_t done, stop_panel, refine, refine2;
};
__device__ __forceinline__ GateFlags gate_flags(const SmallState* st_) {
  gbl<const SmallState>* st = G(st_);
  return GateFlags{st->h.done, st->h.stop_panel, st->h.refine, st->h.refine2};
}
__device__ __forceinline__ bool gated_off(const PanelArgs& a, const GateFlags& f) {
  if (!a.gate) return false;
  if (f.done || a.panel > f.stop_panel) return true;
  if (a.gate == 2) return f.refine != a.panel + 1;
  return a.gate == 3 && f.refine2 != a.panel + 1;
}

// ----------------------------------------------------------------------------- tails
// Called by every thread of the tail block with the reduced Gram sred ((k+sw) x nz, entry
// (c, z) at sred[c * nz + z]); its last sw columns belong to the panel W:
// red(c, j) = sred[c * nz + (nz - sw) + j].
__device__ __forceinline__ double red(const PanelArgs& a, const double* sred, int c, int j) {
  return sred[c * a.nz + (a.nz - a.sw) + j];
}

__device__ __forceinline__ void tail_breakdown(const PanelArgs& a, int kkeep, int f = -1) {
  SmallState* st = a.st;
  if (threadIdx.x == 0) {
    if (a.standalone) {
      st->h.status = 2;
      st->h.done = 1;
      st->fail_col = f;
    } else {  // this panel is discarded: stop after the previous one
      st->h.stop_panel = a.panel - 1;
      st->h.k_used = kkeep;
      st->h.truncated += 1;
    }
  }
  __syncthreads();
}

// Convergence check of the one-stage variants after Hessenberg columns 0..ncols-1:
// the current panel still completes, later panels of the cycle are skipped.
__device__ void tail_check(SmallState* st, int ncols, int panel) {
  if (threadIdx.x == 0) {
    double est = fabs(st->gg[ncols]);
    if (est <= st->tol * st->bnorm && ncols < st->m) {
      st->h.stop_panel = panel;
      st->h.k_used = ncols;
    }
  }
  __syncthreads();
}

// Pythagorean Gram G = Gw - P^T P (P = sred rows 0..k-1, Gw = rows k..k+s-1) and its
// Cholesky factor into R (ld kMaxS).  A pivot fails when it is at most tol * Gw_jj, or, for
// the explicit second pass (second = true, the panel holds Y = W - Q P1), at most
// max(tol * Gw_jj, pivot_tol^2 * refW_j) with refW the raw Gram diagonal of W.
// Returns the failing pivot or -1.
__device__ __forceinline__ int tail_pip_chol(const PanelArgs& a, const double* sred, double* P, double* R, double tol,
                             bool second = false) {
  const int k = a.k, s = a.sw, tid = threadIdx.x, nt = blockDim.x;
  __shared__ double sG[kMaxS * kMaxS], sRef[kMaxS];
  for (int idx = tid; idx < k * s; idx += nt) {
    int c = idx % k, j = idx / k;
    P[c + j * kLd] = red(a, sred, c, j);
  }
  for (int idx = tid; idx < s * s; idx += nt) {
    int i = idx % s, j = idx / s;
    // P^T P entry in four interleaved partial sums (independent LDS loads and FMAs)
    double p0 = 0.0, p1 = 0.0, p2 = 0.0, p3 = 0.0;
    int c = 0;
    for (; c + 3 < k; c += 4) {
      p0 += red(a, sred, c, i) * red(a, sred, c, j);
      p1 += red(a, sred, c + 1, i) * red(a, sred, c + 1, j);
      p2 += red(a, sred, c + 2, i) * red(a, sred, c + 2, j);
      p3 += red(a, sred, c + 3, i) * red(a, sred, c + 3, j);
    }
    for (; c < k; ++c) p0 += red(a, sred, c, i) * red(a, sred, c, j);
    const double v = red(a, sred, k + i, j) - ((p0 + p1) + (p2 + p3));
    sG[i + j * kMaxS] = v;
    if (i == j) {
      const double d = red(a, sred, k + i, j);
      const double pt = a.st->pivot_tol;
      sRef[i] = second ? fmax(tol * d, pt * pt * a.st->refW[i]) : tol * d;
    }
  }
  __syncthreads();
  return small_chol_upper(sG, kMaxS, R, kMaxS, s, sRef, 1.0);
}

// Shifted Cholesky QR (Fukaya et al. 2020) of the explicit pass's panel: with that pass's
// Pythagorean Gram G, Rs = Chol(G + mu I), mu = 10 pivot_tol trace(G) -- well above the
// Gram's rounding level, so G + mu I is positive definite and (Y - Q P2) Rs^{-1} is well
// conditioned.  Returns the failing pivot or -1.
__device__ __forceinline__ int tail_shifted_chol(const PanelArgs& a, const double* sred, double* Rs) {
  const int k = a.k, s = a.sw, tid = threadIdx.x, nt = blockDim.x;
  __shared__ double sG[kMaxS * kMaxS];
  __shared__ double s_mu;
  for (int idx = tid; idx < s * s; idx += nt) {
    int i = idx % s, j = idx / s;
    double v = red(a, sred, k + i, j);
    for (int c = 0; c < k; ++c) v -= red(a, sred, c, i) * red(a, sred, c, j);
    sG[i + j * kMaxS] = v;
  }
  __syncthreads();
  if (tid == 0) {
    double tr = 0.0;
    for (int j = 0; j < s; ++j) tr += sG[j + j * kMaxS];
    s_mu = 10.0 * a.st->pivot_tol * tr;
  }
  __syncthreads();
  for (int j = tid; j < s; j += nt) sG[j + j * kMaxS] += s_mu;
  __syncthreads();
  return block_chol_upper(sG, kMaxS, Rs, kMaxS, s, nullptr, 0.0);
}

// Plain Cholesky of rows r0..r0+s-1 of sred (a q^T q Gram) into R (ld kMaxS).
__device__ __forceinline__ int tail_chol_rows(const PanelArgs& a, const double* sred, int r0, double* R, double tol) {
  const int s = a.sw, tid = threadIdx.x, nt = blockDim.x;
  __shared__ double sG[kMaxS * kMaxS];
  for (int idx = tid; idx < s * s; idx += nt) {
    int i = idx % s, j = idx / s;
    sG[i + j * kMaxS] = red(a, sred, r0 + i, j);
  }
  __syncthreads();
  return block_chol_upper(sG, kMaxS, R, kMaxS, s, nullptr, tol);
}

// Write T = R^{-1} (s x s) for the next update kernel.
__device__ void tail_set_tinv(SmallState* st, const double* R, int s) {
  // in LDS (R copied first), then one store of T
  __shared__ double lR[kMaxS * kMaxS], lX[kMaxS * kMaxS];
  const int tid = threadIdx.x;
  if (tid < s * s) lR[tid % s + (tid / s) * kMaxS] = R[tid % s + (tid / s) * kMaxS];
  __syncthreads();
  block_tri_inv_upper(lR, kMaxS, lX, kMaxS, s);
  if (tid < s * s) st->Tcur[tid % s + (tid / s) * kMaxS] = lX[tid % s + (tid / s) * kMaxS];
  if (tid == 0) st->identity_t = 0;
  __syncthreads();
}

// The panel's final factors (P, R): V_panel = Q P + Q_new R.  Solver mode: Hessenberg
// block, and (one-stage) Givens + convergence check.  Stand-alone: R factor assembly.
__device__ __forceinline__ void tail_emit_panel(const PanelArgs& a, const double* P, const double* R, bool givens,
                                const double* lH) {
  SmallState* st = a.st;
  const int k = a.k, s = a.sw, tid = threadIdx.x, nt = blockDim.x;
  const int c0 = a.wcol;
  if (a.standalone) {
    for (int idx = tid; idx < (k + s) * s; idx += nt) {
      int i = idx % (k + s), j = idx / (k + s);
      double v = (i < k) ? P[i + j * kLd] : ((i - k) <= j ? R[(i - k) + j * kMaxS] : 0.0);
      st->Hh[(i < k ? i : c0 + i - k) + (c0 + j) * kLd] = v;
    }
    __syncthreads();
    return;
  }
  block_hessenberg_panel(lH, st->Hh, P, R, st->theta, st->sigma, st->tau, k, s);
  if (givens) {
    givens_append(st, st->Hh, k - 1, k - 1 + s);
    tail_check(st, k - 1 + s, a.panel);
  }
}

// Stage-1 PIP tail of a panel of compile-time width S (the solver's and the stand-alone
// orthogonalization's common step size), the same operations in the same order per entry as
// tail_pip_chol, tail_set_tinv and block_hessenberg_panel, spread over the waves of the tail:
//   wave 0        G(i,j) = Gw(i,j) - P^T P (four interleaved partial sums), the row-oriented
//                 Cholesky (d_j = G_jj - sum_{i<j} R_ij^2, R_jc = (G_jc - sum_{i<j} R_ij R_ic)
//                 / R_jj) and X = R^{-1} by columns, in registers: lane c holds column c of
//                 G, R and X, and row j of R reaches every lane by wave broadcasts as soon as
//                 step j has formed it (the running sums of the later steps take their terms
//                 then); R to LDS, T = X to st->Tcur;
//   waves 1..S-1  solver: column c = wave of M = S B - [H S; 0] for the rows i < k (lane i),
//                 which need P, H and the basis parameters only;
//   the others    P to st->Pcur for the next update.
// Straight-line code (S fixed): no branch waits on a load.  tail_pip_regs ends with a barrier
// and returns the failing pivot or -1; on success tail_pip_regs_emit forms the rows
// k .. k+S-1 of M, solves with T = S(k-1 .. k+S-2, 0 .. S-1) and stores the new Hessenberg
// columns (solver), or writes P and R into the R factor (stand-alone).
template <int S>
__device__ __forceinline__ int tail_pip_regs(const PanelArgs& a, const double* sred, const double* lH,
                                             const double* lB, double* sR, double* lM) {
  static_assert(S >= 1 && S * S <= kWave && S <= kTailThreads / kWave - 1, "one wave per Hessenberg column");
  SmallState* st = a.st;
  const int k = a.k, nz = a.nz, tid = threadIdx.x, wave = tid / kWave, lane = tid % kWave;
  const double* pw = sred + (nz - S);  // P(r, j) = pw[r * nz + j], Gw(i, j) = pw[(k + i) * nz + j]
  __shared__ int s_fail;
  if (wave == 0) {
    double gv = 0.0;
    if (lane < S * S) {
      const int i = lane % S, j = lane / S;
      double p0 = 0.0, p1 = 0.0, p2 = 0.0, p3 = 0.0;
      int c = 0;
      for (; c + 3 < k; c += 4) {
        p0 += pw[c * nz + i] * pw[c * nz + j];
        p1 += pw[(c + 1) * nz + i] * pw[(c + 1) * nz + j];
        p2 += pw[(c + 2) * nz + i] * pw[(c + 2) * nz + j];
        p3 += pw[(c + 3) * nz + i] * pw[(c + 3) * nz + j];
      }
      for (; c < k; ++c) p0 += pw[c * nz + i] * pw[c * nz + j];
      gv = pw[(k + i) * nz + j] - ((p0 + p1) + (p2 + p3));
    }
    // v[j]: G(j, lane) - sum_{i < step} R(i, j) R(i, lane); d[j]: the running pivot of row j.
    // Every step runs (a failed pivot only records its index; nothing is used then).
    double v[S], d[S], r[S];
#pragma unroll
    for (int j = 0; j < S; ++j) {
      v[j] = __shfl(gv, (j + lane * S) & (kWave - 1), kWave);
      d[j] = wave_bcast(gv, j + j * S);
      r[j] = 0.0;
    }
    const double tol = st->pip_tol;
    int fail = -1;
#pragma unroll
    for (int j = 0; j < S; ++j) {
      const double ref = tol * pw[(k + j) * nz + j];
      if (!(d[j] > 1.0 * ref) && fail < 0) fail = j;
      const double rjj = sqrt(d[j]);
      const double rjc = v[j] / rjj;  // R(j, lane) for lanes past j
      r[j] = lane == j ? rjj : (lane > j ? rjc : 0.0);
#pragma unroll
      for (int jp = j + 1; jp < S; ++jp) {
        const double rj = wave_bcast(rjc, jp);  // R(j, jp)
        d[jp] -= rj * rj;
        v[jp] -= rj * rjc;
      }
    }
    if (lane < S) {
#pragma unroll
      for (int i = 0; i < S; ++i) sR[i + lane * kMaxS] = r[i];
    }
    if (fail < 0) {
      // column `lane` of X: X(i,c) = ([i == c] - sum_{l=i+1..c} R(i,l) X(l,c)) / R(i,i); the
      // terms l > c are R(i,l) * 0 and leave the sum as it is
      double x[S];
#pragma unroll
      for (int i = S - 1; i >= 0; --i) {
        double w = (i == lane) ? 1.0 : 0.0;
#pragma unroll
        for (int l = i + 1; l < S; ++l) w -= wave_bcast(r[i], l) * x[l];
        x[i] = w / wave_bcast(r[i], i);
      }
      if (lane < S) {
#pragma unroll
        for (int i = 0; i < S; ++i) st->Tcur[i + lane * kMaxS] = x[i];
      }
      if (lane == 0) st->identity_t = 0;
    }
    if (lane == 0) s_fail = fail;
  } else if (wave < S) {
    if (!a.standalone && lane < k) {
      const int c = wave, i = lane;
      // S(i, l) for i < k: l = 0 -> [i == k-1]; l >= 1 -> P(i, l-1)
      const double sc = pw[i * nz + c - 1], sc1 = c + 1 <= S ? pw[i * nz + c] : 0.0;
      const double scm = c - 1 == 0 ? (i == k - 1 ? 1.0 : 0.0) : pw[i * nz + c - 2];
      double w = sc * lB[c] + sc1 * lB[kMaxS + c];
      if (lB[2 * kMaxS + c] != 0.0) w -= scm * lB[2 * kMaxS + c];
      const double* pc = pw + (c - 1);
#pragma unroll 4
      for (int l = (i > 0 ? i - 1 : 0); l < k - 1; ++l) w -= lH[i + l * kLd] * pc[l * nz];
      lM[i + c * kLd] = w;
    }
  } else {
    for (int idx = tid - S * kWave; idx < k * S; idx += blockDim.x - S * kWave) {
      const int c = idx % k, j = idx / k;
      st->Pcur[c + j * kLd] = pw[c * nz + j];
    }
  }
  __syncthreads();
  return s_fail;
}

template <int S>
__device__ __forceinline__ void tail_pip_regs_emit(const PanelArgs& a, const double* sred, const double* sR,
                                                   const double* lB, const double* lM) {
  SmallState* st = a.st;
  const int k = a.k, nz = a.nz, tid = threadIdx.x;
  const double* pw = sred + (nz - S);
  if (a.standalone) {
    const int c0 = a.wcol;
    for (int idx = tid; idx < (k + S) * S; idx += blockDim.x) {
      const int i = idx % (k + S), j = idx / (k + S);
      const double v = (i < k) ? pw[i * nz + j] : ((i - k) <= j ? sR[(i - k) + j * kMaxS] : 0.0);
      st->Hh[(i < k ? i : c0 + i - k) + (c0 + j) * kLd] = v;
    }
    return;
  }
  const int i = tid - kWave;  // wave 1, lane i: row i
  if (i < 0 || i >= k + S) return;
  double m[S];
  if (i < k) {
    // column 0: S(i,0) theta_0 + S(i,1) sigma_0
    m[0] = (i == k - 1 ? 1.0 : 0.0) * lB[0] + pw[i * nz] * lB[kMaxS];
#pragma unroll
    for (int c = 1; c < S; ++c) m[c] = lM[i + c * kLd];
  } else {
    // S(i, l) for i >= k: l = 0 -> 0; l >= 1 -> R(i-k, l-1)
    double Srow[S + 1];
    Srow[0] = 0.0;
#pragma unroll
    for (int l = 1; l <= S; ++l) Srow[l] = sR[(i - k) + (l - 1) * kMaxS];
#pragma unroll
    for (int c = 0; c < S; ++c) {
      double w = Srow[c] * lB[c] + Srow[c + 1] * lB[kMaxS + c];
      if (c >= 1 && lB[2 * kMaxS + c] != 0.0) w -= Srow[c - 1] * lB[2 * kMaxS + c];
      m[c] = w;
    }
  }
  // T(0,0) = 1, T(q,0) = 0, T(0,c) = P(k-1,c-1), T(q,c) = R(q-1,c-1)
  double x[S];
  x[0] = m[0] / 1.0;
#pragma unroll
  for (int c = 1; c < S; ++c) {
    double w = m[c];
    w -= x[0] * pw[(k - 1) * nz + c - 1];
#pragma unroll
    for (int q = 1; q < c; ++q) w -= x[q] * sR[(q - 1) + (c - 1) * kMaxS];
    x[c] = w / sR[(c - 1) + (c - 1) * kMaxS];
  }
#pragma unroll
  for (int c = 0; c < S; ++c) st->Hh[i + (k - 1 + c) * kLd] = x[c];
}

__device__ __forceinline__ void panel_tail(const PanelArgs& a, const double* sred, const double* lH, const double* lB) {
  SmallState* st = a.st;
  const int k = a.k, s = a.sw, tid = threadIdx.x, nt = blockDim.x;
  __shared__ double sR[kMaxS * kMaxS], sR2[kMaxS * kMaxS], sP[kLd * kMaxS];
  switch (a.tail) {
    case TAIL_NORM0: {
      if (tid == 0) st->G2[0] = red(a, sred, 0, 0);
      __syncthreads();
    } break;
    case TAIL_SA_NORM: {
      if (tid == 0) {
        double r = sqrt(red(a, sred, 0, 0));
        if (!(r > 0.0)) {
          st->h.status = 2;
          st->h.done = 1;
        } else {
          st->Tcur[0] = 1.0 / r;
          st->identity_t = 0;
          st->Hh[0] = r;
        }
      }
      __syncthreads();
    } break;
    case TAIL_PIP: {
      // the previous panel's block column of the stage-2 Gram (nz - s leading columns of
      // the reduction: [Qhat(:, 0:k)]^T Qhat(:, k-np:k)), written before this panel's
      // Cholesky so that it survives a breakdown of this panel (read by later kernels only)
      const int np = a.nz - s;
      for (int idx = tid; idx < k * np; idx += nt) {
        int c = idx % k, z = idx / k;
        int col = k - np + z;
        if (c <= col) st->G2[c + col * kLd] = sred[c * a.nz + z];
      }
      // (panels of the common width 5 take the register form)
      const bool regs = s == 5;
      const int f = regs ? tail_pip_regs<5>(a, sred, lH, lB, sR, sP)
                         : tail_pip_chol(a, sred, st->Pcur, sR, st->pip_tol);
      if (f >= 0) {
        if (a.standalone == 1) { tail_breakdown(a, a.kkeep, f); break; }
        if (a.fast) {
          // this cycle's program has no fallback pass: every later kernel of the cycle returns
          // at entry (x is not touched before the cycle's last kernel) and the host runs the
          // cycle again with the full program
          if (tid == 0) {
            st->h.redo = 1;
            st->h.stop_panel = -2;
          }
          __syncthreads();
          break;
        }
        // The Pythagorean Gram has cancelled to rounding: apply the projection
        // explicitly (the next update computes Y = W - Q P1 with T = I) and let the
        // gated second pass orthogonalize Y.
        for (int idx = tid; idx < k * s; idx += nt) {
          int c = idx % k, j = idx / k;
          st->P1[c + j * kLd] = red(a, sred, c, j);
        }
        for (int j = tid; j < s; j += nt) st->refW[j] = red(a, sred, k + j, j);
        if (tid == 0) {
          st->identity_t = 1;
          st->h.refine = a.panel + 1;
          st->h.fallbacks += 1;
        }
        __syncthreads();
        break;
      }
      if (regs) {
        tail_pip_regs_emit<5>(a, sred, sR, lB, sP);
        break;
      }
      tail_set_tinv(st, sR, s);
      for (int idx = tid; idx < k * s; idx += nt) {  // P from the reduction, in LDS
        int c = idx % k, j = idx / k;
        sP[c + j * kLd] = red(a, sred, c, j);
      }
      __syncthreads();
      tail_emit_panel(a, sP, sR, false, lH);
    } break;
    case TAIL_PIP_FB: {
      // second pass on the panel Y = W - Q P1: P2 = Q^T Y, R = Chol(Y^T Y - P2^T P2);
      // V_panel = Q (P1 + P2) + Q_new R
      int f = tail_pip_chol(a, sred, st->Pcur, sR, st->pivot_tol, true);
      if (f >= 0 && a.shifted) {
        // Y is beyond Cholesky QR: the update forms Z = (Y - Q P2) Rs^{-1} with the shifted
        // factor, and the gated pass after it orthogonalizes Z (P1 accumulates P2)
        const int fs = tail_shifted_chol(a, sred, st->Rs);
        if (fs >= 0) { tail_breakdown(a, a.kkeep, fs); break; }
        for (int idx = tid; idx < k * s; idx += nt) {
          int c = idx % k, j = idx / k;
          st->P1[c + j * kLd] += st->Pcur[c + j * kLd];
        }
        tail_set_tinv(st, st->Rs, s);
        if (tid == 0) {
          st->h.refine2 = a.panel + 1;
          st->h.shifted += 1;
        }
        __syncthreads();
        break;
      }
      if (f >= 0) { tail_breakdown(a, a.kkeep, f); break; }
      tail_set_tinv(st, sR, s);
      for (int idx = tid; idx < k * s; idx += nt) {
        int c = idx % k, j = idx / k;
        sP[c + j * kLd] = st->P1[c + j * kLd] + st->Pcur[c + j * kLd];
      }
      __syncthreads();
      tail_emit_panel(a, sP, sR, false, lH);
    } break;
    case TAIL_PIP_FB2: {
      // pass on Z = (Y - Q P2) Rs^{-1}: P3 = Q^T Z, R3 = Chol(Z^T Z - P3^T P3);
      // V_panel = Q (P1 + P2 + P3 Rs) + Q_new (R3 Rs).  A final pivot (R3 Rs)_jj^2 at most
      // pivot_tol^2 refW_j is a column numerically in span(Q): breakdown.
      __shared__ int s_dep;
      int f = tail_pip_chol(a, sred, st->Pcur, sR, st->pivot_tol);
      if (f < 0) {
        for (int idx = tid; idx < s * s; idx += nt) {
          int i = idx % s, j = idx / s;
          double v = 0.0;
          for (int l = i; l <= j; ++l) v += sR[i + l * kMaxS] * st->Rs[l + j * kMaxS];
          sR2[i + j * kMaxS] = (i <= j) ? v : 0.0;
        }
        __syncthreads();
        if (tid == 0) {
          const double tol = st->pivot_tol;
          int dep = -1;
          for (int j = s - 1; j >= 0; --j) {
            const double d = sR2[j + j * kMaxS];
            if (!(d * d > tol * tol * st->refW[j])) dep = j;
          }
          s_dep = dep;
        }
        __syncthreads();
        f = s_dep;
      }
      if (f >= 0) { tail_breakdown(a, a.kkeep, f); break; }
      tail_set_tinv(st, sR, s);
      for (int idx = tid; idx < k * s; idx += nt) {
        int c = idx % k, j = idx / k;
        double v = st->P1[c + j * kLd];
        for (int l = 0; l <= j; ++l) v += st->Pcur[c + l * kLd] * st->Rs[l + j * kMaxS];
        sP[c + j * kLd] = v;
      }
      __syncthreads();
      tail_emit_panel(a, sP, sR2, false, lH);
    } break;
    case TAIL_G2COL: {
      for (int idx = tid; idx < (k + s) * s; idx += nt) {
        int c = idx % (k + s), j = idx / (k + s);
        int row = (c < k) ? c : a.wcol + (c - k);
        int col = a.wcol + j;
        if (row <= col) st->G2[row + col * kLd] = red(a, sred, c, j);
      }
      __syncthreads();
    } break;
    case TAIL_PIP2_A: {
      int f = tail_pip_chol(a, sred, st->Pcur, st->R1, st->pivot_tol);
      if (f >= 0) { tail_breakdown(a, a.kkeep, f); break; }
      for (int idx = tid; idx < k * s; idx += nt) {
        int c = idx % k, j = idx / k;
        st->P1[c + j * kLd] = st->Pcur[c + j * kLd];
      }
      __syncthreads();
      tail_set_tinv(st, st->R1, s);
    } break;
    case TAIL_PIP2_B: {
      int f = tail_pip_chol(a, sred, st->Pcur, sR2, st->pivot_tol);
      if (f >= 0) { tail_breakdown(a, a.kkeep, f); break; }
      tail_set_tinv(st, sR2, s);
      // P = P1 + P2 R1,  R = R2 R1
      for (int idx = tid; idx < k * s; idx += nt) {
        int c = idx % k, j = idx / k;
        double v = st->P1[c + j * kLd];
        for (int l = 0; l <= j; ++l) v += st->Pcur[c + l * kLd] * st->R1[l + j * kMaxS];
        sP[c + j * kLd] = v;
      }
      for (int idx = tid; idx < s * s; idx += nt) {
        int i = idx % s, j = idx / s;
        double v = 0.0;
        for (int l = i; l <= j; ++l) v += sR2[i + l * kMaxS] * st->R1[l + j * kMaxS];
        sR[i + j * kMaxS] = (i <= j) ? v : 0.0;
      }
      __syncthreads();
      tail_emit_panel(a, sP, sR, true, lH);
    } break;
    case TAIL_BC_P1: {
      for (int idx = tid; idx < k * s; idx += nt) {
        int c = idx % k, j = idx / k;
        st->Pcur[c + j * kLd] = red(a, sred, c, j);
        st->P1[c + j * kLd] = red(a, sred, c, j);
      }
      if (tid == 0) st->identity_t = 1;
      __syncthreads();
    } break;
    case TAIL_BC_A1: {
      int f = tail_chol_rows(a, sred, k, st->Ra, st->pivot_tol);
      if (f >= 0) { tail_breakdown(a, a.kkeep, f); break; }
      tail_set_tinv(st, st->Ra, s);
    } break;
    case TAIL_BC_A2: {
      // this launch has k = 0 (the panel alone)
      int f = tail_chol_rows(a, sred, 0, sR, st->pivot_tol);
      if (f >= 0) { tail_breakdown(a, a.kkeep, f); break; }
      tail_set_tinv(st, sR, s);
      for (int idx = tid; idx < s * s; idx += nt) {
        int i = idx % s, j = idx / s;
        double v = 0.0;
        for (int l = i; l <= j; ++l) v += sR[i + l * kMaxS] * st->Ra[l + j * kMaxS];
        sR2[i + j * kMaxS] = (i <= j) ? v : 0.0;
      }
      __syncthreads();
      for (int idx = tid; idx < s * s; idx += nt) st->Ra[idx % s + (idx / s) * kMaxS] = sR2[idx % s + (idx / s) * kMaxS];
      __syncthreads();
    } break;
    case TAIL_BC_P2: {
      for (int idx = tid; idx < k * s; idx += nt) {
        int c = idx % k, j = idx / k;
        st->Pcur[c + j * kLd] = red(a, sred, c, j);
        st->P2[c + j * kLd] = red(a, sred, c, j);
      }
      if (tid == 0) st->identity_t = 1;
      __syncthreads();
    } break;
    case TAIL_BC_C: {
      int f = tail_chol_rows(a, sred, k, sR2, st->pivot_tol);
      if (f >= 0) { tail_breakdown(a, a.kkeep, f); break; }
      tail_set_tinv(st, sR2, s);
      // P = P1 + P2 Ra,  R = Rc Ra
      for (int idx = tid; idx < k * s; idx += nt) {
        int c = idx % k, j = idx / k;
        double v = st->P1[c + j * kLd];
        for (int l = 0; l <= j; ++l) v += st->P2[c + l * kLd] * st->Ra[l + j * kMaxS];
        sP[c + j * kLd] = v;
      }
      for (int idx = tid; idx < s * s; idx += nt) {
        int i = idx % s, j = idx / s;
        double v = 0.0;
        for (int l = i; l <= j; ++l) v += sR2[i + l * kMaxS] * st->Ra[l + j * kMaxS];
        sR[i + j * kMaxS] = (i <= j) ? v : 0.0;
      }
      __syncthreads();
      tail_emit_panel(a, sP, sR, true, lH);
    } break;
    case TAIL_CGS_H1: {
      for (int c = tid; c < k; c += nt) {
        st->Pcur[c] = red(a, sred, c, 0);
        st->P1[c] = red(a, sred, c, 0);
      }
      if (tid == 0) st->identity_t = 1;
      __syncthreads();
    } break;
    case TAIL_CGS_H2: {
      // h2 = sred(0:k), ||w1||^2 = sred(k); beta^2 = ||w1||^2 - ||h2||^2 (Pythagorean)
      const int j = k - 1;  // Hessenberg column of this iteration
      for (int c = tid; c < k; c += nt) {
        st->Pcur[c] = red(a, sred, c, 0);
        st->Hh[c + j * kLd] = st->P1[c] + red(a, sred, c, 0);
      }
      __syncthreads();
      if (tid == 0) {
        double nw = red(a, sred, k, 0), h2 = 0.0;
        for (int c = 0; c < k; ++c) h2 += red(a, sred, c, 0) * red(a, sred, c, 0);
        double b2 = nw - h2;
        double beta = (b2 > st->pivot_tol * nw) ? sqrt(b2) : 0.0;
        st->Hh[k + j * kLd] = beta;
        st->Wk[0] = beta;
        if (beta > 0.0) {
          st->Tcur[0] = 1.0 / beta;
          st->identity_t = 0;
        }
      }
      __syncthreads();
      givens_append(st, st->Hh, j, j + 1);
      if (tid == 0) {
        double est = fabs(st->gg[k]);
        bool stop = (st->Wk[0] == 0.0) || (est <= st->tol * st->bnorm);
        if (stop && k < st->m) {
          st->h.stop_panel = a.panel;
          st->h.k_used = k;
        }
      }
      __syncthreads();
    } break;
    case TAIL_GRAM_OUT: {
      for (int idx = tid; idx < (k + s) * s; idx += nt) {
        int c = idx % (k + s), j = idx / (k + s);
        int row = (c < k) ? c : a.wcol + (c - k);
        st->Wk[row + (a.wcol + j) * kLd] = red(a, sred, c, j);
      }
      __syncthreads();
    } break;
    default:
      break;
  }
}

// First level of a cross-block reduction with many blocks: block g sums the partials of
// blocks [g*chunk, min(nblocks, (g+1)*chunk)) in block order, for every entry, into
// part2[g * E + e].  The tail then sums the few group partials in group order.
struct RedArgs {
  PanelArgs a;
  double* part2;
  int32_t chunk;
  int32_t pad;
};
struct PReduceBody {
  typedef RedArgs Args;
  static constexpr int kThreads = 256;
  static constexpr int kMinWaves = 1;
  static __device__ void run(const RedArgs& ra, int bid, int) {
    const PanelArgs& a = ra.a;
    const SmallState* st = Gp(a.st);
    if (gated_off(a, st)) return;
    const int E = (a.k + a.sw) * a.nz;
    const int b0 = bid * ra.chunk, b1 = min(a.nblocks, b0 + ra.chunk);
    for (int e = threadIdx.x; e < E; e += blockDim.x)
      ra.part2[(size_t)bid * E + e] = b1 > b0 ? sum_strided(a.part1 + (size_t)b0 * E + e, E, b1 - b0) : 0.0;
  }
};

// The reduction of a panel launch: one block sums the per-block partial Grams in a fixed
// order and runs the FP64 tail (Cholesky, Hessenberg block, Givens, ...).
struct PTailBody {
  typedef PanelArgs Args;
  static constexpr int kThreads = kTailThreads;
  static constexpr int kMinWaves = 1;
  static __device__ __forceinline__ void run(const PanelArgs& a, int bid, int nb);
};
// (Forced inline, like the tail it runs: as a called function its argument block and LDS
// arrays would be reached through generic pointers, the block kept in scratch memory.)
__device__ __forceinline__ void PTailBody::run(const PanelArgs& a_, int, int) {
  PanelArgs a = wave_uniform(a_);  // (scalar registers: the partials' loads need the vector ones)
  a.st = Gp(a.st);  // (device memory: global, not flat, accesses in every helper)
  SmallState* st = a.st;
  __shared__ double sred[kMaxCols * kMaxNz];
  __shared__ double scratch[kTailThreads];
  __shared__ double lH[kLd * kLd];
  __shared__ double lB[3 * kMaxS];
  // Every load this tail needs goes out before the gate check, which then waits for memory
  // together with them: the gate's flags, for a solver tail H and the basis parameters of its
  // Hessenberg block, and the partial Grams (allocated whether or not this panel runs).
  const GateFlags gf = gate_flags(st);
  HessPrefetch pf;
  double bp = 0.0;
  if (!a.standalone) {
    hessenberg_prefetch(st->Hh, a.k, pf);
    if (threadIdx.x < 3 * kMaxS) bp = G(&st->theta[0])[threadIdx.x];  // theta, sigma, tau
  }
  const int E = (a.k + a.sw) * a.nz;
  PartialLoads pl;
  const bool pre = partials_load(a.part1, E, a.nblocks, pl);
  // (keeps the loads above the gate check: the compiler would otherwise sink them past it, to
  // the only path that uses them)
  __asm__ volatile("" ::: "memory");
  if (gated_off(a, gf)) return;
  if (!a.standalone) {
    hessenberg_store(pf, lH);
    if (threadIdx.x < 3 * kMaxS) lB[threadIdx.x] = bp;
  }
  // (each ends with a barrier, after which lH and lB are complete as well)
  if (pre) partials_sum(pl, E, a.nblocks, sred, scratch);
  else tail_sum_partials(a.part1, E, a.nblocks, sred, scratch);
  panel_tail(a, sred, lH, lB);
}

}  // namespace tsg
