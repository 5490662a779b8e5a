// Small dense float64 routines executed by one thread block (the tails of the
// reduction kernels and the end-of-cycle kernel).  Matrices are column-major; every
// routine must be called by all threads of the block and ends with a barrier.
#pragma once

#include "state.hpp"

namespace tsg {

// Upper Cholesky factor R of the k x k symmetric matrix G (upper triangle read):
// R^T R = G, R_jj > 0 (Fig. 3's Chol).  Row-oriented: pivot d_j = G_jj - sum_{i<j} R_ij^2;
// the pivot fails when it is not > tol * ref_j (ref = ref_diag, or diag(G) if NULL),
// which with tol = 0 is the usual "not positive definite" test.  Returns -1 on success
// or the first failing pivot index.  The strictly lower part of R is zeroed.
__device__ int block_chol_upper(const double* G, int ldg, double* R, int ldr, int k,
                                const double* ref_diag, double tol) {
  __shared__ double s_piv;
  __shared__ int s_fail;
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int idx = tid; idx < k * k; idx += nt) {
    int i = idx % k, c = idx / k;
    if (i > c) R[i + c * ldr] = 0.0;
  }
  __syncthreads();
  for (int j = 0; j < k; ++j) {
    if (tid == 0) {
      double d = G[j + j * ldg];
      for (int i = 0; i < j; ++i) {
        double r = R[i + j * ldr];
        d -= r * r;
      }
      double ref = ref_diag ? ref_diag[j] : G[j + j * ldg];
      int fail = !(d > tol * ref);
      s_fail = fail;
      s_piv = fail ? 0.0 : sqrt(d);
      if (!fail) R[j + j * ldr] = s_piv;
    }
    __syncthreads();
    if (s_fail) return j;
    const double rjj = s_piv;
    for (int c = j + 1 + tid; c < k; c += nt) {
      double v = G[j + c * ldg];
      for (int i = 0; i < j; ++i) v -= R[i + j * ldr] * R[i + c * ldr];
      R[j + c * ldr] = v / rjj;
    }
    __syncthreads();
  }
  return -1;
}

// block_chol_upper's factorization for k <= 16 by wave 0 alone (lane c owns column c; the
// same operations in the same order, one wave-level sync per step instead of three block
// barriers).  Called by every thread of the block; ends with a barrier.
__device__ int small_chol_upper(const double* G, int ldg, double* R, int ldr, int k, const double* ref_diag,
                                double tol) {
  __shared__ int s_fail;
  const int tid = threadIdx.x;
  if (tid < kWave) {
    const int c = tid;
    int fail = -1;
    if (c < k)
      for (int i = c + 1; i < k; ++i) R[i + c * ldr] = 0.0;
    for (int j = 0; j < k; ++j) {
      double d = G[j + j * ldg];
      for (int i = 0; i < j; ++i) {
        const double r = R[i + j * ldr];
        d -= r * r;
      }
      const double ref = ref_diag ? ref_diag[j] : G[j + j * ldg];
      if (!(d > tol * ref)) {
        fail = j;
        break;
      }
      const double rjj = sqrt(d);
      if (c > j && c < k) {
        double v = G[j + c * ldg];
        for (int i = 0; i < j; ++i) v -= R[i + j * ldr] * R[i + c * ldr];
        R[j + c * ldr] = v / rjj;
      }
      if (c == j) R[j + j * ldr] = rjj;
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    }
    if (tid == 0) s_fail = fail;
  }
  __syncthreads();
  return s_fail;
}

// Right-looking upper Cholesky in LDS of the kb x kb (kb <= 64) symmetric matrix whose upper
// triangle is in sR (ld kLd; the strict lower part must be zero), in place: R^T R = G.  A pivot
// d_j <= ptol * ref[j] (ref in LDS) stops it; rows 0 .. j-1 are then final and the failing
// index is returned (-1: success).  For exactly 256 threads.  One barrier per step: every
// thread takes the pivot itself, the trailing update uses row j divided on the fly, and row j
// is scaled in place during the next step (which reads neither it nor its diagonal).  (A
// single-wave version with wave-level syncs only was measured slower: the per-step chain of
// dependent LDS accesses of one wave costs more than the barrier of four.)
__device__ int lds_chol_upper256(double* sR, const double* ref, double ptol, int kb) {
  const int tid = threadIdx.x, nt = blockDim.x;
  int jp = -1, fail = -1;
  double rp = 0.0, rpi = 0.0;
  for (int j = 0; j < kb; ++j) {
    const double d = sR[j + j * kLd];
    const bool bad = !(d > ptol * ref[j]);
    if (jp >= 0) {  // finish row j - 1
      for (int c = jp + 1 + tid; c < kb; c += nt) sR[jp + c * kLd] *= rpi;
      if (tid == 0) sR[jp + jp * kLd] = rp;
    }
    jp = -1;
    if (bad) {
      fail = j;
      break;
    }
    const double rjj = sqrt(d), rinv = 1.0 / rjj;
    // trailing update on a 16 x 16 thread grid (at most 4 x 4 entries per thread): all
    // loads of a column's entries before its stores
    {
      const int r0 = j + 1 + tid % 16, c0 = j + 1 + tid / 16;
      double ri[4];
#pragma unroll
      for (int m = 0; m < 4; ++m) ri[m] = (r0 + 16 * m < kb) ? sR[j + (r0 + 16 * m) * kLd] * rinv : 0.0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int c = c0 + 16 * q;
        if (c >= kb) break;
        const double rjc = sR[j + c * kLd] * rinv;
        double v[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) v[m] = (r0 + 16 * m <= c) ? sR[r0 + 16 * m + c * kLd] : 0.0;
#pragma unroll
        for (int m = 0; m < 4; ++m)
          if (r0 + 16 * m <= c) sR[r0 + 16 * m + c * kLd] = v[m] - ri[m] * rjc;
      }
    }
    jp = j;
    rp = rjj;
    rpi = rinv;
    __syncthreads();
  }
  if (jp >= 0) {  // the last row when no pivot failed
    for (int c = jp + 1 + tid; c < kb; c += nt) sR[jp + c * kLd] *= rpi;
    if (tid == 0) sR[jp + jp * kLd] = rp;
  }
  __syncthreads();
  return fail;
}

// X = R^{-1} for upper-triangular k x k R with R and X in LDS (ld kLd): one thread per
// column of X, back substitution over its own column.  Ends with a barrier.
__device__ void lds_tri_inv_upper(const double* R, double* X, int k) {
  for (int c = threadIdx.x; c < k; c += blockDim.x) {
    for (int i = k - 1; i >= 0; --i) {
      double v = (i == c) ? 1.0 : 0.0;
      if (i <= c) {
        for (int l = i + 1; l <= c; ++l) v -= R[i + l * kLd] * X[l + c * kLd];
        v /= R[i + i * kLd];
      }
      X[i + c * kLd] = v;
    }
  }
  __syncthreads();
}

// X = R^{-1} for upper-triangular k x k R (one thread per column of X).
__device__ void block_tri_inv_upper(const double* R, int ldr, double* X, int ldx, int k) {
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int c = tid; c < k; c += nt) {
    for (int i = k - 1; i >= 0; --i) {
      double v = (i == c) ? 1.0 : 0.0;
      if (i <= c) {
        for (int l = i + 1; l <= c; ++l) v -= R[i + l * ldr] * X[l + c * ldx];
        v /= R[i + i * ldr];
      }
      X[i + c * ldx] = v;
    }
  }
  __syncthreads();
}

// C (a x b) = A (a x l) * B (l x b), general, parallel over entries.
__device__ void block_gemm(const double* A, int lda, const double* B, int ldb, double* C, int ldc,
                           int a, int l, int b) {
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int idx = tid; idx < a * b; idx += nt) {
    int i = idx % a, j = idx / a;
    double v = 0.0;
    for (int t = 0; t < l; ++t) v += A[i + t * lda] * B[t + j * ldb];
    C[i + j * ldc] = v;
  }
  __syncthreads();
}

// Hessenberg block of one s-step panel (the small-matrix algebra of Fig. 1):
//   [w_0, W] = Qb_{1:k+s} S,  S(:,1) = e_k,  S(:,2:s+1) = [P; R]
//   A [w_0..w_{s-1}] = [w_0..w_s] B,  B(i,i) = theta_i, B(i+1,i) = sigma_i, B(i-1,i) = -tau_i
//   H(1:k+s, k:k+s-1) = (S B - [H(1:k,1:k-1) S(1:k-1,1:s); 0]) T^{-1},
//   T = S(k:k+s-1, 1:s).
// P (k x s, ld kLd) and R (s x s, ld kMaxS) are the panel factors, H (ld kLd) holds
// columns 0..k-2 on entry.  M is a kLd x kMaxS scratch.  0-based: the new columns are
// k-1 .. k+s-2 and rows 0 .. k+s-1.
__device__ void block_hessenberg_panel(double* H, const double* P, const double* R,
                                       const double* theta, const double* sigma, const double* tau, int k,
                                       int s, double* M) {
  (void)M;  // the products and the solve run in LDS
  const int tid = threadIdx.x, nt = blockDim.x;
  const int rows = k + s;
  // LDS copies of the operands (H(0:k, 0:k-1) is upper Hessenberg), of R, of T and of
  // the basis parameters; loops over matrices on 64-row thread grids (no integer division)
  __shared__ double lH[kLd * kLd];
  __shared__ double lP[kLd * kMaxS];
  __shared__ double lM[kLd * kMaxS];
  __shared__ double lR[kMaxS * kMaxS], lT[kMaxS * kMaxS], lB[3 * kMaxS];
  const int rg = tid % kWave, cg = tid / kWave, ncg = nt / kWave;
  for (int l = cg; l < k - 1; l += ncg)
    for (int i = rg; i < k; i += kWave) lH[i + l * kLd] = H[i + l * kLd];
  for (int c = cg; c < s; c += ncg)
    for (int i = rg; i < k; i += kWave) lP[i + c * kLd] = P[i + c * kLd];
  if (tid < s * s) {
    const int a = tid % s, c = tid / s;
    lR[a + c * kMaxS] = R[a + c * kMaxS];
    // T = S(k-1 .. k+s-2, 0 .. s-1): T(0,0) = 1, T(a,0) = 0, T(0,c) = P(k-1,c-1), T(a,c) = R(a-1,c-1)
    lT[a + c * kMaxS] = c == 0 ? (a == 0 ? 1.0 : 0.0) : (a == 0 ? P[(k - 1) + (c - 1) * kLd] : R[(a - 1) + (c - 1) * kMaxS]);
  }
  if (tid < s) {
    lB[tid] = theta[tid];
    lB[kMaxS + tid] = sigma[tid];
    lB[2 * kMaxS + tid] = tau[tid];
  }
  __syncthreads();
  auto Sv = [&](int i, int l) -> double {  // S(i, l), 0-based, l in [0, s]
    if (l == 0) return (i == k - 1) ? 1.0 : 0.0;
    return (i < k) ? lP[i + (l - 1) * kLd] : lR[(i - k) + (l - 1) * kMaxS];
  };
  for (int c = cg; c < s; c += ncg)
    for (int i = rg; i < rows; i += kWave) {
      double v = Sv(i, c) * lB[c] + Sv(i, c + 1) * lB[kMaxS + c];
      if (c >= 1 && lB[2 * kMaxS + c] != 0.0) v -= Sv(i, c - 1) * lB[2 * kMaxS + c];
      if (c >= 1 && i < k) {
#pragma unroll 4
        for (int l = (i > 0 ? i - 1 : 0); l < k - 1; ++l) v -= lH[i + l * kLd] * lP[l + (c - 1) * kLd];
      }
      lM[i + c * kLd] = v;
    }
  __syncthreads();
  // right solve with T (upper triangular), one thread per row (rows <= 64):
  // X(i,c) = (M(i,c) - sum_{a<c} X(i,a) T(a,c)) / T(c,c), written over M
  if (tid < rows) {
    for (int c = 0; c < s; ++c) {
      double v = lM[tid + c * kLd];
      for (int a = 0; a < c; ++a) v -= lM[tid + a * kLd] * lT[a + c * kMaxS];
      lM[tid + c * kLd] = v / lT[c + c * kMaxS];
    }
  }
  __syncthreads();
  for (int c = cg; c < s; c += ncg)
    for (int i = rg; i < rows; i += kWave) H[i + (k - 1 + c) * kLd] = lM[i + c * kLd];
  __syncthreads();
}

// Append Hessenberg columns c0..c1-1 (0-based) to the incremental Givens QR held in
// st (rotations gc/gs, rhs gg, triangular Rg).  One thread; columns are copied to
// a local buffer so the rotation chain runs in registers / LDS.
__device__ void givens_append(SmallState* st, const double* H, int c0, int c1) {
  __shared__ double col[kLd + 1];
  __shared__ double lc[kLd], ls[kLd];
  for (int i = threadIdx.x; i < c0; i += blockDim.x) {
    lc[i] = st->gc[i];
    ls[i] = st->gs[i];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int c = c0; c < c1; ++c) {
      for (int i = 0; i <= c + 1; ++i) col[i] = H[i + c * kLd];
      for (int i = 0; i < c; ++i) {
        double cs = lc[i], sn = ls[i];
        double a = col[i], b = col[i + 1];
        col[i] = cs * a + sn * b;
        col[i + 1] = -sn * a + cs * b;
      }
      double a = col[c], b = col[c + 1];
      double rho = hypot(a, b);
      double cs = 1.0, sn = 0.0;
      if (rho != 0.0) {
        cs = a / rho;
        sn = b / rho;
      }
      st->gc[c] = cs;
      st->gs[c] = sn;
      lc[c] = cs;
      ls[c] = sn;
      col[c] = rho;
      for (int i = 0; i <= c; ++i) st->Rg[i + c * kLd] = col[i];
      double gk = st->gg[c];
      st->gg[c] = cs * gk;
      st->gg[c + 1] = -sn * gk;
    }
  }
  __syncthreads();
}

// coef(0:k) = Rg(0:k,0:k)^{-1} gg(0:k) (back substitution, one thread).
__device__ void givens_solve(SmallState* st, int k) {
  if (threadIdx.x == 0) {
    for (int i = k - 1; i >= 0; --i) {
      double v = st->gg[i];
      for (int l = i + 1; l < k; ++l) v -= st->Rg[i + l * kLd] * st->coef[l];
      st->coef[i] = v / st->Rg[i + i * kLd];
    }
  }
  __syncthreads();
}

}  // namespace tsg
