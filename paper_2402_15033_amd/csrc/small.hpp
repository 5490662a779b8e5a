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

// LDS leading dimension of the blocked small-matrix routines below: odd, so that the entries
// of one row in 16 different columns (the panel reads) fall in 16 different bank pairs.
constexpr int kLdsLd = kLd + 1;

// Blocked right-looking upper Cholesky in LDS of the kb x kb (kb <= 64) symmetric matrix whose
// upper triangle is in sR (ld LD; the strict lower part must be zero), in place: R^T R = G.
// Four columns per step: every thread factors the 4 x 4 diagonal block itself (the pivots
// d_j = the Schur complement diagonal, in the same order as the unblocked algorithm), solves
// the block's rows for the columns it needs, and takes the rank-4 update off the trailing
// entries it owns (a 16 x 16 thread grid, entries (ti + 16 m, tc + 16 q)).  A pivot
// d_j <= ptol * ref[j] (ref in LDS) stops it: rows 0 .. j-1 are then final and the failing
// index is returned (-1: success).  One barrier per step: the rows of a finished block are
// read by every thread during the step and written by their owners at the start of the next.
// For exactly 256 threads; ends with a barrier.
// (Forced inline: as a called function its LDS pointers would be generic ones, every access a
// flat memory operation with a wait on both counters.)
template <int LD>
__device__ __forceinline__ int lds_chol_upper_blk(double* sR, const double* ref, double ptol, int kb) {
  constexpr int B = 4;
  const int tid = threadIdx.x, ti = tid % 16, tc = tid / 16;
  double pend[4] = {0.0, 0.0, 0.0, 0.0};
  int prow = -1, fail = -1;
  for (int j0 = 0; j0 < kb; j0 += B) {
    if (prow >= 0) {  // the previous block's rows this thread owns
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int c = tc + 16 * q;
        if (c >= prow && c < kb) sR[prow + c * LD] = pend[q];
      }
    }
    prow = -1;
    const int bw = min(B, kb - j0);
    double D[B][B];
#pragma unroll
    for (int p = 0; p < B; ++p)
#pragma unroll
      for (int q = 0; q < B; ++q) D[p][q] = (p <= q && q < bw) ? sR[(j0 + p) + (j0 + q) * LD] : 0.0;
    // the block's rows, in place in D: R(p, p) and R(p, q > p); nok = rows that passed
    double rinv[B];
    int nok = bw;
#pragma unroll
    for (int p = 0; p < B; ++p) {
      rinv[p] = 0.0;
      if (p < nok) {
        double d = D[p][p];
#pragma unroll
        for (int r = 0; r < p; ++r) d -= D[r][p] * D[r][p];
        if (!(d > ptol * ref[j0 + p])) {
          nok = p;
        } else {
          const double rd = sqrt(d), ri = 1.0 / rd;
          D[p][p] = rd;
          rinv[p] = ri;
#pragma unroll
          for (int q = p + 1; q < B; ++q) {
            double v = D[p][q];
#pragma unroll
            for (int r = 0; r < p; ++r) v -= D[r][p] * D[r][q];
            D[p][q] = v * ri;
          }
        }
      }
    }
    // the block's rows in the thread's columns c and rows i beyond the block:
    // R(j0 + p, c) = (S(j0 + p, c) - sum_{r < p} R(j0 + r, j0 + p) R(j0 + r, c)) / R(p, p)
    double X[4][B], Y[4][B];
    auto solve = [&](int c, double (&x)[B]) {
      double sv[B];
#pragma unroll
      for (int p = 0; p < B; ++p) sv[p] = (p < bw) ? sR[(j0 + p) + c * LD] : 0.0;
#pragma unroll
      for (int p = 0; p < B; ++p) {
        double v = sv[p];
#pragma unroll
        for (int r = 0; r < p; ++r) v -= D[r][p] * x[r];
        x[p] = p < nok ? v * rinv[p] : 0.0;
      }
    };
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int c = tc + 16 * q;
      if (c >= j0 + bw && c < kb) solve(c, X[q]);
      const int i = ti + 16 * q;
      if (i >= j0 + bw && i < kb) solve(i, Y[q]);
    }
    if (nok == bw) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int c = tc + 16 * q;
        if (c < j0 + bw || c >= kb) continue;
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          const int i = ti + 16 * m;
          if (i < j0 + bw || i > c) continue;
          double v = sR[i + c * LD];
#pragma unroll
          for (int p = 0; p < B; ++p) v -= Y[m][p] * X[q][p];
          sR[i + c * LD] = v;
        }
      }
    }
    // this thread's entries in the block's final rows (at most one of its rows lies in it)
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int i = ti + 16 * m;
      if (i >= j0 && i < j0 + nok) {
        prow = i;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int c = tc + 16 * q;
          double v = 0.0;  // (columns left of row i are never written)
#pragma unroll
          for (int p = 0; p < B; ++p)
            if (p == i - j0) {
#pragma unroll
              for (int u = 0; u < B; ++u)
                if (c - j0 == u) v = D[p][u];
              if (c >= j0 + bw) v = X[q][p];
            }
          pend[q] = v;
        }
      }
    }
    __syncthreads();
    if (nok < bw) {
      fail = j0 + nok;
      break;
    }
  }
  if (prow >= 0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int c = tc + 16 * q;
      if (c >= prow && c < kb) sR[prow + c * LD] = pend[q];
    }
  }
  __syncthreads();
  return fail;
}

// X = R^{-1} for the k x k (k <= 64) upper-triangular R in LDS (ld LD) into X (LDS, ld LD,
// strict lower part zero), right-looking over blocks of four rows from the last: with S = I
// at the start, the block's rows are X(J, c) = R_JJ^{-1} S(J, c) (c in the block or beyond),
// and the finished rows take S(i, c) -= R(i, J) X(J, c) off every row i above the block.
// Every thread inverts the 4 x 4 diagonal block itself; entries are owned on a 16 x 16 thread
// grid (ti + 16 m, tc + 16 q); one barrier per block, the block's rows written by their owners
// at the start of the next step.  For exactly 256 threads; ends with a barrier.
template <int LD>
__device__ __forceinline__ void lds_tri_inv_upper_blk(const double* R, double* X, int k) {
  constexpr int B = 4;
  const int tid = threadIdx.x, ti = tid % 16, tc = tid / 16;
  for (int idx = tid; idx < kLd * LD; idx += 256) {
    const int i = idx % LD, c = idx / LD;
    X[idx] = (i == c && i < k) ? 1.0 : 0.0;
  }
  __syncthreads();
  double pend[4] = {0.0, 0.0, 0.0, 0.0};
  int prow = -1;
  const int nblk = (k + B - 1) / B;
  for (int J = nblk - 1; J >= 0; --J) {
    if (prow >= 0) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int c = tc + 16 * q;
        if (c >= prow && c < k) X[prow + c * LD] = pend[q];
      }
    }
    prow = -1;
    const int j0 = J * B, bw = min(B, k - j0);
    // Ti = R_JJ^{-1} (upper), column by column: Ti(p, q) = (delta_pq - sum_{p<r<=q} R(p,r) Ti(r,q)) / R(p,p)
    double Rb[B][B], Ti[B][B];
#pragma unroll
    for (int p = 0; p < B; ++p)
#pragma unroll
      for (int q = 0; q < B; ++q) Rb[p][q] = (p <= q && q < bw) ? R[(j0 + p) + (j0 + q) * LD] : 0.0;
    double dinv[B];
#pragma unroll
    for (int p = 0; p < B; ++p) dinv[p] = p < bw ? 1.0 / Rb[p][p] : 0.0;
#pragma unroll
    for (int q = 0; q < B; ++q)
#pragma unroll
      for (int p = B - 1; p >= 0; --p) {
        double v = (p == q) ? 1.0 : 0.0;
#pragma unroll
        for (int r = p + 1; r < B; ++r)
          if (r <= q) v -= Rb[p][r] * Ti[r][q];
        Ti[p][q] = (p <= q && q < bw) ? v * dinv[p] : 0.0;
      }
    // X(J, c) for the thread's columns c >= j0 (in the block or beyond)
    double Xc[4][B];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int c = tc + 16 * q;
#pragma unroll
      for (int p = 0; p < B; ++p) Xc[q][p] = 0.0;
      if (c >= j0 && c < k) {
        double sv[B];
#pragma unroll
        for (int p = 0; p < B; ++p) sv[p] = (p < bw) ? X[(j0 + p) + c * LD] : 0.0;
#pragma unroll
        for (int p = 0; p < B; ++p) {
          double v = 0.0;
#pragma unroll
          for (int r = 0; r < B; ++r) v += Ti[p][r] * sv[r];
          Xc[q][p] = v;
        }
      }
    }
    // rows i above the block: S(i, c) -= sum_p R(i, j0 + p) X(j0 + p, c)
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int i = ti + 16 * m;
      if (i >= j0) continue;
      double ri[B];
#pragma unroll
      for (int p = 0; p < B; ++p) ri[p] = (p < bw) ? R[i + (j0 + p) * LD] : 0.0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int c = tc + 16 * q;
        if (c < j0 || c >= k) continue;
        double v = X[i + c * LD];
#pragma unroll
        for (int p = 0; p < B; ++p) v -= ri[p] * Xc[q][p];
        X[i + c * LD] = v;
      }
    }
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int i = ti + 16 * m;
      if (i >= j0 && i < j0 + bw) {
        prow = i;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          double v = 0.0;
#pragma unroll
          for (int p = 0; p < B; ++p)
            if (p == i - j0) v = Xc[q][p];
          pend[q] = v;
        }
      }
    }
    __syncthreads();
  }
  if (prow >= 0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int c = tc + 16 * q;
      if (c >= prow && c < k) X[prow + c * LD] = pend[q];
    }
  }
  __syncthreads();
}

// C = A B for upper-triangular k x k (k <= 64) A and B in LDS (ld LD), into C (any memory,
// ld kLd; strict lower part not written): C(i, c) = sum_{i <= l <= c} A(i, l) B(l, c) in the order
// l = 0, 1, ...  For exactly 256 threads on a 16 x 16 grid (at most 4 x 4 entries each).
template <int LD, typename CPtr>
__device__ __forceinline__ void lds_trmm_upper256(const double* A, const double* B, CPtr C, int k) {
  const int tid = threadIdx.x, ti = tid % 16, tc = tid / 16;
  double acc[4][4];
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[m][q] = 0.0;
  for (int l = 0; l < k; ++l) {
    double a[4], b[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int i = ti + 16 * m;
      a[m] = (i <= l) ? A[i + l * LD] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int c = tc + 16 * q;
      b[q] = (l <= c && c < k) ? B[l + c * LD] : 0.0;
    }
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[m][q] += a[m] * b[q];
  }
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = ti + 16 * m, c = tc + 16 * q;
      if (i < k && c < k) C[i + c * kLd] = acc[m][q];
    }
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

// H(0:k, 0:k-1) (global, ld kLd) into registers, every load in flight at once: the first half
// of a copy to LDS that a tail issues before its reduction, so that both wait for memory
// together.  For exactly kTailThreads threads; hessenberg_store completes it.
struct HessPrefetch {
  static constexpr int kPer = kLd * kLd / kTailThreads;
  double v[kPer];
};
__device__ __forceinline__ void hessenberg_prefetch(const double* H, int k, HessPrefetch& pf) {
#pragma unroll
  for (int u = 0; u < HessPrefetch::kPer; ++u) {
    const int idx = threadIdx.x + kTailThreads * u, i = idx % kLd, l = idx / kLd;
    pf.v[u] = (i < k && l < k - 1) ? H[i + l * kLd] : 0.0;
  }
}
__device__ __forceinline__ void hessenberg_store(const HessPrefetch& pf, double* lH) {
#pragma unroll
  for (int u = 0; u < HessPrefetch::kPer; ++u) lH[threadIdx.x + kTailThreads * u] = pf.v[u];
}

// Hessenberg block of one s-step panel (the small-matrix algebra of Fig. 1):
//   [w_0, W] = Qb_{1:k+s} S,  S(:,1) = e_k,  S(:,2:s+1) = [P; R]
//   A [w_0..w_{s-1}] = [w_0..w_s] B,  B(i,i) = theta_i, B(i+1,i) = sigma_i, B(i-1,i) = -tau_i
//   H(1:k+s, k:k+s-1) = (S B - [H(1:k,1:k-1) S(1:k-1,1:s); 0]) T^{-1},
//   T = S(k:k+s-1, 1:s).
// P (k x s, ld kLd, LDS) and R (s x s, ld kMaxS, LDS) are the panel factors; lH (LDS, ld
// kLd) holds H(0:k, 0:k-1) on entry (hessenberg_prefetch), H (global, ld kLd) receives the
// new columns.  0-based: the new columns are k-1 .. k+s-2 and rows 0 .. k+s-1.
__device__ void block_hessenberg_panel(const double* lH, double* H, const double* P, const double* R,
                                       const double* theta, const double* sigma, const double* tau, int k,
                                       int s) {
  const int tid = threadIdx.x, nt = blockDim.x;
  const int rows = k + s;
  // LDS copies of P, R, T and the basis parameters; loops over matrices on 64-row thread
  // grids (no integer division)
  __shared__ double lP[kLd * kMaxS];
  __shared__ double lM[kLd * kMaxS];
  __shared__ double lR[kMaxS * kMaxS], lT[kMaxS * kMaxS], lB[3 * kMaxS];
  const int rg = tid % kWave, cg = tid / kWave, ncg = nt / kWave;
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
