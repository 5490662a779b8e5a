// Newton basis from Leja-ordered Ritz values (Bai, Hu and Reichel's Newton-basis GMRES,
// which the paper names as the better-conditioned alternative to the monomial basis of
// its experiments, Sec. IV and Sec. VI).
//
// From the k x k Hessenberg matrix H of a restart cycle (A Q_k = Q_{k+1} H):
//   1. its eigenvalues (the Ritz values) by Francis's implicit double-shift QR iteration;
//   2. their modified Leja ordering: the point of largest modulus first, then each next
//      point maximizes the product of its distances to the points already taken (sums of
//      logarithms), the conjugate of a complex point right after it; ties go to the larger
//      imaginary part, then to the lower index;
//   3. the step scaling sigma = the capacity estimate exp(mean_j log|z_k - z_j|) of the
//      last Leja point z_k (the Gershgorin half-width when that is not a positive finite
//      number);
//   4. the real form of the first s points: step i computes
//      w_{i+1} = ((A - theta_i I) w_i + tau_i w_{i-1}) / sigma with theta_i = Re z_i and
//      tau_i = Im(z_{i-1})^2 / sigma when z_i closes a complex pair (else 0); a pair cut
//      by position s contributes its real part alone.
//
// The routines are written for one wave: every lane runs the same control flow on values
// read from LDS, and the row/column updates are split over the lanes (lane, nl).  `sync`
// orders the wave's LDS accesses between phases.  They also compile for the host, where
// one "lane" does all the work.
#pragma once

#include "common.hpp"

namespace tsg {

constexpr double kRitzEps = 2.220446049250313e-16;  // 2^-52

// Eigenvalues (wr, wi) of the n x n upper Hessenberg matrix H (column-major, ld kLd;
// destroyed).  Only the active diagonal window is transformed: the eigenvalues of a block
// upper-triangular matrix are those of its diagonal blocks.  Returns 0, or -1 when the
// iteration did not converge within 30 n double-shift steps.  wr, wi: n entries, written
// by every lane with the same values.
template <typename Sync>
__host__ __device__ inline int hess_eigvals(double* H, int n, double* wr, double* wi, int lane, int nl,
                                            Sync sync) {
#define HH(i, j) H[(i) + (j) * kLd]
  double anorm = 0.0;  // for the deflation test next to a zero diagonal
  for (int j = 0; j < n; ++j)
    for (int i = 0; i <= (j + 1 < n ? j + 1 : n - 1); ++i) anorm += fabs(HH(i, j));
  int hi = n - 1, its = 0, total = 0;
  while (hi >= 0) {
    int l = hi;
    for (; l > 0; --l) {  // the lowest l with no negligible subdiagonal in l..hi
      double sc = fabs(HH(l - 1, l - 1)) + fabs(HH(l, l));
      if (sc == 0.0) sc = anorm;
      if (fabs(HH(l, l - 1)) <= kRitzEps * sc) break;
    }
    if (l == hi) {  // 1 x 1 block
      const double v = HH(hi, hi);
      sync();
      if (lane == 0) {
        wr[hi] = v;
        wi[hi] = 0.0;
      }
      hi -= 1;
      its = 0;
      continue;
    }
    if (l == hi - 1) {  // 2 x 2 block: lambda = d + p +- sqrt(p^2 + bc), p = (a - d) / 2
      const double a = HH(hi - 1, hi - 1), b = HH(hi - 1, hi), c = HH(hi, hi - 1), d = HH(hi, hi);
      const double p = 0.5 * (a - d), q = p * p + b * c;
      double r1, r2, i1, i2;
      if (q >= 0.0) {
        const double zz = p + copysign(sqrt(q), p);
        r1 = d + zz;
        r2 = zz != 0.0 ? d - b * c / zz : d + zz;
        i1 = i2 = 0.0;
      } else {
        r1 = r2 = d + p;
        i1 = sqrt(-q);
        i2 = -i1;
      }
      sync();
      if (lane == 0) {
        wr[hi - 1] = r1;
        wi[hi - 1] = i1;
        wr[hi] = r2;
        wi[hi] = i2;
      }
      hi -= 2;
      its = 0;
      continue;
    }
    if (total >= 30 * n) return -1;
    // the two shifts through their sum and product
    double tr, det;
    if (its == 10 || its == 20) {
      // exceptional shifts after a stall, with the constants 0.75 and -0.4375 of the
      // published EISPACK routine hqr (Wilkinson and Reinsch, Handbook for Automatic
      // Computation II, 1971; Francis's implicit double-shift QR): both shifts near
      // H(hi, hi) + 0.75 ex, a complex pair of imaginary part ~0.66 ex
      const double ex = fabs(HH(hi, hi - 1)) + fabs(HH(hi - 1, hi - 2));
      const double a = 0.75 * ex + HH(hi, hi);
      tr = 2.0 * a;
      det = a * a + 0.4375 * ex * ex;
    } else {
      const double a = HH(hi - 1, hi - 1), b = HH(hi - 1, hi), c = HH(hi, hi - 1), d = HH(hi, hi);
      tr = a + d;
      det = a * d - b * c;
    }
    its += 1;
    total += 1;
    // first column of (H - s1 I)(H - s2 I) on the window, then chase the bulge
    double x = HH(l, l) * HH(l, l) + HH(l, l + 1) * HH(l + 1, l) - tr * HH(l, l) + det;
    double y = HH(l + 1, l) * (HH(l, l) + HH(l + 1, l + 1) - tr);
    double z = HH(l + 1, l) * HH(l + 2, l + 1);
    for (int k = l; k <= hi - 1; ++k) {
      const int three = k <= hi - 2;  // 3-element reflector, else the final 2-element one
      // Householder P = I - beta v v^T with v = [1, v1, v2] mapping (x, y, z) to a multiple of e1
      const double scl = fabs(x) + fabs(y) + (three ? fabs(z) : 0.0);
      double beta = 0.0, v1 = 0.0, v2 = 0.0;
      if (scl != 0.0) {
        const double xs = x / scl, ys = y / scl, zs = three ? z / scl : 0.0;
        const double sig = ys * ys + zs * zs;
        if (sig != 0.0) {
          const double mu = sqrt(xs * xs + sig);
          const double w0 = xs <= 0.0 ? xs - mu : -sig / (xs + mu);
          beta = 2.0 * w0 * w0 / (sig + w0 * w0);
          v1 = ys / w0;
          v2 = zs / w0;
        }
      }
      sync();  // every lane has read what it needs before the updates
      if (beta != 0.0) {
        const int j0 = k - 1 > l ? k - 1 : l;
        for (int j = j0 + lane; j <= hi; j += nl) {  // rows k..k+2 from the left
          double p = HH(k, j) + v1 * HH(k + 1, j) + (three ? v2 * HH(k + 2, j) : 0.0);
          p *= beta;
          HH(k, j) -= p;
          HH(k + 1, j) -= p * v1;
          if (three) HH(k + 2, j) -= p * v2;
        }
        sync();
        const int i1 = three ? (k + 3 < hi ? k + 3 : hi) : hi;
        for (int i = l + lane; i <= i1; i += nl) {  // columns k..k+2 from the right
          double p = HH(i, k) + v1 * HH(i, k + 1) + (three ? v2 * HH(i, k + 2) : 0.0);
          p *= beta;
          HH(i, k) -= p;
          HH(i, k + 1) -= p * v1;
          if (three) HH(i, k + 2) -= p * v2;
        }
        sync();
      }
      if (k < hi - 1) {
        x = HH(k + 1, k);
        y = HH(k + 2, k);
        z = k < hi - 2 ? HH(k + 3, k) : 0.0;
      }
    }
  }
  sync();
  return 0;
#undef HH
}

// Modified Leja ordering of the k points (wr, wi) (closed under conjugation) into
// (zr, zi, second); then the capacity estimate of the ordered set (NaN for k < 2).
// logs: k scratch entries.  Every array is shared by the wave.
template <typename Sync>
__host__ __device__ inline double leja_order(const double* wr, const double* wi, int k, double* zr, double* zi,
                                             int* second, double* logs, int* used, int lane, int nl, Sync sync) {
  for (int j = lane; j < k; j += nl) {
    logs[j] = 0.0;
    used[j] = 0;
  }
  sync();
  int pos = 0;
  double last_log = 0.0;
  while (pos < k) {
    // next point: the largest modulus first, then the largest log-product
    int best = -1;
    double bs = 0.0;
    for (int j = 0; j < k; ++j) {
      if (used[j]) continue;
      const double sc = pos == 0 ? hypot(wr[j], wi[j]) : logs[j];
      if (best < 0 || sc > bs || (sc == bs && wi[j] > wi[best])) {
        best = j;
        bs = sc;
      }
    }
    int take[2] = {best, -1};
    if (wi[best] != 0.0 && pos + 1 < k) {  // its conjugate next
      double bd = 0.0;
      for (int j = 0; j < k; ++j) {
        if (used[j] || j == best) continue;
        const double d = hypot(wr[j] - wr[best], wi[j] + wi[best]);
        if (take[1] < 0 || d < bd) {
          take[1] = j;
          bd = d;
        }
      }
    }
    sync();
    for (int t = 0; t < 2 && take[t] >= 0; ++t) {
      const int c = take[t];
      if (pos == k - 1) last_log = logs[c];
      if (lane == 0) {
        zr[pos] = wr[c];
        zi[pos] = wi[c];
        second[pos] = t;
        used[c] = 1;
      }
      sync();
      for (int j = lane; j < k; j += nl)
        if (!used[j]) logs[j] += log(hypot(wr[j] - wr[c], wi[j] - wi[c]));
      sync();
      pos += 1;
    }
  }
  return k < 2 ? __builtin_nan("") : exp(last_log / (double)(k - 1));
}

// Real-form Newton parameters of the first s ordered points with step scaling sig.
__host__ __device__ inline void newton_real_form(const double* zr, const double* zi, const int* second, int s,
                                                 double sig, double* theta, double* tau, double* sigma) {
  for (int i = 0; i < s; ++i) {
    theta[i] = zr[i];
    tau[i] = (i > 0 && second[i]) ? zi[i - 1] * zi[i - 1] / sig : 0.0;
    sigma[i] = sig;
  }
}

// The whole computation on H (LDS, k x k, destroyed).  Returns 0, or -1 when the QR
// iteration did not converge (outputs untouched then).  Lane 0 writes theta/tau/sigma.
struct RitzScratch {
  double wr[kLd], wi[kLd], zr[kLd], zi[kLd], logs[kLd];
  int second[kLd], used[kLd];
};
template <typename Sync>
__host__ __device__ inline int ritz_newton(double* H, int k, int s, double lo, double hi, RitzScratch& w,
                                           double* theta, double* tau, double* sigma, int lane, int nl, Sync sync) {
  if (hess_eigvals(H, k, w.wr, w.wi, lane, nl, sync) != 0) return -1;
  double c = leja_order(w.wr, w.wi, k, w.zr, w.zi, w.second, w.logs, w.used, lane, nl, sync);
  if (!(c > 0.0) || !(c < __builtin_inf())) c = 0.5 * (hi - lo);
  if (!(c > 0.0)) c = 1.0;
  if (lane == 0) newton_real_form(w.zr, w.zi, w.second, s, c, theta, tau, sigma);
  sync();
  return 0;
}

}  // namespace tsg
