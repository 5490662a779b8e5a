// Sparse, vector and end-of-cycle kernels of the tsgmres library.
#pragma once

#include "panel.hpp"
#include "precond.hpp"
#include "ritz.hpp"

namespace tsg {

constexpr int kRowBlock = 256;  // threads (rows) per block of the row-parallel kernels

// ------------------------------------------------------------------ matrix powers

constexpr int kSegCap = 8 * kWave;  // products staged per wave (rows of <= 8 nonzeros on average)

// acc(r) = sum_p val[p] x[col[p]] for the 64 rows r0 .. r0+63 of one wave.  The wave's
// nonzeros form one contiguous CSR segment: it is loaded with fully coalesced accesses,
// multiplied by the gathered x, staged in LDS, and every lane then sums its own row's
// slice.  Segments longer than kSegCap fall back to the per-row loop.
template <typename T, typename VT>
__device__ __forceinline__ T csr_row_dot(gbl<const int32_t>* __restrict__ row_ptr,
                                         gbl<const int32_t>* __restrict__ col, gbl<const VT>* __restrict__ val,
                                         gbl<const T>* __restrict__ x, int64_t n, int64_t r0, int lane, T* prod) {
#pragma clang fp contract(off)
  const int64_t r = r0 + lane;
  const int nrows = (int)min((int64_t)kWave, n - r0);
  const int rp = (r < n) ? row_ptr[r] : 0;
  const int rp1 = (r < n) ? row_ptr[r + 1] : 0;
  const int base = __shfl(rp, 0, kWave);
  const int end = __shfl(rp1, nrows - 1, kWave);
  const int cnt = end - base;
  T acc = (T)0;
  if (cnt <= kSegCap) {
#pragma unroll 4
    for (int e = lane; e < cnt; e += kWave) {
      // the CSR arrays stream through once per product: non-temporal, so x stays cached
      const VT a = __builtin_nontemporal_load(&val[base + e]);
      const int32_t cidx = __builtin_nontemporal_load(&col[base + e]);
      prod[e] = (T)a * x[cidx];
    }
    wave_lds_sync();
    for (int e = rp - base; e < rp1 - base; ++e) acc += prod[e];
    wave_lds_sync();
  } else {
    for (int p = rp; p < rp1; ++p) acc += (T)val[p] * x[col[p]];
  }
  return acc;
}

// ------------------------------------------------------------------ packed operator
// SELL-64 layout of the operator (built once per CSR handle by tsg_csr_pack): slices of 64
// consecutive rows, one wave each; slice s holds width w_s = its longest row, stored entry
// by entry -- element e of row 64 s + l at off_s + 64 e + l -- so that the wave's loads of
// values and columns are fully coalesced 64-entry runs and no row pointer is read.  Short
// rows are padded with value 0 and column delta 0.  Columns are stored as int16 deltas
// col - row when every delta fits (FMT_SELL16: 2 bytes instead of 4 per nonzero), else as
// int32 columns (FMT_SELL32).
enum OpFormat : int { FMT_CSR = 0, FMT_SELL16 = 1, FMT_SELL32 = 2 };

// acc += sum over entries e0 .. e0 + K - 1 of one slice: all K value and column loads, then
// all K x gathers are issued before the first product (two dependent memory round trips
// per group); products rounded, then summed in entry order.  Plain loads: with the
// non-temporal hint on the value and column streams the step ran at 5.3 TB/s instead
// of 5.8 (2048^2 Laplacian, FP64).
template <int K, typename T, typename VT, int FMT>
__device__ __forceinline__ T sell_group(gbl<const VT>* __restrict__ sval, const void* scol_,
                                        gbl<const T>* __restrict__ x, int64_t q0, int64_t rb, T acc) {
#pragma clang fp contract(off)
  VT v[K];
  int64_t c[K];
#pragma unroll
  for (int u = 0; u < K; ++u) {
    const int64_t q = q0 + (int64_t)u * kWave;
    v[u] = sval[q];
    if (FMT == FMT_SELL16)
      c[u] = G(reinterpret_cast<const int16_t*>(scol_))[q];
    else
      c[u] = G(reinterpret_cast<const int32_t*>(scol_))[q];
  }
  T xv[K];
#pragma unroll
  for (int u = 0; u < K; ++u) xv[u] = x[FMT == FMT_SELL16 ? rb + c[u] : c[u]];
#pragma unroll
  for (int u = 0; u < K; ++u) {
    const T prod = (T)v[u] * xv[u];
    acc += prod;
  }
  return acc;
}

// acc(r) = sum_e val * x[col] for row r = 64 slice + lane of a packed operator; the
// products are rounded before they are summed, in the rows' CSR order (as csr_row_dot).
// The slice index is uniform over the wave, so its width w is too: every lane runs all w
// entries (rows past n are all padding -- value 0, delta 0 -- and gather x[n - 1], an
// index in range).  Entries go in groups of 8, the last w mod 8 as one group of that size,
// so a slice of width <= 8 costs two dependent memory round trips.
template <typename T, typename VT, int FMT>
__device__ __forceinline__ T sell_row_dot(gbl<const int64_t>* __restrict__ soff, gbl<const VT>* __restrict__ sval,
                                          const void* scol_, gbl<const T>* __restrict__ x, int64_t n, int64_t slice,
                                          int lane) {
  const int64_t off = soff[slice];
  const int w = (int)((soff[slice + 1] - off) >> 6);
  const int64_t r = slice * kWave + lane;
  const int64_t rb = r < n ? r : n - 1;
  T acc = (T)0;
  int e0 = 0;
  for (; e0 + 8 <= w; e0 += 8) acc = sell_group<8, T, VT, FMT>(sval, scol_, x, off + (int64_t)e0 * kWave + lane, rb, acc);
  const int64_t q0 = off + (int64_t)e0 * kWave + lane;
  switch (w - e0) {
    case 1: acc = sell_group<1, T, VT, FMT>(sval, scol_, x, q0, rb, acc); break;
    case 2: acc = sell_group<2, T, VT, FMT>(sval, scol_, x, q0, rb, acc); break;
    case 3: acc = sell_group<3, T, VT, FMT>(sval, scol_, x, q0, rb, acc); break;
    case 4: acc = sell_group<4, T, VT, FMT>(sval, scol_, x, q0, rb, acc); break;
    case 5: acc = sell_group<5, T, VT, FMT>(sval, scol_, x, q0, rb, acc); break;
    case 6: acc = sell_group<6, T, VT, FMT>(sval, scol_, x, q0, rb, acc); break;
    case 7: acc = sell_group<7, T, VT, FMT>(sval, scol_, x, q0, rb, acc); break;
    default: break;
  }
  return acc;
}

// Per slice: its width (longest row) and whether every column delta col - row of its rows
// fits int16.  One wave per slice.
__global__ __launch_bounds__(kRowBlock) void sell_analyze_kernel(const int32_t* __restrict__ row_ptr,
                                                                 const int32_t* __restrict__ col, int64_t n,
                                                                 int64_t nslices, int* width, int* fits16) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t slice = (int64_t)blockIdx.x * (kRowBlock / kWave) + threadIdx.x / kWave;
  if (slice >= nslices) return;
  const int64_t r = slice * kWave + lane;
  int len = 0, ok = 1;
  if (r < n) {
    const int p0 = row_ptr[r], p1 = row_ptr[r + 1];
    len = p1 - p0;
    for (int p = p0; p < p1; ++p) {
      const int64_t d = (int64_t)col[p] - r;
      if (d < -32768 || d > 32767) ok = 0;
    }
  }
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) {
    len = max(len, __shfl_xor(len, o, kWave));
    ok = min(ok, __shfl_xor(ok, o, kWave));
  }
  if (lane == 0) {
    width[slice] = len;
    fits16[slice] = ok;
  }
}

// Fill the packed arrays from CSR: one thread per (padded) row.
__global__ __launch_bounds__(kRowBlock) void sell_fill_kernel(const int32_t* __restrict__ row_ptr,
                                                              const int32_t* __restrict__ col,
                                                              const double* __restrict__ val, int64_t n,
                                                              int64_t nslices, const int64_t* __restrict__ soff,
                                                              double* __restrict__ v64, float* __restrict__ v32,
                                                              void* scol, int fmt) {
  const int64_t r = (int64_t)blockIdx.x * kRowBlock + threadIdx.x;
  if (r >= nslices * kWave) return;
  const int64_t slice = r / kWave;
  const int lane = (int)(r % kWave);
  const int64_t off = soff[slice];
  const int w = (int)((soff[slice + 1] - off) >> 6);
  const int p0 = r < n ? row_ptr[r] : 0, p1 = r < n ? row_ptr[r + 1] : 0;
  for (int e = 0; e < w; ++e) {
    const int64_t q = off + (int64_t)e * kWave + lane;
    const int p = p0 + e;
    const bool real = p < p1;
    const double v = real ? val[p] : 0.0;
    v64[q] = v;
    v32[q] = (float)v;
    if (fmt == FMT_SELL16) static_cast<int16_t*>(scol)[q] = real ? (int16_t)((int64_t)col[p] - r) : (int16_t)0;
    else static_cast<int32_t*>(scol)[q] = real ? col[p] : (int32_t)(r < n ? r : 0);
  }
}

// One step of the matrix-powers kernel (Sec. III): y = (A x - theta x + tau xm) / sigma,
// with the step's theta, sigma, tau read from the request's state (tau != 0 only where
// the Newton basis closes a complex pair; xm is the basis vector before x).
// 4 waves x 64 rows per block; blocks are mapped XCD-contiguously so the x gathers of
// neighbouring rows hit the same L2.  Values of type VT (float64, or the float32 copy of
// the mixed-precision form), vectors of type T.
struct MpkArgs {
  const int32_t* row_ptr;  // CSR; packed: the slice offsets (int64)
  const void* col;         // CSR int32; packed: int16 deltas or int32 columns
  const void* val;         // VT[nnz] (packed: padded)
  const void* x;           // T[n]
  void* y;                 // T[n]
  const void* xm;          // T[n], the vector before x (NULL at a panel's first step)
  const void* xs;          // T[n], the vector the shift applies to: x, or (right
                           // preconditioning) the basis vector w with x = M^{-1} w
  int64_t n;
  const SmallState* st;
  int32_t step;            // index of the step in the panel (0 .. s-1)
  int32_t panel;
};
template <typename T, typename VT, int FMT>
struct MpkBody {
  typedef MpkArgs Args;
  static constexpr int kThreads = kRowBlock;
  static constexpr int kMinWaves = 1;
  static __device__ void run(const MpkArgs& a, int bid, int nb) {
    gbl<const SmallState>* st = G(a.st);
    if (st->h.done || a.panel > st->h.stop_panel) return;
    gbl<const VT>* __restrict__ val = G(reinterpret_cast<const VT*>(a.val));
    gbl<const T>* __restrict__ x = G(reinterpret_cast<const T*>(a.x));
    gbl<T>* __restrict__ y = G(reinterpret_cast<T*>(a.y));
    const int64_t n = a.n;
    const int lane = threadIdx.x & (kWave - 1);
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int64_t r0 = (int64_t)xcd_tile(bid, nb) * kRowBlock + wv * kWave;
    if (r0 >= n) return;
    const double theta = st->theta[a.step], sigma = st->sigma[a.step], tau = st->tau[a.step];
    const int64_t r = r0 + lane, rc = r < n ? r : n - 1;
    // the shift and pair terms are loaded before the row's products
    T xsv = (T)0, xmv = (T)0;
    if (theta != 0.0) xsv = G(reinterpret_cast<const T*>(a.xs))[rc];
    if (tau != 0.0 && a.xm) xmv = G(reinterpret_cast<const T*>(a.xm))[rc];
    T acc;
    if (FMT == FMT_CSR) {
      __shared__ T prod[kRowBlock / kWave][kSegCap];
      acc = csr_row_dot<T, VT>(G(a.row_ptr), G(reinterpret_cast<const int32_t*>(a.col)), val, x, n, r0, lane,
                               prod[wv]);
    } else {
      acc = sell_row_dot<T, VT, FMT>(G(reinterpret_cast<const int64_t*>(a.row_ptr)), val, a.col, x, n,
                                     r0 / kWave, lane);
    }
    if (r < n) {
      T v = acc;
      if (theta != 0.0) v -= (T)theta * xsv;
      if (tau != 0.0 && a.xm) v += (T)tau * xmv;
      // (non-temporal, like every basis column a streaming kernel writes: the next step's
      // gathers of it and the Gram's reads ran faster than after plain stores -- SpMV steps
      // 43.2 -> 41.1 us, Grams 193 -> 184 us per launch on the 2048^2 Laplace solve)
      __builtin_nontemporal_store(v / (T)sigma, &y[r]);
    }
  }
};

// y = A x in float64 (stand-alone SpMV entry point).
__global__ __launch_bounds__(kRowBlock) void spmv_f64_kernel(
    const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
    const double* __restrict__ val, const double* __restrict__ x, double* __restrict__ y,
    int64_t n) {
  const int64_t r = (int64_t)xcd_tile(blockIdx.x, gridDim.x) * kRowBlock + threadIdx.x;
  if (r >= n) return;
  const int p0 = row_ptr[r], p1 = row_ptr[r + 1];
  double acc = 0.0;
  for (int p = p0; p < p1; ++p) acc += val[p] * x[col[p]];
  y[r] = acc;
}

// ------------------------------------------------------------------ restart residual
// r = b - A x (float64), stored into basis column 0 (type T); per-block ||r||^2
// partials.  residual_tail_kernel sums them in a fixed order and decides convergence
// (explicit residual test), then initializes the cycle: beta, T = 1/beta for the
// scaling pass, Givens rhs, cleared Hessenberg and stage-2 Gram.
struct ResidArgs {
  const int32_t* row_ptr;  // as in MpkArgs
  const void* col;
  const double* val;
  const double* x;
  const double* b;
  void* r_out;  // T[n]: basis column 0
  int64_t n;
  const SmallState* st;
  double* part1;
};
template <typename T, int FMT>
struct ResidBody {
  typedef ResidArgs Args;
  static constexpr int kThreads = kRowBlock;
  static constexpr int kMinWaves = 1;
  static __device__ void run(const ResidArgs& a, int bid, int nb);
};
template <typename T, int FMT>
__device__ void ResidBody<T, FMT>::run(const ResidArgs& a, int bid, int nb) {
  gbl<const SmallState>* __restrict__ st = G(a.st);
  if (st->h.done) return;
  gbl<const double>* __restrict__ val = G(a.val);
  gbl<const double>* __restrict__ x = G(a.x);
  gbl<const double>* __restrict__ b = G(a.b);
  gbl<T>* __restrict__ r_out = G(reinterpret_cast<T*>(a.r_out));
  const int64_t n = a.n;
  gbl<double>* part1 = G(a.part1);
  __shared__ double prod[kRowBlock / kWave][kSegCap];
  const int lane = threadIdx.x & (kWave - 1);
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int64_t r0 = (int64_t)xcd_tile(bid, nb) * kRowBlock + wv * kWave;
  double rr = 0.0;
  if (r0 < n) {
    const double acc =
        FMT == FMT_CSR
            ? csr_row_dot<double, double>(G(a.row_ptr), G(reinterpret_cast<const int32_t*>(a.col)), val, x, n, r0,
                                          lane, prod[wv])
            : sell_row_dot<double, double, FMT>(G(reinterpret_cast<const int64_t*>(a.row_ptr)), val, a.col, x,
                                                n, r0 / kWave, lane);
    const int64_t r = r0 + lane;
    if (r < n) {
      double v = b[r] - acc;
      __builtin_nontemporal_store((T)v, &r_out[r]);
      rr = v * v;
    }
  }
  __shared__ double wsum[kRowBlock / kWave];
  rr = wave_sum(rr);
  if ((threadIdx.x & (kWave - 1)) == 0) wsum[threadIdx.x / kWave] = rr;
  __syncthreads();
  if (threadIdx.x == 0) {
    double sum = 0.0;
    for (int w = 0; w < kRowBlock / kWave; ++w) sum += wsum[w];
    part1[bid] = sum;
  }
}

// Arguments of the one-block kernels that act on one request's small state.
struct TailArgs {
  SmallState* st;
  const double* part1;
  int32_t nblocks;
  int32_t two_stage;
};
struct RTailBody {
  typedef TailArgs Args;
  static constexpr int kThreads = kTailThreads;
  static constexpr int kMinWaves = 1;
  static __device__ void run(const TailArgs& a, int bid, int nb);
};
__device__ void RTailBody::run(const TailArgs& a, int, int) {
  SmallState* st = Gp(a.st);  // (global, not flat, accesses)
  const double* part1 = a.part1;
  const int nblocks = a.nblocks;
  if (st->h.done) return;
  __shared__ double s_tot[1];
  __shared__ double scratch[kTailThreads];
  __shared__ int s_go;
  block_sum_partials(part1, 1, nblocks, s_tot, scratch);
  const int tid = threadIdx.x, nt = blockDim.x;
  if (tid == 0) {
    double beta = sqrt(s_tot[0]);
    st->h.relres = beta / st->bnorm;
    s_go = 0;
    if (st->h.relres <= st->tol) {
      st->h.done = 1;
      st->h.status = 0;
    } else if (st->h.iters >= st->max_iters) {
      st->h.done = 1;
      st->h.status = 1;
    } else if (st->h.cycles > 0 && st->h.k_used == 0) {
      st->h.done = 1;  // the previous cycle could keep no vector: no progress possible
      st->h.status = 2;
    } else {
      s_go = 1;
      st->beta = beta;
      st->inv_beta = 1.0 / beta;
      st->Tcur[0] = 1.0 / beta;
      st->identity_t = 0;
      st->h.stop_panel = 1 << 30;
      st->h.k_used = st->m;
      st->h.refine = 0;
      st->h.refine2 = 0;
      st->h.redo = 0;
      st->gscale = beta;
    }
  }
  __syncthreads();
  if (!s_go) return;
  for (int i = tid; i < kLd * kLd; i += nt) {
    st->Hh[i] = 0.0;
    st->G2[i] = 0.0;
  }
  for (int i = tid; i <= kLd; i += nt) st->gg[i] = (i == 0) ? st->beta : 0.0;
}

// per-block partials of ||b||^2; norm_tail_kernel -> st->bnorm (float64, deterministic).
__global__ __launch_bounds__(kRowBlock) void norm_kernel(const double* __restrict__ b, int64_t n,
                                                         double* part1) {
  const int64_t r = (int64_t)blockIdx.x * kRowBlock + threadIdx.x;
  double v = (r < n) ? b[r] * b[r] : 0.0;
  __shared__ double wsum[kRowBlock / kWave];
  v = wave_sum(v);
  if ((threadIdx.x & (kWave - 1)) == 0) wsum[threadIdx.x / kWave] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double sum = 0.0;
    for (int w = 0; w < kRowBlock / kWave; ++w) sum += wsum[w];
    part1[blockIdx.x] = sum;
  }
}

__global__ __launch_bounds__(kTailThreads) void norm_tail_kernel(SmallState* st, const double* part1,
                                                                 int nblocks) {
  __shared__ double s_tot[1];
  __shared__ double scratch[kTailThreads];
  block_sum_partials(part1, 1, nblocks, s_tot, scratch);
  if (threadIdx.x == 0) st->bnorm = sqrt(s_tot[0]);
}

// ------------------------------------------------------------------ Gershgorin interval
// Per-block min(a_ii - r_i) and max(a_ii + r_i), r_i = sum_{j != i} |a_ij|.
__global__ __launch_bounds__(kRowBlock) void gershgorin_kernel(
    const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
    const double* __restrict__ val, int64_t n, double* out /* [2 * gridDim] */) {
  const int64_t r = (int64_t)blockIdx.x * kRowBlock + threadIdx.x;
  double lo = INFINITY, hi = -INFINITY;
  if (r < n) {
    double d = 0.0, rad = 0.0;
    for (int p = row_ptr[r]; p < row_ptr[r + 1]; ++p) {
      if (col[p] == r) d += val[p];
      else rad += fabs(val[p]);
    }
    lo = d - rad;
    hi = d + rad;
  }
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) {
    lo = fmin(lo, __shfl_xor(lo, o, kWave));
    hi = fmax(hi, __shfl_xor(hi, o, kWave));
  }
  __shared__ double slo[kRowBlock / kWave], shi[kRowBlock / kWave];
  if ((threadIdx.x & (kWave - 1)) == 0) {
    slo[threadIdx.x / kWave] = lo;
    shi[threadIdx.x / kWave] = hi;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kRowBlock / kWave; ++w) {
      lo = fmin(lo, slo[w]);
      hi = fmax(hi, shi[w]);
    }
    out[2 * blockIdx.x] = lo;
    out[2 * blockIdx.x + 1] = hi;
  }
}

__global__ __launch_bounds__(kRowBlock) void minmax_final_kernel(const double* in, int nb, double* out) {
  double lo = INFINITY, hi = -INFINITY;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) {
    lo = fmin(lo, in[2 * i]);
    hi = fmax(hi, in[2 * i + 1]);
  }
  __shared__ double slo[kRowBlock], shi[kRowBlock];
  slo[threadIdx.x] = lo;
  shi[threadIdx.x] = hi;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < (int)blockDim.x; ++i) {
      lo = fmin(lo, slo[i]);
      hi = fmax(hi, shi[i]);
    }
    out[0] = lo;
    out[1] = hi;
  }
}

// float64 -> float32 copy (CSR values of the mixed-precision form).
__global__ __launch_bounds__(kRowBlock) void to_f32_kernel(const double* __restrict__ a,
                                                           float* __restrict__ b, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kRowBlock + threadIdx.x;
  if (i < n) b[i] = (float)a[i];
}

// ------------------------------------------------------------------ solution update
// x += V(:, 0:ku) coef (x float64, basis type T).  coef is uniform across the block.
struct XupdArgs {
  double* x;
  const void* V;  // T basis
  int64_t ld, n;
  const SmallState* st;
  double* t;      // non-NULL (right preconditioning): t = V coef instead of x += V coef
};
// acc += sum over columns c0 .. c0 + K - 1 of V(r, c) coef(c), in column order; the K loads
// are issued before the first product.
template <int K, typename T>
__device__ __forceinline__ double xupd_group(gbl<const T>* __restrict__ V, int64_t ld, int64_t r, int c0,
                                            gbl<const double>* coef, double acc) {
  T q[K];
#pragma unroll
  for (int u = 0; u < K; ++u) q[u] = __builtin_nontemporal_load(&V[(int64_t)(c0 + u) * ld + r]);
#pragma unroll
  for (int u = 0; u < K; ++u) acc += (double)q[u] * coef[c0 + u];
  return acc;
}

template <typename T>
struct XupdBody {
  typedef XupdArgs Args;
  static constexpr int kThreads = kRowBlock;
  static constexpr int kMinWaves = 1;
  static __device__ void run(const XupdArgs& a, int bid, int) {
    gbl<const SmallState>* __restrict__ st = G(a.st);
    if (st->h.done || st->h.redo) return;
    gbl<const T>* __restrict__ V = G(reinterpret_cast<const T*>(a.V));
    gbl<double>* __restrict__ x = G(a.x);
    const int ku = st->h.k_used;
    const int64_t r = (int64_t)bid * kRowBlock + threadIdx.x;
    if (r >= a.n) return;
    // columns in groups of 16, then one of 8, then one of the remaining size, each group's
    // loads issued before its first product; the sum runs in column order
    gbl<const double>* coef = st->coef;
    double acc = 0.0;
    int c = 0;
    for (; c + 16 <= ku; c += 16) acc = xupd_group<16>(V, a.ld, r, c, coef, acc);
    if (c + 8 <= ku) {
      acc = xupd_group<8>(V, a.ld, r, c, coef, acc);
      c += 8;
    }
    switch (ku - c) {
      case 1: acc = xupd_group<1>(V, a.ld, r, c, coef, acc); break;
      case 2: acc = xupd_group<2>(V, a.ld, r, c, coef, acc); break;
      case 3: acc = xupd_group<3>(V, a.ld, r, c, coef, acc); break;
      case 4: acc = xupd_group<4>(V, a.ld, r, c, coef, acc); break;
      case 5: acc = xupd_group<5>(V, a.ld, r, c, coef, acc); break;
      case 6: acc = xupd_group<6>(V, a.ld, r, c, coef, acc); break;
      case 7: acc = xupd_group<7>(V, a.ld, r, c, coef, acc); break;
      default: break;
    }
    if (a.t) G(a.t)[r] = acc;
    else __builtin_nontemporal_store(x[r] + acc, &x[r]);
  }
};

// ------------------------------------------------------------------ end of cycle
// Back substitution z = U(0:k,0:k)^{-1} g(0:k) for upper-triangular U in LDS (ld kLd),
// column-oriented, by wave 0 with wave-level synchronization; g is overwritten.
__device__ void wave_back_subst(const double* U, double* g, double* z, int k) {
  const int lane = threadIdx.x;
  for (int i = k - 1; i >= 0; --i) {
    const double zi = g[i] / U[i + i * kLd];  // every lane (g[i] is final)
    if (lane == 0) z[i] = zi;
    if (lane < i) g[lane] -= U[lane + i * kLd] * zi;
    wave_lds_sync();
  }
}

// One block.  Two-stage: stage 2 = CholQR of the kept columns, R2 = Chol(G2) (Fig. 5 with
// s_hat = m); then the projected least-squares problem in its Qhat form:
//   z = argmin || beta R2(1,1) e_1 - (R2 Hhat) z ||,
// which equals R2(1:m,1:m)^{-1} y for y = argmin || beta R2(1,1) e_1 - H y ||, H = R2 Hhat R2^{-1}
// (substitute y = R2 z), so neither R2^{-1} nor H is formed; x += Qhat z follows.  Other
// variants: z from the incremental Givens factorization of their Hessenberg matrix.  Then
// the iteration counters advance.
struct CycleEndBody {
  typedef TailArgs Args;
  static constexpr int kThreads = 256;
  static constexpr int kMinWaves = 1;
  static __device__ void run(const TailArgs& a, int bid, int nb);
};
__device__ void CycleEndBody::run(const TailArgs& a, int, int) {
  SmallState* st = Gp(a.st);  // (global, not flat, accesses)
  const int two_stage = a.two_stage;
  if (st->h.done || st->h.redo) return;
  constexpr int LL = kLdsLd;
  const int tid = threadIdx.x, nt = blockDim.x;
  __shared__ double sG[kLd * LL];
  __shared__ double sR[kLd * LL];
  __shared__ double sM[kLd * LL];
  __shared__ double sg[kLd + 1], sz[kLd];
  __shared__ int s_ku;
  if (tid == 0) s_ku = st->h.k_used;
  __syncthreads();
  int ku = s_ku;
  const int ritz = st->ritz_pending;
  double est = 0.0;
  if (two_stage && ku > 0) {
    int kb = ku + 1;
    // every global read up front, all in flight at once (one memory round trip instead of
    // one per loop trip): the upper triangle of G2 (kb x kb) into sR, Hhat (kb x ku) into sG
    __shared__ double sdiag[kLd];
    {
      static_assert(kThreads == 256, "16 entries per thread");
      constexpr int PER = kLd * kLd / kThreads;
      double g[PER], h[PER];
#pragma unroll
      for (int u = 0; u < PER; ++u) {
        const int idx = tid + kThreads * u, r = idx % kLd, c = idx / kLd;
        g[u] = (r <= c && c < kb) ? st->G2[r + c * kLd] : 0.0;
        h[u] = (r < kb && c < ku) ? st->Hh[r + c * kLd] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < PER; ++u) {
        const int idx = tid + kThreads * u, r = idx % kLd, c = idx / kLd;
        sR[r + c * LL] = g[u];
        sG[r + c * LL] = h[u];
        if (r == c) sdiag[r] = g[u];
      }
    }
    __syncthreads();
    // Cholesky of the upper triangle; a pivot d_j <= tol * G_jj truncates
    const int fail = lds_chol_upper_blk<LL>(sR, sdiag, st->pivot_tol, kb);
    if (fail >= 0) {  // keep the leading `fail` columns (rows 0..fail-1 of R are final)
      kb = fail;
      if (tid == 0) st->h.truncated += 1;
    }
    ku = kb - 1;
    if (ku > 0) {
      // sM = R2(0:kb,0:kb) Hhat(0:kb,0:ku): entries (ti + 16 m, tj + 16 q) per thread, the
      // sum over l in increasing order (terms outside l in [i, min(kb - 1, j + 1)] are exact
      // zeros)
      {
        const int ti = tid % 16, tj = tid / 16;
        double acc[4][4];
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
          for (int q = 0; q < 4; ++q) acc[m][q] = 0.0;
        for (int l = 0; l < kb; ++l) {
          double ra[4], hb[4];
#pragma unroll
          for (int m = 0; m < 4; ++m) {
            const int i = ti + 16 * m;
            ra[m] = (i <= l) ? sR[i + l * LL] : 0.0;
          }
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int j = tj + 16 * q;
            hb[q] = (j < ku && l <= j + 1) ? sG[l + j * LL] : 0.0;
          }
#pragma unroll
          for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[m][q] += ra[m] * hb[q];
        }
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int i = ti + 16 * m, j = tj + 16 * q;
            if (i < kb && j < ku) sM[i + j * LL] = acc[m][q];
          }
      }
      for (int i = tid; i <= kLd; i += nt) sg[i] = 0.0;
      __syncthreads();
      if (ritz) {  // for the Newton shifts: H(0:ku, 0:ku) = sM(0:ku, 0:ku) R2(0:ku, 0:ku)^{-1}
        for (int r = tid; r < ku; r += nt) {
          for (int j = 0; j < ku; ++j) {
            double v = sM[r + j * LL];
            for (int l = 0; l < j; ++l) v -= st->Wk[r + l * kLd] * sR[l + j * LL];
            st->Wk[r + j * kLd] = v / sR[j + j * LL];
          }
        }
        __syncthreads();
      }
      if (tid < kWave) {
        // wave 0: Givens QR of sM and back substitution.  Lane t keeps its column's running
        // top entry (row i after the rotations so far) in a register and reads row i + 1,
        // which no rotation has touched yet, from LDS; rotation i is formed by every lane
        // from lane i's entries; the rotated row i (final) goes to LDS
        const int lane = tid;
        const bool col = lane < ku;
        double x = col ? sM[lane * LL] : 0.0;
        double y = col ? sM[1 + lane * LL] : 0.0;
        double gi = st->beta * sR[0];  // the running right-hand side entry (every lane)
        double gl = 0.0, dl = 1.0;     // lane l: its final right-hand side and R(l, l)
        for (int i = 0; i < ku; ++i) {
          const double yn = (col && i + 2 <= ku) ? sM[(i + 2) + lane * LL] : 0.0;
          const double a = wave_bcast(x, i), b = wave_bcast(y, i);
          const double rho = hypot(a, b);
          double c = 1.0, s = 0.0;
          if (rho != 0.0) {
            const double ri = 1.0 / rho;
            c = a * ri;
            s = b * ri;
          }
          if (lane > i && col) {
            sM[i + lane * LL] = c * x + s * y;
            x = -s * x + c * y;
          }
          if (lane == i) {
            sM[i + i * LL] = rho;
            gl = c * gi;
            dl = rho;
          }
          gi = -s * gi;
          y = yn;
        }
        est = fabs(gi);
        // z = R^{-1} g: z_i = g_i / R(i, i), then g_l -= R(l, i) z_i for l < i
        wave_lds_sync();
        double z = 0.0;
        for (int i = ku - 1; i >= 0; --i) {
          const double zi = wave_bcast(gl, i) / wave_bcast(dl, i);
          if (lane == i) z = zi;
          if (lane < i) gl -= sM[lane + i * LL] * zi;
        }
        if (col) st->coef[lane] = z;
      }
    }
  } else if (!two_stage && ku > 0) {
    for (int i = tid; i < ku * ku; i += nt) {
      const int r = i % ku, c = i / ku;
      sM[r + c * kLd] = st->Rg[r + c * kLd];
    }
    for (int i = tid; i <= ku; i += nt) sg[i] = st->gg[i];
    __syncthreads();
    if (tid < kWave) {
      est = fabs(sg[ku]);
      wave_back_subst(sM, sg, sz, ku);
      for (int i = tid; i < ku; i += kWave) st->coef[i] = sz[i];
    }
  }
  __syncthreads();
  if (tid == 0) {
    st->h.k_used = ku > 0 ? ku : 0;
    st->h.iters += ku > 0 ? ku : 0;
    st->h.cycles += 1;
    st->h.est = est / st->bnorm;
  }
}

// ------------------------------------------------------------------ Leja-Ritz basis
// After a cycle end, while the request's Newton shifts are pending and the cycle kept at
// least s columns: the Ritz values of its k x k Hessenberg matrix (two-stage with
// s_hat = m: the one CycleEndBody formed in Wk; otherwise Hh, which holds H itself),
// their Leja ordering and the real-form parameters of the first s, which every later
// matrix-powers step reads.  One wave.  If the QR iteration does not converge the
// current basis stays.
struct RitzBody {
  typedef TailArgs Args;
  static constexpr int kThreads = kWave;
  static constexpr int kMinWaves = 1;
  static __device__ void run(const TailArgs& a, int bid, int nb);
};
struct WaveLdsSync {
  __device__ void operator()() const { wave_lds_sync(); }
};
__device__ void RitzBody::run(const TailArgs& a, int, int) {
  SmallState* st = Gp(a.st);  // (global, not flat, accesses)
  if (!st->ritz_pending || st->h.done || st->h.redo) return;
  const int k = st->h.k_used, s = st->s, lane = threadIdx.x;
  if (k < s) return;  // stays pending for the next cycle
  __shared__ double sH[kLd * kLd];
  __shared__ RitzScratch w;
  __shared__ double prm[3 * kMaxS];
  const double* src = a.two_stage ? st->Wk : st->Hh;
  for (int idx = lane; idx < k * k; idx += kWave) {
    const int i = idx % k, j = idx / k;
    sH[i + j * kLd] = (i <= j + 1) ? src[i + j * kLd] : 0.0;
  }
  wave_lds_sync();
  const int rc = ritz_newton(sH, k, s, st->glo, st->ghi, w, prm, prm + kMaxS, prm + 2 * kMaxS, lane, kWave,
                             WaveLdsSync());
  if (rc == 0) {
    for (int i = lane; i < s; i += kWave) {
      st->theta[i] = prm[i];
      st->tau[i] = prm[kMaxS + i];
      st->sigma[i] = prm[2 * kMaxS + i];
    }
  }
  if (lane == 0) {
    st->ritz_pending = 0;
    if (rc == 0) st->h.newton_from = (int32_t)st->h.cycles;
  }
}

// Stand-alone form for a given Hessenberg matrix (device, column-major, leading
// dimension ldh): out = [Leja-ordered Ritz values: real parts (k), imaginary parts (k);
// theta (s), tau (s), sigma (s); status (0 ok, 1 no convergence)].
__global__ __launch_bounds__(kWave) void ritz_newton_kernel(const double* H, int64_t ldh, int k, int s, double lo,
                                                           double hi, double* out) {
  __shared__ double sH[kLd * kLd];
  __shared__ RitzScratch w;
  __shared__ double prm[3 * kMaxS];
  const int lane = threadIdx.x;
  for (int idx = lane; idx < k * k; idx += kWave) {
    const int i = idx % k, j = idx / k;
    sH[i + j * kLd] = (i <= j + 1) ? H[i + j * ldh] : 0.0;
  }
  wave_lds_sync();
  const int rc = ritz_newton(sH, k, s, lo, hi, w, prm, prm + kMaxS, prm + 2 * kMaxS, lane, kWave, WaveLdsSync());
  if (rc == 0) {
    for (int i = lane; i < k; i += kWave) {
      out[i] = w.zr[i];
      out[k + i] = w.zi[i];
    }
    for (int i = lane; i < s; i += kWave) {
      out[2 * k + i] = prm[i];
      out[2 * k + s + i] = prm[kMaxS + i];
      out[2 * k + 2 * s + i] = prm[2 * kMaxS + i];
    }
  }
  if (lane == 0) out[2 * k + 3 * s] = rc == 0 ? 0.0 : 1.0;
}

// ------------------------------------------------------------------ big-panel stage 2
// Two-stage with big panels (s_hat < m), at the end of big panel [b0, b1) of the cycle:
// stage 2 = BCGS-PIP of the big panel against the final columns 0..b0-1 (Fig. 5), from
// the stage-2 Gram block columns the panels' reductions accumulated in st->G2:
//   P2 = G2(:b0, b0:b1),  R2 = Chol(G2(b0:b1, b0:b1) - P2^T P2),  T2 = R2^{-1},
//   Bs(:b1, b0:b1) = [-P2 T2; T2]  (the apply launches then form Y(:, b0:b1) <- Y(:, :b1) Bs).
// The basis change Y_old = Y_new M (M = I but M(:b0, b0:b1) = P2, M(b0:b1, b0:b1) = R2)
// transforms the Hessenberg matrix, H <- M H M(:b1-1, :b1-1)^{-1}; the least-squares
// problem over the final columns is refactored by Givens from scratch and the residual
// checked (the cycle stops after this big panel when it is below tol).  A stage-2 pivot
// failure at column f keeps the big panel's first f columns and ends the cycle.
struct S2Args {
  SmallState* st;
  int32_t b0, b1, panel;
  int32_t standalone;  // stand-alone orthogonalization: R-factor update instead of H and Givens
};
struct Stage2Body {
  typedef S2Args Args;
  static constexpr int kThreads = 256;
  static constexpr int kMinWaves = 1;
  static __device__ void run(const S2Args& a, int bid, int nb);
};
__device__ void Stage2Body::run(const S2Args& a, int, int) {
  SmallState* st = Gp(a.st);  // (global, not flat, accesses)
  if (st->h.done || a.panel > st->h.stop_panel) return;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int b0 = a.b0, w = a.b1 - a.b0;
  __shared__ double sG[kLd * kLd];   // w x w Gram, then reused for M H
  __shared__ double sR[kLd * kLd];   // R2, then H
  __shared__ double sM[kLd * kLd];   // T2, then M
  __shared__ double sref[kLd];
  __shared__ int s_kept;
  // G = Gb - P2^T P2 (G2 holds the upper triangle)
  for (int idx = tid; idx < w * w; idx += nt) {
    const int i = idx % w, j = idx / w;
    const int r = b0 + min(i, j), c = b0 + max(i, j);
    double v = st->G2[r + c * kLd];
    if (i == j) sref[i] = v;
    for (int l = 0; l < b0; ++l) v -= st->G2[l + (b0 + i) * kLd] * st->G2[l + (b0 + j) * kLd];
    sG[i + j * kLd] = v;
  }
  __syncthreads();
  const int f = block_chol_upper(sG, kLd, sR, kLd, w, sref, st->pivot_tol);
  if (tid == 0) s_kept = f < 0 ? w : f;
  __syncthreads();
  if (a.standalone && f >= 0) {  // stand-alone: the big panel's Gram is not positive definite
    if (tid == 0) {
      st->h.status = 2;
      st->h.done = 1;
      st->fail_col = b0 + f;
    }
    return;
  }
  const int kept = s_kept;
  if (kept == 0) {  // nothing of this big panel survives: keep the final columns before it
    if (tid == 0) {
      st->h.stop_panel = a.panel - 1;
      st->h.k_used = b0 > 0 ? b0 - 1 : 0;
      st->h.truncated += 1;
    }
    return;
  }
  block_tri_inv_upper(sR, kLd, sM, kLd, kept);  // T2
  __syncthreads();
  const int e1 = b0 + kept, b1 = a.b1;
  // Bs(:b1, b0:b1) in full (the apply launches read every row below their chunk's end):
  // rows < b0 = -P2 T2, rows b0 .. e1-1 = T2, rows from e1 on and the columns beyond kept zero
  for (int idx = tid; idx < b1 * w; idx += nt) {
    const int r = idx % b1, j = idx / b1;
    double v = 0.0;
    if (j < kept && r < e1) {
      if (r < b0) {
        for (int l = 0; l <= j; ++l) v -= st->G2[r + (b0 + l) * kLd] * sM[l + j * kLd];
      } else if (r - b0 <= j) {
        v = sM[(r - b0) + j * kLd];
      }
    }
    st->Bs[r + (b0 + j) * kLd] = v;
  }
  __syncthreads();
  if (a.standalone) {
    // the R factor X = Y Rh of the columns so far: Y(:, b0:b1) = Q(:, :b0) P2 + Q(:, b0:b1) R2,
    // so Rh(:b0, b0:b1) += P2 Rh(b0:b1, b0:b1) and Rh(b0:b1, b0:b1) = R2 Rh(b0:b1, b0:b1)
    // (the big panel's rows have no entries left of column b0); Rb in LDS first (sG is free)
    for (int idx = tid; idx < w * w; idx += nt) {
      const int i = idx % w, j = idx / w;
      sG[i + j * kLd] = i <= j ? st->Hh[(b0 + i) + (b0 + j) * kLd] : 0.0;
    }
    __syncthreads();
    for (int idx = tid; idx < b1 * w; idx += nt) {
      const int r = idx % b1, j = idx / b1;
      double v;
      if (r < b0) {
        v = st->Hh[r + (b0 + j) * kLd];
        for (int l = 0; l <= j; ++l) v += st->G2[r + (b0 + l) * kLd] * sG[l + j * kLd];
      } else {
        const int i = r - b0;
        v = 0.0;
        for (int l = i; l <= j; ++l) v += sR[i + l * kLd] * sG[l + j * kLd];
      }
      st->Hh[r + (b0 + j) * kLd] = v;
    }
    __syncthreads();
    return;
  }
  // M (e1 x e1) into sM; X = M H(:e1, :c) into sG; H(:e1, :c) = X M(:c, :c)^{-1}
  const int c = e1 - 1;
  for (int idx = tid; idx < e1 * e1; idx += nt) {
    const int r = idx % e1, j = idx / e1;
    double v = (r == j) ? 1.0 : 0.0;
    if (j >= b0) {
      if (r < b0) v = st->G2[r + j * kLd];                       // P2
      else v = (r <= j) ? sR[(r - b0) + (j - b0) * kLd] : 0.0;   // R2
    }
    sM[r + j * kLd] = v;
  }
  __syncthreads();
  for (int idx = tid; idx < e1 * c; idx += nt) {
    const int r = idx % e1, j = idx / e1;
    double v = 0.0;
    for (int l = r; l <= min(e1 - 1, j + 1); ++l) v += sM[r + l * kLd] * st->Hh[l + j * kLd];
    sG[r + j * kLd] = v;
  }
  __syncthreads();
  // right solve by the upper-triangular M(:c, :c), one row per thread
  for (int r = tid; r < e1; r += nt) {
    for (int j = 0; j < c; ++j) {
      double v = sG[r + j * kLd];
      for (int l = 0; l < j; ++l) v -= sR[r + l * kLd] * sM[l + j * kLd];
      sR[r + j * kLd] = v / sM[j + j * kLd];
    }
  }
  __syncthreads();
  for (int idx = tid; idx < e1 * c; idx += nt) {
    const int r = idx % e1, j = idx / e1;
    st->Hh[r + j * kLd] = (r <= j + 1) ? sR[r + j * kLd] : 0.0;
  }
  if (tid == 0 && b0 == 0) st->gscale = st->beta * sM[0];
  __syncthreads();
  // least squares over the final columns 0..c-1, refactored from scratch
  for (int i = tid; i <= kLd; i += nt) st->gg[i] = (i == 0) ? st->gscale : 0.0;
  __syncthreads();
  givens_append(st, st->Hh, 0, c);
  if (tid == 0) {
    if (kept < w) {
      st->h.stop_panel = a.panel;
      st->h.k_used = c;
      st->h.truncated += 1;
    } else if (c < st->m && fabs(st->gg[c]) <= st->tol * st->bnorm) {
      st->h.stop_panel = a.panel;
      st->h.k_used = c;
    }
  }
  __syncthreads();
}

// ------------------------------------------------------------------ stand-alone ortho
// Stage 2 of the stand-alone two-stage scheme: R2 = Chol(G2), Rinv = R2^{-1} (st->Wk),
// R = R2 R1 with R1 the stage-1 factor in st->Hh (into st->G2).  One block of 256 threads;
// every small matrix in LDS, each step parallel over a 16 x 16 thread grid.
__global__ __launch_bounds__(256) void sa_stage2_kernel(SmallState* st, int k) {
  if (st->h.done) return;
  constexpr int LL = kLdsLd;
  const int tid = threadIdx.x, nt = blockDim.x;
  __shared__ double sR[kLd * LL];
  __shared__ double sX[kLd * LL];
  __shared__ double sR1[kLd * LL];
  __shared__ double sdiag[kLd];
  {  // every global read up front, all in flight at once
    constexpr int PER = kLd * kLd / 256;
    double g[PER], h[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int idx = tid + 256 * u, r = idx % kLd, c = idx / kLd;
      const bool in = r <= c && c < k;
      g[u] = in ? st->G2[r + c * kLd] : 0.0;
      h[u] = in ? st->Hh[r + c * kLd] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int idx = tid + 256 * u, r = idx % kLd, c = idx / kLd;
      sR[r + c * LL] = g[u];
      sR1[r + c * LL] = h[u];
      if (r == c) sdiag[r] = g[u];
    }
  }
  __syncthreads();
  if (lds_chol_upper_blk<LL>(sR, sdiag, 0.0, k) >= 0) {
    if (tid == 0) {
      st->h.status = 2;
      st->h.done = 1;
    }
    return;
  }
  lds_tri_inv_upper_blk<LL>(sR, sX, k);
  for (int c = tid / kWave; c < k; c += nt / kWave)
    for (int r = tid % kWave; r < k; r += kWave) st->Wk[r + c * kLd] = sX[r + c * LL];
  lds_trmm_upper256<LL>(sR, sR1, G(st->G2), k);
}

// Copy a k x k upper-triangular factor (ld kLd, from src) to the caller's R (ldr).
__global__ __launch_bounds__(256) void copy_r_kernel(const SmallState* st, int which, int k,
                                                     double* R, int ldr) {
  const double* src = which == 0 ? st->Hh : st->G2;
  for (int idx = threadIdx.x; idx < k * k; idx += blockDim.x) {
    int i = idx % k, j = idx / k;
    R[i + (int64_t)j * ldr] = (i <= j) ? src[i + j * kLd] : 0.0;
  }
}

// The factors of one stand-alone panel (columns k .. k+s-1 against the k before them) from
// the R assembly in st->Hh: P = Hh(0:k, k:k+s) (ldp), R = Hh(k:k+s, k:k+s) (ldr, strictly
// lower part 0).  Returns at entry after a breakdown (nothing written).
__global__ __launch_bounds__(256) void copy_panel_kernel(const SmallState* st, int k, int s, double* P, int ldp,
                                                         double* R, int ldr) {
  if (st->h.done) return;
  for (int idx = threadIdx.x; idx < k * s; idx += blockDim.x) {
    const int i = idx % k, j = idx / k;
    P[i + (int64_t)j * ldp] = st->Hh[i + (k + j) * kLd];
  }
  for (int idx = threadIdx.x; idx < s * s; idx += blockDim.x) {
    const int i = idx % s, j = idx / s;
    R[i + (int64_t)j * ldr] = i <= j ? st->Hh[(k + i) + (k + j) * kLd] : 0.0;
  }
}

// ||I - G||_F for the k x k Gram in st->Wk (upper triangle valid) -> st->Wk[kLd*kLd-1].
__global__ __launch_bounds__(256) void orth_err_kernel(SmallState* st, int k) {
  __shared__ double s[256];
  double acc = 0.0;
  for (int idx = threadIdx.x; idx < k * k; idx += blockDim.x) {
    int i = idx % k, j = idx / k;
    double g = (i <= j) ? st->Wk[i + j * kLd] : st->Wk[j + i * kLd];
    double e = ((i == j) ? 1.0 : 0.0) - g;
    acc += e * e;
  }
  s[threadIdx.x] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int i = 0; i < (int)blockDim.x; ++i) t += s[i];
    st->beta = sqrt(t);
  }
}

}  // namespace tsg
