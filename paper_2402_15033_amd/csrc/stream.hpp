// Lean streaming kernels of the panel steps:
//   gram_kernel   -- the reduction  G = V(:, 0:ncol)^T V(:, ncol-nz : ncol)  (no update)
//   update_kernel -- the update     W <- (W - Q P) T  in place            (no reduction)
// The fused kernel in panel.hpp (update + Gram of its own output in one pass) is kept
// for the steps whose next reduction needs exactly the columns just written.
#pragma once

#include "panel.hpp"

namespace tsg {

// Reduction over the first ncol = k + sw basis columns (Q = V(:,0:k), W = V(:,wcol:wcol+sw)),
// against the last nz of them (nz = nprev + sw: the previous panel's nprev columns -- their
// block column of the stage-2 Gram -- and the panel W).  Block = NW waves, column c of the
// loaded set is owned by wave c % NW for the whole launch; the nz right-hand columns are
// exchanged through a double-buffered LDS tile (one barrier per batch); the next batch's
// loads are issued before the current batch is processed.  Partials: ncol x nz per block.
template <typename T, int NZ, int NW, int RPL>
__global__ __launch_bounds__(NW * kWave) void gram_kernel(PanelArgs a) {
  SmallState* st = a.st;
  if (gated_off(a, st)) return;
  constexpr int SL = kMaxCols / NW;  // column slots per wave
  constexpr int BR = kWave * RPL;
  const int lane = threadIdx.x & (kWave - 1);
  const int wv = threadIdx.x / kWave;
  const int k = a.k, ncol = a.k + a.sw, nz = a.nz, z0 = ncol - nz;
  const T* __restrict__ V = reinterpret_cast<const T*>(a.V);
  const int64_t ld = a.ld;
  __shared__ T lz[2][NZ][BR];

  T acc[SL][NZ];
#pragma unroll
  for (int sl = 0; sl < SL; ++sl)
#pragma unroll
    for (int z = 0; z < NZ; ++z) acc[sl][z] = (T)0;

  const int64_t rb = (int64_t)blockIdx.x * a.rows_per_block;
  const int64_t re = min(a.n, rb + a.rows_per_block);
  int64_t colof[SL];
#pragma unroll
  for (int sl = 0; sl < SL; ++sl) {
    const int c = wv + NW * sl;
    colof[sl] = ((c < k) ? (int64_t)c : (int64_t)a.wcol + (c - k)) * ld;
  }
  T v[SL][RPL], vn[SL][RPL];
  auto load = [&](T (&dst)[SL][RPL], int64_t r0) {
#pragma unroll
    for (int sl = 0; sl < SL; ++sl) {
      const int c = wv + NW * sl;
#pragma unroll
      for (int t = 0; t < RPL; ++t) {
        const int64_t row = r0 + lane + kWave * t;
        dst[sl][t] = (c < ncol && row < re) ? V[colof[sl] + row] : (T)0;
      }
    }
  };
  load(v, rb);
  int buf = 0;
  for (int64_t r0 = rb; r0 < re; r0 += BR) {
    if (r0 + BR < re) load(vn, r0 + BR);
#pragma unroll
    for (int sl = 0; sl < SL; ++sl) {
      const int c = wv + NW * sl;
      if (c >= z0 && c < ncol) {
#pragma unroll
        for (int t = 0; t < RPL; ++t) lz[buf][c - z0][lane + kWave * t] = v[sl][t];
      }
    }
    __syncthreads();
#pragma unroll
    for (int z = 0; z < NZ; ++z) {
      if (z < nz) {
        T zv[RPL];
#pragma unroll
        for (int t = 0; t < RPL; ++t) zv[t] = lz[buf][z][lane + kWave * t];
#pragma unroll
        for (int sl = 0; sl < SL; ++sl) {
#pragma unroll
          for (int t = 0; t < RPL; ++t) acc[sl][z] += v[sl][t] * zv[t];
        }
      }
    }
#pragma unroll
    for (int sl = 0; sl < SL; ++sl)
#pragma unroll
      for (int t = 0; t < RPL; ++t) v[sl][t] = vn[sl][t];
    buf ^= 1;
  }
  double* part = a.part1 + (size_t)blockIdx.x * ncol * nz;
#pragma unroll
  for (int sl = 0; sl < SL; ++sl) {
    const int c = wv + NW * sl;
    if (c < ncol) {
#pragma unroll
      for (int z = 0; z < NZ; ++z) {
        if (z < nz) {
          T sum = wave_sum(acc[sl][z]);
          if (lane == 0) part[c * nz + z] = (double)sum;
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------------------
// The same reduction G = V(:, 0:ncol)^T V(:, ncol-nz:ncol) on the FP64 matrix cores
// (v_mfma_f64_16x16x4f64: D(16x16) += A(16x4) B(4x16); lane l holds A(l%16, l/16),
// B(l/16, l%16) and D(l/16 + 4r, l%16) in accumulator register r -- the layout was
// measured on gfx950 with a one-wave probe).
//   A = V(rows, tile columns)^T, B = V(rows, Z columns): the K dimension is the rows.
// A block of 8 waves stages batches of BR = 64 * floor(64 / ncol) rows of all ncol <= 64
// columns in LDS (column-major, row stride BR + 1; double-buffered, one barrier per batch),
// loading the next two batches into registers while the matrix cores consume the current
// one.  The K-steps (4 rows each) of a batch are dealt to the waves round-robin; every
// wave accumulates all MT 16-column tiles: 4 MT doubles of accumulators per lane instead
// of one copy of every Gram entry per lane, so occupancy stays at 2 blocks per CU.  The 8
// waves' tiles are summed in LDS in wave order at the end.  Requires nz <= 16.
typedef double dbl4 __attribute__((ext_vector_type(4)));

constexpr int kMfmaTile = kMaxCols * (kWave + 1);  // doubles per LDS tile buffer

template <int MT>
__global__ __launch_bounds__(512) void gram_mfma_kernel(PanelArgs a) {
  SmallState* st = a.st;
  if (gated_off(a, st)) return;
  constexpr int NW = 8, SL = 8;
  const int lane = threadIdx.x & (kWave - 1);
  const int wv = threadIdx.x / kWave;
  const int k = a.k, ncol = a.k + a.sw, nz = a.nz, z0 = ncol - nz;
  // a batch is RB chunks of 64 rows of all ncol columns (ncol * RB <= 64 load items, so
  // narrow reductions still keep 64 wave loads in flight); LDS row stride BR + 1
  const int RB = kMaxCols / ncol;
  const int BR = kWave * RB, LDT = BR + 1;
  const int items = ncol * RB;
  const double* __restrict__ V = reinterpret_cast<const double*>(a.V);
  const int64_t ld = a.ld;
  __shared__ double lt[2][kMfmaTile];

  const int64_t rb = (int64_t)blockIdx.x * a.rows_per_block;
  const int64_t re = min(a.n, rb + a.rows_per_block);
  // load item t = wv + 8 sl: column c = t % ncol, 64-row chunk t / ncol of the batch
  int64_t colbase[SL];
  int rowoff[SL], ldsof[SL];
#pragma unroll
  for (int sl = 0; sl < SL; ++sl) {
    const int t = wv + NW * sl;
    const int c = t % ncol, chunk = t / ncol;
    colbase[sl] = ((c < k) ? (int64_t)c : (int64_t)a.wcol + (c - k)) * ld;
    rowoff[sl] = chunk * kWave;
    ldsof[sl] = c * LDT + chunk * kWave;
  }
  double v[SL], vn[SL], vnn[SL];
  auto load = [&](double (&dst)[SL], int64_t r0) {
#pragma unroll
    for (int sl = 0; sl < SL; ++sl) {
      const int t = wv + NW * sl;
      const int64_t row = r0 + rowoff[sl] + lane;
      dst[sl] = (t < items && row < re) ? V[colbase[sl] + row] : 0.0;
    }
  };
  dbl4 acc[MT];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt) acc[mt] = dbl4{0.0, 0.0, 0.0, 0.0};
  const int li = lane & 15, lk = lane >> 4;
  const bool zok = li < nz;
  const int ksteps = BR / 4;  // K-steps of 4 rows per batch, dealt to the waves round-robin
  // prefetch depth 2: batches r0+BR and r0+2BR are in flight while r0 is consumed
  load(v, rb);
  if (rb + BR < re) load(vn, rb + BR);
  int buf = 0;
  for (int64_t r0 = rb; r0 < re; r0 += BR) {
    if (r0 + 2 * BR < re) load(vnn, r0 + 2 * BR);
    double* T = lt[buf];
#pragma unroll
    for (int sl = 0; sl < SL; ++sl) {
      const int t = wv + NW * sl;
      if (t < items) T[ldsof[sl] + lane] = v[sl];
    }
    __syncthreads();
    for (int ks = wv; ks < ksteps; ks += NW) {
      const int row = ks * 4 + lk;
      const double bv = zok ? T[(z0 + li) * LDT + row] : 0.0;
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        const int c = mt * 16 + li;
        const double av = (c < ncol) ? T[c * LDT + row] : 0.0;
        acc[mt] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[mt], 0, 0, 0);
      }
    }
#pragma unroll
    for (int sl = 0; sl < SL; ++sl) {
      v[sl] = vn[sl];
      vn[sl] = vnn[sl];
    }
    buf ^= 1;
  }
  __syncthreads();
  // sum the 8 waves' partial tiles in wave order: red[w][c][z], c < 16 MT, z < 16
  double* red = &lt[0][0];  // 8 x 64 x 16 doubles = 64 KiB fits in the two tiles
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int c = mt * 16 + lk + 4 * r;
      red[(wv * kMaxCols + c) * 16 + li] = acc[mt][r];
    }
  __syncthreads();
  double* part = a.part1 + (size_t)blockIdx.x * ncol * nz;
  for (int e = threadIdx.x; e < ncol * 16; e += blockDim.x) {
    const int c = e / 16, z = e % 16;
    if (z < nz) {
      double sum = 0.0;
#pragma unroll
      for (int w = 0; w < NW; ++w) sum += red[(w * kMaxCols + c) * 16 + z];
      part[c * nz + z] = sum;
    }
  }
}

// W <- (W - Q P) T in place (PF_HAS_P / PF_HAS_T), one row per thread: every lane reads
// its row of the k + sw columns (each wave access is a coalesced 64-row segment of one
// column), P and T are uniform (scalar loads).  No LDS, no barrier, high occupancy.
template <typename T, int S>
__global__ __launch_bounds__(256) void update_kernel(PanelArgs a) {
  const SmallState* st = a.st;
  if (gated_off(a, st)) return;
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= a.n) return;
  const int k = a.k, sw = a.sw;
  const bool hasP = a.flags & PF_HAS_P;
  const bool hasT = (a.flags & PF_HAS_T) && !st->identity_t;
  T* __restrict__ V = reinterpret_cast<T*>(a.V);
  const int64_t ld = a.ld;
  T* W = V + (int64_t)a.wcol * ld + r;
  T y[S];
#pragma unroll
  for (int j = 0; j < S; ++j) y[j] = (j < sw) ? W[(int64_t)j * ld] : (T)0;
  if (hasP) {
    const double* P = st->Pcur;
#pragma unroll 8
    for (int c = 0; c < k; ++c) {
      const T qc = V[(int64_t)c * ld + r];
#pragma unroll
      for (int j = 0; j < S; ++j) y[j] -= qc * (T)P[c + j * kLd];
    }
  }
  if (hasT) {
    const double* Tm = st->Tcur;
#pragma unroll
    for (int j = S - 1; j >= 0; --j) {
      T v = (T)0;
#pragma unroll
      for (int i = 0; i <= j; ++i) v += y[i] * (T)Tm[i + j * kMaxS];
      y[j] = v;
    }
  }
#pragma unroll
  for (int j = 0; j < S; ++j)
    if (j < sw) W[(int64_t)j * ld] = y[j];
}

}  // namespace tsg
