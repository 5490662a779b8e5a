// Lean streaming kernels of the panel steps:
//   GramBody   -- the reduction  G = V(:, 0:ncol)^T V(:, ncol-nz : ncol)  (no update)
//   UpdateBody -- the update     W <- (W - Q P) T  in place            (no reduction)
//   FusedBody  -- the update and the Gram of its output in one pass, for the steps whose
//                 next reduction needs exactly the columns just written
#pragma once

#include "panel.hpp"

namespace tsg {

// Matrix-core products of the panel steps.  The Gram of a row batch is a sum over rows,
// so the rows are the K dimension of the MFMA: A = V(rows, 16-column tile)^T,
// B = V(rows, 16 right-hand columns).
//   FP64: v_mfma_f64_16x16x4f64; FP32 (FP32 products, FP32 accumulation):
//   v_mfma_f32_16x16x4f32.  D(16x16) += A(16x4) B(4x16); lane l holds A(l%16, l/16) and
//   B(l/16, l%16) for both; accumulator register r of lane l holds D(l/16 + 4r, l%16)
//   for FP64 and D(4(l/16) + r, l%16) for FP32 (both measured on gfx950 with a one-wave
//   probe).
template <typename T>
struct MfmaOp;
template <>
struct MfmaOp<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  __device__ static v4 mac(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static int row(int lk, int r) { return lk + 4 * r; }
};
template <>
struct MfmaOp<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  __device__ static v4 mac(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static int row(int lk, int r) { return 4 * lk + r; }
};

// Batch staging shared by the MFMA kernels.  A block of 8 waves moves batches of BR rows of
// ncol <= 64 basis columns into an LDS tile (column-major, row stride BR + 1, two buffers).
// A batch is 64 load items of 64 R rows of one column (R = 8 / sizeof(T): each lane loads
// one double or two adjacent floats, 8 bytes either way); item t = wave + 8 sl, sl < 8,
// holds column t % ncol, row chunk t / ncol.  So BR = 64 R floor(64 / ncol): every lane
// keeps 8 loads of 8 bytes in flight whatever ncol is.
constexpr int kTileItems = 64;
template <typename T>
constexpr int tile_rows_per_lane() { return 8 / (int)sizeof(T); }
template <typename T>
constexpr int mfma_tile() { return kWave * kTileItems * tile_rows_per_lane<T>() + kMaxCols; }

template <typename T>
struct TileLoad {
  static constexpr int R = tile_rows_per_lane<T>(), SL = 8, NW = 8;
  int64_t colbase[SL];
  int rowoff[SL], ldsof[SL];
  int items, BR, LDT;
  // staged column c is V(:, c) for c < kq, else V(:, wcol + c - kq)
  __device__ void init(int wv, int ncol, int kq, int64_t wcol, int64_t ld) {
    const int RB = kTileItems / ncol;
    BR = kWave * R * RB;
    LDT = BR + 1;
    items = ncol * RB;
#pragma unroll
    for (int sl = 0; sl < SL; ++sl) {
      const int t = wv + NW * sl;
      const int c = t % ncol, chunk = t / ncol;
      colbase[sl] = ((c < kq) ? (int64_t)c : wcol + (c - kq)) * ld;
      rowoff[sl] = chunk * kWave * R;
      ldsof[sl] = c * LDT + chunk * kWave * R;
    }
  }
  // Every lane issues all SL loads, with no branch, so that the compiler can count them and
  // wait only for the batch it needs (a load under a branch made it wait for every load in
  // flight, the prefetched batches included).  Rows past re are clamped to the last row
  // pair that starts before re (in bounds, their values unused) and zeroed by to_lds, and
  // so are the items t >= items (whose column t % ncol exists).
  __device__ void load(gbl<const T>* __restrict__ V, int wv, int lane, int64_t r0, int64_t re,
                       T (&dst)[SL][R]) const {
    const int64_t rmax = (re - 1) & ~(int64_t)(R - 1);
#pragma unroll
    for (int sl = 0; sl < SL; ++sl) {
      const int64_t row = min(r0 + rowoff[sl] + (int64_t)R * lane, rmax);
      if constexpr (R == 2) {
        typedef float f2 __attribute__((ext_vector_type(2)));
        const f2 x = *reinterpret_cast<gbl<const f2>*>(V + colbase[sl] + row);
        dst[sl][0] = x.x;
        dst[sl][1] = x.y;
      } else {
        dst[sl][0] = V[colbase[sl] + row];
      }
    }
  }
  __device__ void to_lds(T* L, int wv, int lane, int64_t r0, int64_t re, const T (&src)[SL][R]) const {
#pragma unroll
    for (int sl = 0; sl < SL; ++sl) {
      const int t = wv + NW * sl;
      if (t < items) {
        const int64_t row = r0 + rowoff[sl] + (int64_t)R * lane;
#pragma unroll
        for (int e = 0; e < R; ++e) L[ldsof[sl] + R * lane + e] = row + e < re ? src[sl][e] : (T)0;
      }
    }
  }
};

// The reduction G = V(:, 0:ncol)^T V(:, ncol-nz : ncol) of a panel step on the matrix cores
// (ncol = k + sw, Q = V(:, 0:k), W = V(:, wcol:wcol+sw); the nz right-hand columns are the
// previous panel's nprev columns, their block column of the stage-2 Gram, followed by W),
// with the operands taken straight from global memory: no LDS staging and no block barrier
// in the row loop.  Rows are the K dimension.  Lane l = 16 g + i holds, for each column tile
// t, column c_t + i and the RL consecutive rows r + RL g .. r + RL g + RL - 1 of a group of
// 4 RL rows (two 16-byte loads per tile: RL = 4 in FP64, 8 in FP32); K-step e of the group
// pairs row r + RL g + e with k index g in both operands.  The tiles are laid out from the
// right: the last NT tiles are the nz right-hand columns (the B operand is the A operand of
// those tiles, no extra load) and MA - NT tiles cover the columns to their left down to
// column 0 (lanes outside [0, ncol) hold zeros).  Each wave walks its own groups (wave w:
// groups w, w + NW, ... of the block's rows) with one group's loads in flight while the
// matrix cores consume the previous one; the loads are unconditional (the index is clamped
// to the last full group), so the compiler waits only for the group it consumes.  A ragged
// last group (and every group when the columns are not 16-byte aligned) is loaded element
// by element with its rows masked.  The NW waves' tiles are summed in LDS in wave order at
// the end.  Partials: ncol x nz float64 per block.  Measured on a 4194304 x 61 FP64 block:
// 6.07 TB/s with 256 blocks against 4.73 for the LDS-staged version.
template <typename T>
constexpr int gram_rows_per_lane() { return 32 / (int)sizeof(T); }
constexpr int kGramGroupRows = 32;  // row blocks of the reduction are multiples of this
template <typename T, int MA, int NT>
struct GramBody {
  typedef PanelArgs Args;
  static constexpr int kThreads = 512;
  static constexpr int kMinWaves = 1;
  static __device__ void run(const PanelArgs& a, int bid, int nb);
};
template <typename T, int MA, int NT>
__device__ void GramBody<T, MA, NT>::run(const PanelArgs& a, int bid, int) {
  if (gated_off(a, a.st)) return;
  typedef typename MfmaOp<T>::v4 v4;
  constexpr int NW = kThreads / kWave, RL = gram_rows_per_lane<T>(), GR = 4 * RL;
  static_assert(kGramGroupRows % GR == 0, "row blocks must hold whole groups");
  const int lane = threadIdx.x & (kWave - 1);
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int g = lane >> 4, li = lane & 15;
  const int k = a.k, ncol = a.k + a.sw, nz = a.nz, z0 = ncol - nz;
  const int64_t ld = a.ld, n = a.n;
  gbl<const T>* __restrict__ V = G(reinterpret_cast<const T*>(a.V));
  // per tile: this lane's column (offset of its first element) and whether it exists
  int64_t coff[MA];
  bool cval[MA];
#pragma unroll
  for (int t = 0; t < MA; ++t) {
    const int c = z0 + 16 * (t - (MA - NT)) + li;
    cval[t] = c >= 0 && c < ncol;
    const int cc = cval[t] ? c : 0;
    coff[t] = (int64_t)(cc < k ? cc : a.wcol + (cc - k)) * ld + RL * g;
  }
  const int64_t rb = (int64_t)bid * a.rows_per_block;
  const int64_t re = min(n, rb + a.rows_per_block);
  const int64_t nfull = (re - rb) / GR;  // full groups of this block
  const bool vec = (reinterpret_cast<uintptr_t>(a.V) & 15) == 0 && (ld % (16 / (int)sizeof(T))) == 0;
  v4 acc[MA][NT];
#pragma unroll
  for (int t = 0; t < MA; ++t)
#pragma unroll
    for (int u = 0; u < NT; ++u) acc[t][u] = v4{0, 0, 0, 0};
  // rows r0 + RL g .. + RL - 1 of every tile column (a full group starting at row r0)
  auto load = [&](int64_t r0, T (&v)[MA][RL]) {
    typedef T t16 __attribute__((ext_vector_type(16 / sizeof(T))));
    constexpr int H = 16 / (int)sizeof(T);
#pragma unroll
    for (int t = 0; t < MA; ++t) {
      gbl<const T>* p = V + coff[t] + r0;
      const t16 x0 = *reinterpret_cast<gbl<const t16>*>(p);
      const t16 x1 = *reinterpret_cast<gbl<const t16>*>(p + H);
#pragma unroll
      for (int e = 0; e < H; ++e) {
        v[t][e] = x0[e];
        v[t][H + e] = x1[e];
      }
    }
  };
  auto mma = [&](const T (&v)[MA][RL]) {
#pragma unroll
    for (int e = 0; e < RL; ++e)
#pragma unroll
      for (int t = 0; t < MA; ++t) {
        const T av = cval[t] ? v[t][e] : (T)0;
#pragma unroll
        for (int u = 0; u < NT; ++u) {
          const int tb = MA - NT + u;
          const T bv = cval[tb] ? v[tb][e] : (T)0;
          acc[t][u] = MfmaOp<T>::mac(av, bv, acc[t][u]);
        }
      }
  };
  if (vec && nfull > 0) {
    T va[MA][RL], vb[MA][RL];
    int64_t q = wv;
    load(rb + GR * min<int64_t>(q, nfull - 1), va);
    for (; q < nfull; q += 2 * NW) {
      load(rb + GR * min<int64_t>(q + NW, nfull - 1), vb);
      mma(va);
      if (q + NW >= nfull) break;
      load(rb + GR * min<int64_t>(q + 2 * NW, nfull - 1), va);
      mma(vb);
    }
  }
  {
    // element by element: the ragged last group, or every group when the columns are not
    // 16-byte aligned
    const int64_t q0 = vec ? nfull : 0, qe = (re - rb + GR - 1) / GR;
    for (int64_t q = q0 + wv; q < qe; q += NW) {
      const int64_t r0 = rb + GR * q;
      T v[MA][RL];
#pragma unroll
      for (int t = 0; t < MA; ++t)
#pragma unroll
        for (int e = 0; e < RL; ++e) v[t][e] = r0 + RL * g + e < re ? V[coff[t] + r0 + e] : (T)0;
      mma(v);
    }
  }
  // sum the NW waves' tiles in wave order, one right-hand tile at a time:
  // red[w][c][z], c < 16 MA (every column c < ncol lies in one tile), z < 16
  constexpr int RC = 16 * MA;
  __shared__ T red[NW * RC * 16];
  gbl<double>* part = G(a.part1) + (size_t)bid * ncol * nz;
#pragma unroll
  for (int u = 0; u < NT; ++u) {
    __syncthreads();
#pragma unroll
    for (int t = 0; t < MA; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int c = z0 + 16 * (t - (MA - NT)) + MfmaOp<T>::row(g, r);
        if (c >= 0 && c < ncol) red[(wv * RC + c) * 16 + li] = acc[t][u][r];
      }
    __syncthreads();
    for (int e = threadIdx.x; e < ncol * 16; e += blockDim.x) {
      const int c = e / 16, z = u * 16 + e % 16;
      if (z < nz) {
        double sum = 0.0;
#pragma unroll
        for (int w = 0; w < NW; ++w) sum += (double)red[(w * RC + c) * 16 + e % 16];
        part[c * nz + z] = sum;
      }
    }
  }
}

// Grid of the reduction for MA column tiles: one 8-wave block per CU where the registers
// of MA tiles' loads in flight allow only that (measured: 256 blocks 6.07 TB/s, 512 blocks
// 5.68, 1024 blocks 5.86 at MA = 5), more blocks for narrower reductions (MA = 1: 1024
// blocks 4.70 TB/s, 512 blocks 4.55).
inline int gram_max_blocks(int ma) { return ma <= 1 ? 1024 : (ma == 2 ? 512 : 256); }
// Column tiles of a reduction of ncol columns against its last nz.
inline int gram_tiles(int ncol, int nz) { return (nz + 15) / 16 + (ncol - nz + 15) / 16; }

// y(j) -= sum over columns c0 .. c0 + K - 1 of Q(r, c) P(c, j), in column order; the K
// loads of the row's Q entries are issued before the first product.
template <int K, typename T, int S>
__device__ __forceinline__ void upd_group(gbl<T>* __restrict__ V, int64_t ld, int64_t r, int c0,
                                          gbl<const double>* P, T (&y)[S]) {
  T q[K];
#pragma unroll
  for (int u = 0; u < K; ++u) q[u] = V[(int64_t)(c0 + u) * ld + r];
#pragma unroll
  for (int u = 0; u < K; ++u)
#pragma unroll
    for (int j = 0; j < S; ++j) y[j] -= q[u] * (T)P[c0 + u + j * kLd];
}

// W <- (W - Q P) T in place (PF_HAS_P / PF_HAS_T), one row per thread: every lane reads
// its row of the k + sw columns (each wave access is a coalesced 64-row segment of one
// column), P and T are uniform (scalar loads).  No LDS, no barrier, high occupancy.
// Blocks of kBlock rows: 128 (measured faster than 256 or more), 256 for the gated second
// pass, which almost always returns at entry (half the blocks to dispatch then; 1024-row
// blocks were no faster there).
template <typename T, int S, int kBlock>
struct UpdateBody {
  typedef PanelArgs Args;
  static constexpr int kThreads = kBlock;
  static constexpr int kMinWaves = 1;
  static __device__ void run(const PanelArgs& a, int bid, int nb);
};
template <typename T, int S, int kBlock>
__device__ void UpdateBody<T, S, kBlock>::run(const PanelArgs& a, int bid, int) {
  if (gated_off(a, a.st)) return;
  gbl<const SmallState>* st = G(a.st);
  const int64_t r = (int64_t)bid * blockDim.x + threadIdx.x;
  if (r >= a.n) return;
  const int k = a.k, sw = a.sw;
  const bool hasP = a.flags & PF_HAS_P;
  const bool hasT = (a.flags & PF_HAS_T) && !st->identity_t;
  gbl<T>* __restrict__ V = G(reinterpret_cast<T*>(a.V));
  const int64_t ld = a.ld;
  gbl<T>* W = V + (int64_t)a.wcol * ld + r;
  T y[S];
#pragma unroll
  for (int j = 0; j < S; ++j) y[j] = (j < sw) ? W[(int64_t)j * ld] : (T)0;
  if (hasP) {
    // columns in groups of 16, then one of 8, then one of the remaining size: each group
    // issues all its loads before its first update (few dependent round trips per row)
    gbl<const double>* P = st->Pcur;
    int c = 0;
    for (; c + 16 <= k; c += 16) upd_group<16, T, S>(V, ld, r, c, P, y);
    if (c + 8 <= k) {
      upd_group<8, T, S>(V, ld, r, c, P, y);
      c += 8;
    }
    switch (k - c) {
      case 1: upd_group<1, T, S>(V, ld, r, c, P, y); break;
      case 2: upd_group<2, T, S>(V, ld, r, c, P, y); break;
      case 3: upd_group<3, T, S>(V, ld, r, c, P, y); break;
      case 4: upd_group<4, T, S>(V, ld, r, c, P, y); break;
      case 5: upd_group<5, T, S>(V, ld, r, c, P, y); break;
      case 6: upd_group<6, T, S>(V, ld, r, c, P, y); break;
      case 7: upd_group<7, T, S>(V, ld, r, c, P, y); break;
      default: break;
    }
  }
  if (hasT) {
    gbl<const double>* Tm = st->Tcur;
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



// The fused panel step on the matrix cores: per row, the update
//     q = (W(r,:) - Q(r,:) P) T          (PF_HAS_P / PF_HAS_T; Q = V(:,0:k), W = V(:,wcol:+sw))
// stored in place (PF_STORE), and the Gram of its output  G = [Q, q]^T q  (PF_GRAM_Q: Q rows;
// the q rows always), in one pass over the rows.  Batches of the staged columns (Q when
// it is needed, then W) go through LDS as in TileLoad.  The update is itself a product:
// q = [Q, W] B with B = [-P T; T] ((k+sw) x sw, formed once per block in LDS), so each
// 16-row tile of the batch is multiplied by B on the matrix cores (rows are the M
// dimension, the staged columns the K dimension) and q is written over W in the tile;
// after a barrier the matrix cores reduce the Gram of the tile (rows as the K dimension), and
// the waves store q from LDS in whole row segments.  Partials: (k + sw) x sw float64 per
// block (rows of Q zero unless PF_GRAM_Q).  Requires sw <= 16.
template <typename T, int MT>
struct FusedBody {
  typedef PanelArgs Args;
  static constexpr int kThreads = 512;
  static constexpr int kMinWaves = 4;  // two 8-wave blocks per CU
  static __device__ void run(const PanelArgs& a, int bid, int nb);
};
template <typename T, int MT>
__device__ void FusedBody<T, MT>::run(const PanelArgs& a, int bid, int) {
  if (gated_off(a, a.st)) return;
  gbl<const SmallState>* st = G(a.st);
  typedef typename MfmaOp<T>::v4 v4;
  typedef TileLoad<T> TL;
  constexpr int NW = 8, SL = TL::SL, R = TL::R;
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int wv = __builtin_amdgcn_readfirstlane(tid / kWave);  // wave-uniform
  const int k = a.k, sw = a.sw, flags = a.flags;
  const bool hasP = flags & PF_HAS_P;
  const bool hasT = (flags & PF_HAS_T) && !st->identity_t;
  const bool store = flags & PF_STORE;
  const bool gramQ = flags & PF_GRAM_Q;
  const int kq = (hasP || gramQ || (flags & PF_BMAT)) ? k : 0;  // staged Q columns
  const int ncol = kq + sw;                // staged columns: Q then W
  const int a0 = gramQ ? 0 : kq;           // first staged column on the A side of the Gram
  const int ncolA = ncol - a0;
  gbl<T>* __restrict__ V = G(reinterpret_cast<T*>(a.V));
  const int64_t ld = a.ld;
  __shared__ T lt[2][mfma_tile<T>()];
  __shared__ T lB[(kMaxCols + 4) * 16];  // B(c, j) at c * 16 + j, zero-padded to 16 columns
  // B = [-P T; T]: rows c < kq from the projection, rows kq + i from T (identity if no T);
  // PF_BMAT: B given in st->Bs, staged column c being basis column c (kq = wcol)
  const bool bmat = flags & PF_BMAT;
  for (int idx = tid; idx < (kMaxCols + 4) * 16; idx += blockDim.x) {
    const int c = idx / 16, j = idx % 16;
    double v = 0.0;
    if (j < sw && c < ncol) {
      if (bmat) {
        v = st->Bs[c + (a.wcol + j) * kLd];
      } else if (c < kq) {
        if (hasP) {
          if (hasT) {
            for (int l = 0; l <= j; ++l) v -= st->Pcur[c + l * kLd] * st->Tcur[l + j * kMaxS];
          } else {
            v = -st->Pcur[c + j * kLd];
          }
        }
      } else {
        const int i = c - kq;
        v = hasT ? (i <= j ? st->Tcur[i + j * kMaxS] : 0.0) : (i == j ? 1.0 : 0.0);
      }
    }
    lB[idx] = (T)v;
  }
  const bool gram = flags & (PF_GRAM_Q | PF_GRAM_W);
  TL tl;
  tl.init(wv, ncol, kq, a.wcol, ld);
  const int BR = tl.BR, LDT = tl.LDT;

  const int64_t rb = (int64_t)bid * a.rows_per_block;
  const int64_t re = min(a.n, rb + a.rows_per_block);
  T v[SL][R], vn[SL][R], vnn[SL][R];
  v4 acc[MT];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt) acc[mt] = v4{0, 0, 0, 0};
  const int li = lane & 15, lk = lane >> 4;
  const int ksteps_upd = (ncol + 3) / 4;
  // prefetch depth 2 with three register buffers taking turns, loop unrolled by 6 (the
  // compiler drains the loads in flight at the loop head)
  int buf = 0;
  auto batch = [&](const T (&cur)[SL][R], T (&fut)[SL][R], int64_t r0) {
    tl.load(V, wv, lane, r0 + 2 * BR, re, fut);
    T* L = lt[buf];
    tl.to_lds(L, wv, lane, r0, re, cur);
    __syncthreads();
    // ---- q = [Q, W] B for 16-row tiles: lane holds A(row li, column kk + lk) and
    //      B(kk + lk, li); the wave's rows are its own, so it overwrites their W in place
    for (int m0 = wv * 16; m0 < BR; m0 += NW * 16) {
      v4 d = v4{0, 0, 0, 0};
      for (int ks = 0; ks < ksteps_upd; ++ks) {
        const int c = ks * 4 + lk;
        const T av = (c < ncol) ? L[c * LDT + m0 + li] : (T)0;
        d = MfmaOp<T>::mac(av, lB[c * 16 + li], d);
      }
      if (li < sw) {
#pragma unroll
        for (int r = 0; r < 4; ++r) L[(kq + li) * LDT + m0 + MfmaOp<T>::row(lk, r)] = d[r];
      }
    }
    __syncthreads();
    // ---- Gram of the tile on the matrix cores; q back to HBM in whole row segments
    for (int ks = wv; gram && ks < BR / 4; ks += NW) {
      const int row = ks * 4 + lk;
      const T bv = (li < sw) ? L[(kq + li) * LDT + row] : (T)0;
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        const int c = a0 + mt * 16 + li;
        const T av = (c < ncol) ? L[c * LDT + row] : (T)0;
        acc[mt] = MfmaOp<T>::mac(av, bv, acc[mt]);
      }
    }
    if (store) {
      const int nchunk = BR / (kWave * R);
      for (int t = wv; t < sw * nchunk; t += NW) {
        const int j = t % sw, chunk = t / sw;
        const int rl = chunk * kWave * R + R * lane;
#pragma unroll
        for (int e = 0; e < R; ++e) {
          const int64_t row = r0 + rl + e;
          if (row < re) V[((int64_t)a.wcol + j) * ld + row] = L[(kq + j) * LDT + rl + e];
        }
      }
    }
    buf ^= 1;
  };
  tl.load(V, wv, lane, rb, re, v);
  tl.load(V, wv, lane, rb + BR, re, vn);
  for (int64_t r0 = rb; r0 < re; r0 += 6 * BR) {
    batch(v, vnn, r0);
    if (r0 + BR >= re) break;
    batch(vn, v, r0 + BR);
    if (r0 + 2 * BR >= re) break;
    batch(vnn, vn, r0 + 2 * BR);
    if (r0 + 3 * BR >= re) break;
    batch(v, vnn, r0 + 3 * BR);
    if (r0 + 4 * BR >= re) break;
    batch(vn, v, r0 + 4 * BR);
    if (r0 + 5 * BR >= re) break;
    batch(vnn, vn, r0 + 5 * BR);
  }
  if (!gram) return;
  __syncthreads();
  T* red = &lt[0][0];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int c = mt * 16 + MfmaOp<T>::row(lk, r);
      red[(wv * kMaxCols + c) * 16 + li] = acc[mt][r];
    }
  __syncthreads();
  gbl<double>* part1 = G(a.part1) + (size_t)bid * (k + sw) * sw;
  if (!gramQ) {
    for (int e = tid; e < k * sw; e += blockDim.x) part1[e] = 0.0;
  }
  for (int e = tid; e < ncolA * 16; e += blockDim.x) {
    const int c = e / 16, z = e % 16;
    if (z < sw) {
      double sum = 0.0;
#pragma unroll
      for (int w = 0; w < NW; ++w) sum += (double)red[(w * kMaxCols + c) * 16 + z];
      const int sc = a0 + c;  // staged column
      const int prow = sc < kq ? sc : k + (sc - kq);
      part1[prow * sw + z] = sum;
    }
  }
}

// ----------------------------------------------------------------------------- launcher
// Every per-request kernel of a restart cycle runs through this launcher: one launch
// serves a batch of requests (one, for a plain solve).  Request r owns blocks
// bstart[r] .. bstart[r+1]-1 of the grid and reads its arguments from args[r]; its body
// sees its own block index and block count, so a request computes exactly the same
// thing whatever else shares the launch.
template <typename Body>
__global__ __launch_bounds__(Body::kThreads, Body::kMinWaves) void batched_kernel(const typename Body::Args* __restrict__ args,
                                                                 const int* __restrict__ bstart, int nreq) {
  const int b = blockIdx.x;
  int lo = 0, hi = nreq - 1;  // last r with bstart[r] <= b (requests with no block are skipped)
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (bstart[mid] <= b) lo = mid;
    else hi = mid - 1;
  }
  const typename Body::Args a = args[lo];  // into registers: the bodies' memory clobbers
                                           // would otherwise reload the fields
  Body::run(a, b - bstart[lo], bstart[lo + 1] - bstart[lo]);
}

}  // namespace tsg
