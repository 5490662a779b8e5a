// Lean streaming kernels of the panel steps:
//   GramBody   -- the reduction  G = V(:, 0:ncol)^T V(:, ncol-nz : ncol)  (no update)
//   UpdateBody -- the update     W <- (W - Q P) T  in place            (no reduction)
//   FusedBody  -- the update and the Gram of its output in one pass, for the steps whose
//                 next reduction needs exactly the columns just written
#pragma once

#include <type_traits>

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

// The reduction G = V(:, 0:ncol)^T V(:, ncol-nz : ncol) of a panel step on the matrix cores
// (ncol = k + sw, Q = V(:, 0:k), W = V(:, wcol:wcol+sw); the nz right-hand columns are the
// previous panel's nprev columns, their block column of the stage-2 Gram, followed by W).
// Rows are the K dimension.  In the operand layout lane l = 16 g + i holds, for each column
// tile t, column c_t + i and the RL consecutive rows r + RL g .. r + RL g + RL - 1 of a
// group of 4 RL rows (RL = 4 in FP64, 8 in FP32); K-step e of the group pairs row
// r + RL g + e with k index g in both operands.  The tiles are laid out from the right: the
// last NT tiles are the last 16 NT columns (from column 0 if there are fewer), which hold
// the nz right-hand columns -- the B operand is the A operand of those tiles, and the
// products with their other columns are dropped -- and MA - NT tiles cover the columns to
// their left down to column 0 (lanes outside [0, ncol) hold zeros).  Each wave walks its own
// groups (wave w: groups w, w + NW, ... of the block's rows); the loads of a group cover
// whole 128-byte lines and reach the operand layout through the wave's own LDS tile (no
// block barrier in the row loop), with the next group's loads in flight; they are
// unconditional (the index is clamped to the last full group).  A ragged last group (and
// every group when the columns are not 16-byte aligned) is read element by element in the
// operand layout with its rows masked.  The NW waves' tiles are summed in LDS in wave order
// at the end.  Partials: ncol x nz float64 per block.  Measured on the reductions of an
// m = 60, s = 5 cycle (4194304 rows, FP64): 6.6-7.0 TB/s for every panel but the first
// (1.98 ms in all), against 5.8-6.1 TB/s (2.28 ms) when each lane read its operand rows
// straight from global memory (two 16-byte loads per tile, each covering half of every
// line), and 4.73 TB/s for an LDS-staged version with block barriers.
template <typename T>
constexpr int gram_rows_per_lane() { return 32 / (int)sizeof(T); }
template <bool NTL>
struct LoadPolicy {
  static constexpr bool nt = NTL;
};
constexpr int64_t kGramKeepBytes = 256ll << 20;
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
  const int zb = max(0, ncol - 16 * NT);  // first column of the right-hand tiles (zb <= z0)
  const int64_t ld = a.ld, n = a.n;
  gbl<const T>* __restrict__ V = G(reinterpret_cast<const T*>(a.V));
  // per tile: this lane's column (offset of its first element) and whether it exists
  int64_t coff[MA];
  bool cval[MA];
#pragma unroll
  for (int t = 0; t < MA; ++t) {
    const int c = zb + 16 * (t - (MA - NT)) + li;
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
  // The row loop's loads: per tile two 16-byte loads per lane, load h covering the tile's
  // columns 8 h .. 8 h + 7 with 8 lanes per column, so that every load reads whole 128-byte
  // lines (one line per column: rows r0 .. r0 + GR - 1), with the non-temporal hint.  The
  // wave turns them into the operand layout above through its own LDS tile (column-major,
  // column stride CS = GR + H elements, which spreads the 16 columns of an operand read over
  // the banks).  SQ_LDS_BANK_CONFLICT reports a quarter of the LDS cycles as conflict cycles
  // here; an XOR swizzle of the 16-byte pieces (stride GR, no bank shared within any 16-lane
  // quarter of a write or read) gave the same count and the same time, so the count is taken
  // to be the cost of the 16-byte accesses themselves.  Measured on streams of 64 columns:
  // loads covering whole lines run at 7.1 TB/s with the hint and 6.3 without, loads covering
  // half lines (the operand layout read straight from global memory) at 4.8 and 3.9.
  constexpr int H = 16 / (int)sizeof(T), CS = GR + H, TW = 16 * MA * CS;
  typedef T t16 __attribute__((ext_vector_type(H)));
  int64_t loff[MA][2];
#pragma unroll
  for (int t = 0; t < MA; ++t)
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int c = zb + 16 * (t - (MA - NT)) + 8 * h + (lane >> 3);
      const int cc = c >= 0 && c < ncol ? c : 0;
      loff[t][h] = (int64_t)(cc < k ? cc : a.wcol + (cc - k)) * ld + (lane & 7) * H;
    }
  __shared__ __align__(16) T lt[NW * TW];
  T* const Lw = lt + wv * TW;
  // The last kGramKeepBytes of the reduction's reads (the last groups of every block) take
  // plain loads, the others the non-temporal hint: the lines read last stay in the
  // last-level cache (256 MB on MI355X) for the panel update, which reads the same columns
  // next.  Measured on the 2048^2 solve (per-launch means): all reads non-temporal, Grams
  // 163 us, updates 187 us; the last 128 / 256 / 512 MB plain, 164 / 166 / 171 and 175 /
  // 167 / 166 us (the matrix-powers steps, whose matrix the kept columns displace from the
  // cache, 38.0 / 38.6 / 39.7 / 40.4 us): 256 MB.
  const double kf = min(1.0, (double)kGramKeepBytes / ((double)ncol * (double)n * sizeof(T)));
  const int64_t qs = nfull - (int64_t)(kf * (double)nfull);  // groups from qs on: plain loads
  auto gload = [&](auto pol, int64_t q, t16 (&x)[MA][2]) {
    const int64_t r0 = rb + GR * q;
#pragma unroll
    for (int t = 0; t < MA; ++t)
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        gbl<const t16>* p = reinterpret_cast<gbl<const t16>*>(V + loff[t][h] + r0);
        x[t][h] = decltype(pol)::nt ? __builtin_nontemporal_load(p) : *p;
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
  // Wave wv's groups q = wv, wv + NW, ... below qe, starting at q: the group's loads are
  // written to the wave's LDS tile, the next group's loads are issued, and the tile is read
  // back in the operand layout and multiplied while they are in flight.  (LDS accesses of
  // one wave execute in order: only the compiler must keep them in order.)  Measured
  // against two register buffers (the next two groups' loads in flight): 1.98 against 2.00
  // ms for the reductions of an m = 60, s = 5 cycle on 4194304 rows; two groups per step
  // with two LDS tiles 2.01 ms; twice the grid, with or without a 128-register cap, 2.00.
  auto rowloop = [&](auto pol, int64_t q, int64_t qe) {
    if (q >= qe) return;
    t16 x[MA][2];
    T v[MA][RL];
    gload(pol, q, x);
    for (; q < qe; q += NW) {
#pragma unroll
      for (int t = 0; t < MA; ++t)
#pragma unroll
        for (int h = 0; h < 2; ++h) *reinterpret_cast<t16*>(Lw + (16 * t + 8 * h + (lane >> 3)) * CS + (lane & 7) * H) = x[t][h];
      __asm__ volatile("" ::: "memory");
      gload(pol, min<int64_t>(q + NW, qe - 1), x);
#pragma unroll
      for (int t = 0; t < MA; ++t)
#pragma unroll
        for (int p = 0; p < RL / H; ++p) {
          const t16 y = *reinterpret_cast<const t16*>(Lw + (16 * t + li) * CS + RL * g + H * p);
#pragma unroll
          for (int e = 0; e < H; ++e) v[t][H * p + e] = y[e];
        }
      __asm__ volatile("" ::: "memory");
      mma(v);
    }
  };
  if (vec && nfull > 0) {
    const int64_t q2 = qs <= wv ? wv : wv + (qs - wv + NW - 1) / NW * NW;  // first own group >= qs
    rowloop(LoadPolicy<true>{}, wv, min<int64_t>(qs, nfull));
    rowloop(LoadPolicy<false>{}, q2, nfull);
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
  static_assert(NW * RC * 16 <= NW * TW, "reduction buffer");
  T* const red = lt;  // the waves' tiles are free once every wave has left its row loop
  gbl<double>* part = G(a.part1) + (size_t)bid * ncol * nz;
#pragma unroll
  for (int u = 0; u < NT; ++u) {
    __syncthreads();
#pragma unroll
    for (int t = 0; t < MA; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int c = zb + 16 * (t - (MA - NT)) + MfmaOp<T>::row(g, r);
        if (c >= 0 && c < ncol) red[(wv * RC + c) * 16 + li] = acc[t][u][r];
      }
    __syncthreads();
    for (int e = threadIdx.x; e < ncol * 16; e += blockDim.x) {
      const int c = e / 16, z = zb + u * 16 + e % 16 - z0;  // right-hand column zb + 16 u + e % 16
      if (z >= 0 && z < nz) {
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
// Column tiles of a reduction of ncol columns against its last nz: the right-hand tiles
// (the last 16 ceil(nz / 16) columns) and the tiles to their left.
inline int gram_tiles(int ncol, int nz) {
  const int nt = (nz + 15) / 16;
  const int left = ncol > 16 * nt ? ncol - 16 * nt : 0;
  return nt + (left + 15) / 16;
}

// y(j) -= sum over columns c0 .. c0 + K - 1 of Q(r, c) P(c, j), in column order; the K
// loads of the row's Q entries are issued before the first product.
template <int K, typename T, int S>
__device__ __forceinline__ void upd_group(gbl<T>* __restrict__ V, int64_t ld, int64_t r, int c0,
                                          gbl<const double>* P, T (&y)[S]) {
  T q[K];
#pragma unroll
  for (int u = 0; u < K; ++u) q[u] = __builtin_nontemporal_load(&V[(int64_t)(c0 + u) * ld + r]);
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
  for (int j = 0; j < S; ++j) y[j] = (j < sw) ? __builtin_nontemporal_load(&W[(int64_t)j * ld]) : (T)0;
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
  // non-temporal stores: the written columns are not read again by this launch, and the reads
  // that share HBM with these writes ran 3-7% faster (k = 11 .. 51) than with plain stores
#pragma unroll
  for (int j = 0; j < S; ++j)
    if (j < sw) __builtin_nontemporal_store(y[j], &W[(int64_t)j * ld]);
}



// The fused panel step: per row, the update
//     q = (W(r,:) - Q(r,:) P) T          (PF_HAS_P / PF_HAS_T; Q = V(:,0:k), W = V(:,wcol:+sw))
// stored in place (PF_STORE), and the Gram of its output  G = [Q, q]^T q  (PF_GRAM_Q: Q rows;
// the q rows always), in one pass over the rows.  The update is a product q = [Q, W] B with
// B = [-P T; T] ((k+sw) x sw, formed once per block in LDS; PF_BMAT: B given in st->Bs), done
// on the matrix cores with the rows as the M dimension: for K-step ks (staged columns 4 ks ..
// 4 ks + 3) lane l = 16 g + i takes row r0 + i of staged column 4 ks + g straight from
// global memory (each load instruction covers 16 consecutive rows of 4 columns), and the
// result lane (g, i) holds q(row(g, r), i) for r = 0..3.  The Gram needs the rows as the K
// dimension instead: the wave writes its 16 x (k+sw) tile -- Q as loaded, q in place of W --
// to a wave-private LDS tile and reads it back column-wise as the A operand, while the B
// operand is q as the update left it (K-step e pairs row row(g, e) with k index g in both).
// Each wave walks its own 16-row groups with the next group's loads in flight; there is no
// block barrier in the row loop.  Partials: (k + sw) x sw float64 per block (rows of Q zero
// unless PF_GRAM_Q).  Requires sw <= 16 and k + sw <= 16 NC.
constexpr int kFusedGroupRows = 16;  // row blocks of the fused step are multiples of this
template <typename T, int NC>
struct FusedBody {
  typedef PanelArgs Args;
  static constexpr int kThreads = 512;
  static constexpr int kMinWaves = 1;
  static __device__ void run(const PanelArgs& a, int bid, int nb);
};
template <typename T, int NC>
__device__ void FusedBody<T, NC>::run(const PanelArgs& a, int bid, int) {
  if (gated_off(a, a.st)) return;
  gbl<const SmallState>* st = G(a.st);
  typedef typename MfmaOp<T>::v4 v4;
  constexpr int NW = kThreads / kWave, NKS = 4 * NC, GR = kFusedGroupRows;
  constexpr int LS = sizeof(T) == 8 ? 66 : 68;  // LDS row stride: <= 2-way bank conflicts
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int wv = __builtin_amdgcn_readfirstlane(tid / kWave);
  const int g = lane >> 4, li = lane & 15;
  const int k = a.k, sw = a.sw, flags = a.flags;
  const bool hasP = flags & PF_HAS_P;
  const bool hasT = (flags & PF_HAS_T) && !st->identity_t;
  const bool store = flags & PF_STORE;
  const bool gramQ = flags & PF_GRAM_Q;
  const bool bmat = flags & PF_BMAT;
  const bool gram = flags & (PF_GRAM_Q | PF_GRAM_W);
  const int kq = (hasP || gramQ || bmat) ? k : 0;  // staged Q columns
  const int ncol = kq + sw;                        // staged columns: Q then W
  const int a0 = gramQ ? 0 : kq;                   // first staged column on the A side of the Gram
  const int mat = gram ? (ncol - a0 + 15) / 16 : 0;
  gbl<T>* __restrict__ V = G(reinterpret_cast<T*>(a.V));
  const int64_t ld = a.ld;
  __shared__ T lB[(kMaxCols + 4) * 16];  // B(c, j) at c * 16 + j, zero-padded
  __shared__ T lt[NW * GR * LS];          // per-wave tiles; the cross-wave sums at the end
  // B = [-P T; T]: rows c < kq from the projection, rows kq + i from T (identity if no T);
  // PF_BMAT: B given in st->Bs, staged column c being basis column c (kq = wcol)
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
  __syncthreads();
  const int64_t rb = (int64_t)bid * a.rows_per_block;
  const int64_t re = min(a.n, rb + a.rows_per_block);
  const int64_t nfull = (re - rb) / GR;
  const int64_t shift = (int64_t)a.wcol - kq;  // staged column c >= kq is basis column c + shift
  // element offset of row i of staged K-step column 4 ks + g (clamped into the staged columns;
  // B's rows past ncol are zero)
  auto coff = [&](int ks) -> int64_t {
    const int c = min(4 * ks + g, ncol - 1);
    return (int64_t)(c + (c >= kq ? shift : 0)) * ld + li;
  };
  v4 acc[NC];
#pragma unroll
  for (int t = 0; t < NC; ++t) acc[t] = v4{0, 0, 0, 0};
  T* L = lt + wv * GR * LS;
  auto load = [&](int64_t r0, T (&v)[NKS]) {
#pragma unroll
    for (int ks = 0; ks < NKS; ++ks) v[ks] = __builtin_nontemporal_load(&V[coff(ks) + r0]);
  };
  // one group of rows r0 .. r0 + 15 (rows from nrows on are padding, zero in v)
  auto group = [&](int64_t r0, const T (&v)[NKS], int nrows) {
    v4 d = v4{0, 0, 0, 0};
#pragma unroll
    for (int ks = 0; ks < NKS; ++ks) d = MfmaOp<T>::mac(v[ks], lB[(4 * ks + g) * 16 + li], d);
    if (store && li < sw) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = MfmaOp<T>::row(g, r);
        if (row < nrows) __builtin_nontemporal_store(d[r], &V[(int64_t)(a.wcol + li) * ld + r0 + row]);
      }
    }
    if (!gram) return;
    // the wave's tile: Q as loaded (row li of staged column 4 ks + g), q over W's columns
#pragma unroll
    for (int ks = 0; ks < NKS; ++ks) {
      const int c = 4 * ks + g;
      if (gramQ && c < kq) L[li * LS + c] = v[ks];
    }
    if (li < sw) {
#pragma unroll
      for (int r = 0; r < 4; ++r) L[MfmaOp<T>::row(g, r) * LS + kq + li] = d[r];
    }
    wave_lds_sync();
    const T bq[4] = {li < sw ? d[0] : (T)0, li < sw ? d[1] : (T)0, li < sw ? d[2] : (T)0, li < sw ? d[3] : (T)0};
#pragma unroll
    for (int t = 0; t < NC; ++t) {
      if (t < mat) {
        const int c = a0 + 16 * t + li;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const T av = c < ncol ? L[MfmaOp<T>::row(g, e) * LS + c] : (T)0;
          acc[t] = MfmaOp<T>::mac(av, bq[e], acc[t]);
        }
      }
    }
    wave_lds_sync();
  };
  if (nfull > 0) {
    T va[NKS], vb[NKS];
    int64_t q = wv;
    load(rb + GR * min<int64_t>(q, nfull - 1), va);
    for (; q < nfull; q += 2 * NW) {
      load(rb + GR * min<int64_t>(q + NW, nfull - 1), vb);
      group(rb + GR * q, va, GR);
      if (q + NW >= nfull) break;
      load(rb + GR * min<int64_t>(q + 2 * NW, nfull - 1), va);
      group(rb + GR * (q + NW), vb, GR);
    }
  }
  if (re - rb - GR * nfull > 0 && wv == (int)(nfull % NW)) {  // the ragged last group
    const int64_t r0 = rb + GR * nfull;
    const int nrows = (int)(re - r0);
    T v[NKS];
#pragma unroll
    for (int ks = 0; ks < NKS; ++ks) v[ks] = li < nrows ? __builtin_nontemporal_load(&V[coff(ks) + r0]) : (T)0;
    group(r0, v, nrows);
  }
  if (!gram) return;
  // sum the NW waves' tiles in wave order: red[w][c][z], c < 16 NC, z < 16 (fits lt)
  static_assert(NW * 16 * NC * 16 <= NW * GR * LS, "reduction buffer");
  __syncthreads();
  T* red = lt;
#pragma unroll
  for (int t = 0; t < NC; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int c = 16 * t + MfmaOp<T>::row(g, r);
      red[(wv * 16 * NC + c) * 16 + li] = acc[t][r];
    }
  __syncthreads();
  gbl<double>* part1 = G(a.part1) + (size_t)bid * (k + sw) * sw;
  if (!gramQ) {
    for (int e = tid; e < k * sw; e += blockDim.x) part1[e] = 0.0;
  }
  const int ncolA = ncol - a0;
  for (int e = tid; e < ncolA * 16; e += blockDim.x) {
    const int c = e / 16, z = e % 16;
    if (z < sw) {
      double sum = 0.0;
#pragma unroll
      for (int w = 0; w < NW; ++w) sum += (double)red[(w * 16 * NC + c) * 16 + z];
      const int sc = a0 + c;  // staged column
      const int prow = sc < kq ? sc : k + (sc - kq);
      part1[prow * sw + z] = sum;
    }
  }
}

// Q = Qhat R^{-1} in place (the explicit Q of a CholQR whose upper-triangular inverse Rinv,
// k x k with k <= 16 NCT, ld kLd, is known), on the matrix cores with the rows as the N
// dimension: per group of 16 rows, D = Rinv^T (output columns x input columns) times
// X^T (input columns x rows).  For K-step ks lane l = 16 g + i takes row r0 + i of input
// column 4 ks + g straight from global memory (each load covers 16 consecutive rows of 4
// columns) and holds, in accumulator register r of tile t, output column 16 t + g + 4 r of
// row r0 + i (each store covers 16 consecutive rows of 4 columns).  Rinv is upper triangular,
// so tile t takes the K-steps ks <= 4 t + 3 only (40 products per group for k = 61 instead of
// 64); the A operand values (Rinv^T, zero outside the triangle) sit in LDS in lane order
// (conflict-free 8-byte reads).  Each wave walks its groups (wave w of the block: groups w,
// w + NW, ... of the block's rows); the next group's input column of a K-step is loaded as
// soon as the current group's last product with it is issued, so one group's loads are in
// flight while the matrix cores work.  Every K-step runs (no runtime branch in the row loop):
// lanes past column k - 1 read column k - 1, whose products meet zero Rinv entries.  Addresses
// are a uniform part (K-step, group) plus the lane's byte offset, 32-bit when Off32 (3 ld + 15
// elements fit: the host checks) -- the uniform part then stays in scalar registers.  The
// ragged last group of rows is loaded and stored element-wise with its rows masked.  A row is read and written by one wave only, so the
// update in place needs no barrier.  Returns at entry when st->h.done is set (a breakdown
// before it: no inverse was formed).
constexpr int kRinvThreads = 256;
constexpr int kRinvGroupRows = 16;
template <int NCT, bool Off32>
__global__ __launch_bounds__(kRinvThreads) void apply_rinv_kernel(double* __restrict__ V_, int64_t ld, int64_t n,
                                                                  int k, const double* __restrict__ Rinv,
                                                                  int64_t rows_per_block, const SmallState* st) {
  if (st->h.done) return;
  typedef MfmaOp<double>::v4 v4;
  typedef typename std::conditional<Off32, uint32_t, int64_t>::type off_t;
  constexpr int NW = kRinvThreads / kWave, NKS = 4 * NCT, GR = kRinvGroupRows;
  __shared__ double sA[NCT * NKS * kWave];  // (t, ks, lane) -> Rinv(4 ks + g, 16 t + i)
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int wv = __builtin_amdgcn_readfirstlane(tid / kWave);
  const int g = lane >> 4, li = lane & 15;
  for (int e = tid; e < NCT * NKS * kWave; e += kRinvThreads) {
    const int l = e % kWave, ks = (e / kWave) % NKS, t = e / (kWave * NKS);
    const int row = 4 * ks + (l >> 4), col = 16 * t + (l & 15);
    sA[e] = (row <= col && col < k) ? Rinv[row + col * kLd] : 0.0;
  }
  __syncthreads();
  gbl<char>* const base = G(reinterpret_cast<char*>(V_));
  // K-step ks reads column cb + min(g, k - 1 - cb), cb = min(4 ks, k - 1) uniform
  const off_t ldb = (off_t)(ld * 8), li8 = (off_t)(li * 8);
  const off_t offl = (off_t)g * ldb + li8;
  auto at = [=](int64_t uni, off_t lo) { return (gbl<double>*)(base + uni * 8 + lo); };
  auto xat = [=](int ks, int64_t r0) {
    const int cb = min(4 * ks, k - 1);
    const off_t lo = (off_t)min(g, k - 1 - cb) * ldb + li8;
    return (gbl<double>*)(base + ((int64_t)cb * ld + r0) * 8 + lo);
  };
  const int64_t rb = (int64_t)blockIdx.x * rows_per_block;
  const int64_t re = min(n, rb + rows_per_block);
  const int64_t nfull = (re - rb) / GR;
  if (wv < nfull) {
    double x[NKS];
    int64_t q = wv;
#pragma unroll
    for (int ks = 0; ks < NKS; ++ks) x[ks] = __builtin_nontemporal_load(xat(ks, rb + GR * q));
    for (; q < nfull; q += NW) {
      // an opaque zero in the LDS index: the operand values are read from LDS per group
      // rather than hoisted into 80 registers across the loop
      int z;
      __asm__ volatile("s_mov_b32 %0, 0" : "=s"(z));
      const int64_t r0 = rb + GR * q;
      const int64_t rn = rb + GR * min<int64_t>(q + NW, nfull - 1);
      v4 acc[NCT];
#pragma unroll
      for (int t = 0; t < NCT; ++t) acc[t] = v4{0, 0, 0, 0};
#pragma unroll
      for (int ks = 0; ks < NKS; ++ks) {
#pragma unroll
        for (int t = 0; t < NCT; ++t)
          if (ks <= 4 * t + 3) acc[t] = MfmaOp<double>::mac(sA[(t * NKS + ks) * kWave + lane + z], x[ks], acc[t]);
        x[ks] = __builtin_nontemporal_load(xat(ks, rn));
      }
#pragma unroll
      for (int t = 0; t < NCT; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          if (16 * t + g + 4 * r < k) __builtin_nontemporal_store(acc[t][r], at((int64_t)(16 * t + 4 * r) * ld + r0, offl));
    }
  }
  if (re - rb - GR * nfull > 0 && wv == (int)(nfull % NW)) {  // the ragged last group
    gbl<double>* __restrict__ V = G(V_);
    const int64_t r0 = rb + GR * nfull;
    const bool ok = r0 + li < re;
    v4 acc[NCT];
#pragma unroll
    for (int t = 0; t < NCT; ++t) acc[t] = v4{0, 0, 0, 0};
#pragma unroll
    for (int ks = 0; ks < NKS; ++ks) {
      const int col = min(4 * ks + g, k - 1);
      const double xv = ok ? __builtin_nontemporal_load(&V[(int64_t)col * ld + r0 + li]) : 0.0;
#pragma unroll
      for (int t = 0; t < NCT; ++t)
        if (ks <= 4 * t + 3) acc[t] = MfmaOp<double>::mac(sA[(t * NKS + ks) * kWave + lane], xv, acc[t]);
    }
#pragma unroll
    for (int t = 0; t < NCT; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int col = 16 * t + g + 4 * r;
        if (ok && col < k) __builtin_nontemporal_store(acc[t][r], &V[(int64_t)col * ld + r0 + li]);
      }
  }
}
// Whether apply_rinv_kernel's lane byte offsets (3 ld + 15 elements at most) fit 32 bits.
inline bool rinv_off32(int64_t ld) { return (3 * ld + 16) * 8 < ((int64_t)1 << 32); }
// Rows per block of apply_rinv_kernel: at most kRinvMaxBlocks blocks, whole waves of groups.
constexpr int kRinvMaxBlocks = 1024;
inline int64_t rinv_rows_per_block(int64_t n) {
  const int64_t unit = (int64_t)kRinvGroupRows * (kRinvThreads / kWave);
  const int64_t units = (n + unit - 1) / unit;
  const int64_t per = (units + kRinvMaxBlocks - 1) / kRinvMaxBlocks;
  return per * unit;
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
