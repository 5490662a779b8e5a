// Multicolor Gauss-Seidel preconditioner of right-preconditioned s-step GMRES (the local
// Gauss-Seidel preconditioner of the paper's last experiment, Sec. VI, Fig. 13: block
// Jacobi with Gauss-Seidel in each block, swept by colors on the GPU; one GPU holds the
// whole operator, so the block is the whole matrix).
//
//   coloring  Jones and Plassmann's parallel rounds with hashed priorities: in a round,
//             every uncolored row whose (priority, index) beats those of all its uncolored
//             neighbours takes the smallest color none of its colored neighbours holds.
//             priority(i) = output i of SplitMix64 seeded with 0.  The result equals the
//             greedy coloring in decreasing priority order.  Neighbours are the row's
//             off-diagonal columns: the pattern must be structurally symmetric.
//   sweep     z = M^{-1} w with M = D + L_c (the diagonal and the entries whose column has
//             a lower color than the row): one forward sweep from z = 0 over the colors in
//             increasing order, one launch per color over that color's rows,
//             z_i = (w_i - sum_{j: color(j) < color(i)} a_ij z_j) / a_ii (the entries of higher
//             colors would meet z_j = 0, so they are left out of the layout and z needs no
//             zeroing).
//   layout    built once by tsg_csr_precond on the reordered system P A P^T (rows by
//             block of 8192, then by color): each color's rows cut into slices of 64, one wave
//             per slice; a slice stores its rows' lower-color values and columns entry by
//             entry (entry e of lane l at off + 64 e + l, padded with value 0 at a color-0 row,
//             whose z is already set), so the wave's loads of the operator, of
//             w and of z are coalesced 64-wide runs; per lane the row index and the diagonal.
#pragma once

#include "common.hpp"
#include "state.hpp"

namespace tsg {

__host__ __device__ __forceinline__ uint64_t splitmix_priority(uint64_t i) {
  uint64_t z = (i + 1) * 0x9E3779B97F4A7C15ull;  // state after i + 1 steps from seed 0
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// ------------------------------------------------------------------ coloring (set-up)
__global__ __launch_bounds__(256) void jp_init_kernel(int32_t* c, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) c[i] = -1;
}

// One round: cold -> cnew; per-block count of rows still uncolored into cnt[blockIdx.x].
__global__ __launch_bounds__(256) void jp_round_kernel(const int32_t* __restrict__ row_ptr,
                                                       const int32_t* __restrict__ col, int64_t n,
                                                       const int32_t* __restrict__ cold, int32_t* __restrict__ cnew,
                                                       int32_t* __restrict__ cnt) {
  __shared__ int32_t s_cnt;
  if (threadIdx.x == 0) s_cnt = 0;
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int left = 0;
  if (i < n) {
    int32_t c = cold[i];
    if (c < 0) {
      const uint64_t pi = splitmix_priority((uint64_t)i);
      const int p0 = row_ptr[i], p1 = row_ptr[i + 1];
      bool top = true;
      for (int p = p0; p < p1 && top; ++p) {
        const int64_t j = col[p];
        if (j == i || cold[j] >= 0) continue;
        const uint64_t pj = splitmix_priority((uint64_t)j);
        if (pj > pi || (pj == pi && j > i)) top = false;
      }
      if (top) {  // smallest color no colored neighbour holds
        c = 0;
        for (bool hit = true; hit; ) {
          hit = false;
          for (int p = p0; p < p1; ++p)
            if (col[p] != i && cold[col[p]] == c) { hit = true; break; }
          if (hit) ++c;
        }
      } else {
        left = 1;
      }
    }
    cnew[i] = c;
  }
  if (left) atomicAdd(&s_cnt, 1);  // LDS atomic
  __syncthreads();
  if (threadIdx.x == 0) cnt[blockIdx.x] = s_cnt;
}

// total = sum of the per-block counts (one block).
__global__ __launch_bounds__(1024) void jp_total_kernel(const int32_t* __restrict__ cnt, int nb,
                                                       int32_t* __restrict__ total) {
  __shared__ int32_t s[1024];
  int acc = 0;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) acc += cnt[b];
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *total = s[0];
}

// ------------------------------------------------------------------ reordered system
// The preconditioned solve runs on P A P^T with the rows (and columns) ordered by block of
// consecutive rows, then by color, so that a color's rows form one run per block: its
// sweep reads w and writes z in coalesced runs and the gathers stay near.  Row p of
// P A P^T is row perm[p] of A with its columns renamed by inv (= perm^{-1}) and sorted.
__global__ __launch_bounds__(256) void permute_csr_kernel(const int32_t* __restrict__ row_ptr,
                                                         const int32_t* __restrict__ col,
                                                         const double* __restrict__ val,
                                                         const int32_t* __restrict__ perm,
                                                         const int32_t* __restrict__ inv, int64_t n,
                                                         const int32_t* __restrict__ row_ptr_p,
                                                         int32_t* __restrict__ col_p, double* __restrict__ val_p) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const int32_t i = perm[p];
  const int q0 = row_ptr[i], len = row_ptr[i + 1] - q0, o = row_ptr_p[p];
  for (int k = 0; k < len; ++k) {  // insertion by renamed column
    const int32_t c = inv[col[q0 + k]];
    const double v = val[q0 + k];
    int m = k;
    while (m > 0 && col_p[o + m - 1] > c) {
      col_p[o + m] = col_p[o + m - 1];
      val_p[o + m] = val_p[o + m - 1];
      --m;
    }
    col_p[o + m] = c;
    val_p[o + m] = v;
  }
}

// dst[p] = src[perm[p]] (into the order of P A P^T) and dst[perm[p]] = src[p] (back).
__global__ __launch_bounds__(256) void gather_f64_kernel(const double* __restrict__ src,
                                                        const int32_t* __restrict__ perm, double* __restrict__ dst,
                                                        int64_t n) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p < n) dst[p] = src[perm[p]];
}
__global__ __launch_bounds__(256) void scatter_f64_kernel(const double* __restrict__ src,
                                                         const int32_t* __restrict__ perm, double* __restrict__ dst,
                                                         int64_t n) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p < n) dst[perm[p]] = src[p];
}
__global__ __launch_bounds__(256) void gather_i32_kernel(const int32_t* __restrict__ src,
                                                        const int32_t* __restrict__ perm, int32_t* __restrict__ dst,
                                                        int64_t n) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p < n) dst[p] = src[perm[p]];
}

// ------------------------------------------------------------------ sweep layout (set-up)
// Per slice s (64 consecutive entries p0 .. p0+63 of the list of one color's rows, perm):
// width[s] = the largest count of its rows' entries whose column has a lower color than
// the slice's, sclr[s] (colors: per row of the system swept).  The sweep needs only those
// (the entries of higher colors meet z = 0), so it needs no zeroing pass.
__global__ __launch_bounds__(256) void gs_analyze_kernel(const int32_t* __restrict__ row_ptr,
                                                        const int32_t* __restrict__ col,
                                                        const int32_t* __restrict__ perm,
                                                        const int64_t* __restrict__ sstart,
                                                        const int64_t* __restrict__ send,
                                                        const int64_t* __restrict__ sclr,
                                                        const int32_t* __restrict__ colors, int64_t nslices,
                                                        int32_t* __restrict__ width) {
  const int64_t s = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  if (s >= nslices) return;
  const int64_t p = sstart[s] + lane;
  int cnt = 0;
  if (p < send[s]) {
    const int32_t i = perm[p];
    for (int q = row_ptr[i]; q < row_ptr[i + 1]; ++q) cnt += colors[col[q]] < sclr[s];
  }
  for (int o = kWave / 2; o > 0; o >>= 1) cnt = max(cnt, __shfl_xor(cnt, o, kWave));
  if (lane == 0) width[s] = cnt;
}

// Fill slice s: row index (-1 on padding lanes), diagonal, lower-color values and columns.
__global__ __launch_bounds__(256) void gs_fill_kernel(const int32_t* __restrict__ row_ptr,
                                                     const int32_t* __restrict__ col,
                                                     const double* __restrict__ val,
                                                     const int32_t* __restrict__ perm,
                                                     const int64_t* __restrict__ sstart,
                                                     const int64_t* __restrict__ send,
                                                     const int64_t* __restrict__ sclr,
                                                     const int32_t* __restrict__ colors,
                                                     const int64_t* __restrict__ eoff,
                                                     const int32_t* __restrict__ width, int64_t nslices,
                                                     int32_t padcol, int32_t* __restrict__ prow,
                                                     double* __restrict__ diag, double* __restrict__ gval,
                                                     int32_t* __restrict__ gcol) {
  const int64_t s = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  if (s >= nslices) return;
  const int64_t p = sstart[s] + lane, slot = s * kWave + lane, e0 = eoff[s];
  const int wd = width[s];
  int32_t i = -1;
  double d = 0.0;
  int e = 0;
  if (p < send[s]) {
    i = perm[p];
    for (int q = row_ptr[i]; q < row_ptr[i + 1]; ++q) {
      if (col[q] == i) {
        d = val[q];
      } else if (colors[col[q]] < sclr[s]) {
        gval[e0 + (int64_t)kWave * e + lane] = val[q];
        gcol[e0 + (int64_t)kWave * e + lane] = col[q];
        ++e;
      }
    }
  }
  for (; e < wd; ++e) {  // padding: value 0 at a row of color 0 (swept first: z finite)
    gval[e0 + (int64_t)kWave * e + lane] = 0.0;
    gcol[e0 + (int64_t)kWave * e + lane] = padcol;
  }
  prow[slot] = i;
  diag[slot] = d;
}

// ------------------------------------------------------------------ sweeps (per request)
struct GsArgs {
  const int32_t* prow;     // sweep layout: row index per slot (-1: padding)
  const double* diag;      //   diagonal per slot
  const double* gval;      //   off-diagonal values, entry-major per slice
  const int32_t* gcol;     //   their columns
  const int64_t* eoff;     //   first entry of each slice
  const int32_t* width;    //   entries per lane of each slice
  int64_t slice0;          // color sweep: this color's first slice
  const double* w;         // right-hand side of the sweep
  double* z;               // result
  int64_t n;               // slices of this color
  const SmallState* st;
  int32_t panel;           // -1: gate on the solve's end only; else also on stop_panel
  int32_t pad;
};

__device__ __forceinline__ bool gs_gated(const GsArgs& a) {
  gbl<const SmallState>* st = G(a.st);
  return st->h.done || a.panel > st->h.stop_panel;
}

// acc += sum over entries e0 .. e0 + K - 1 of a sweep slice: the K value
// and column loads, then the K z gathers, are issued before the first product (two
// dependent memory round trips per group); products rounded, then summed in entry order.
template <int K>
__device__ __forceinline__ double gs_group(gbl<const double>* __restrict__ v, gbl<const int32_t>* __restrict__ c,
                                           gbl<const double>* __restrict__ z, int e0, double acc) {
#pragma clang fp contract(off)
  double ve[K], zg[K];
  int32_t ce[K];
#pragma unroll
  for (int u = 0; u < K; ++u) {
    ve[u] = __builtin_nontemporal_load(&v[(int64_t)kWave * (e0 + u)]);
    ce[u] = __builtin_nontemporal_load(&c[(int64_t)kWave * (e0 + u)]);
  }
#pragma unroll
  for (int u = 0; u < K; ++u) zg[u] = z[ce[u]];
#pragma unroll
  for (int u = 0; u < K; ++u) acc += ve[u] * zg[u];
  return acc;
}

// One slice of a color: z_i = (w_i - sum_e a_ie z_col(e)) / a_ii (entries in CSR order),
// the entries in groups of 4, the last width mod 4 as one group of that size.
__device__ __forceinline__ void gs_slice(const GsArgs& a, int64_t s, int lane) {
#pragma clang fp contract(off)
  const int64_t slot = s * kWave + lane;
  const int32_t i = G(a.prow)[slot];
  if (i < 0) return;
  gbl<const double>* __restrict__ v = G(a.gval) + G(a.eoff)[s] + lane;
  gbl<const int32_t>* __restrict__ c = G(a.gcol) + G(a.eoff)[s] + lane;
  gbl<const double>* __restrict__ z = G(a.z);
  const int wd = G(a.width)[s];
  double acc = 0.0;
  int e0 = 0;
  for (; e0 + 4 <= wd; e0 += 4) acc = gs_group<4>(v, c, z, e0, acc);
  switch (wd - e0) {
    case 1: acc = gs_group<1>(v, c, z, e0, acc); break;
    case 2: acc = gs_group<2>(v, c, z, e0, acc); break;
    case 3: acc = gs_group<3>(v, c, z, e0, acc); break;
    default: break;
  }
  G(a.z)[i] = (G(a.w)[i] - acc) / G(a.diag)[slot];
}

struct GsColorBody {  // one color: 4 slices per block, one per wave
  typedef GsArgs Args;
  static constexpr int kThreads = 256;
  static constexpr int kMinWaves = 1;
  static __device__ void run(const GsArgs& a, int bid, int) {
    if (gs_gated(a)) return;
    const int64_t s = (int64_t)bid * (kThreads / kWave) + threadIdx.x / kWave;
    if (s < a.n) gs_slice(a, a.slice0 + s, threadIdx.x & (kWave - 1));
  }
};

// Stand-alone sweep launches (no request state).
__global__ __launch_bounds__(256) void gs_color_kernel(GsArgs a) {
  const int64_t s = (int64_t)blockIdx.x * 4 + threadIdx.x / kWave;
  if (s < a.n) gs_slice(a, a.slice0 + s, threadIdx.x & (kWave - 1));
}

// x += z (the preconditioned cycle update x += M^{-1} Q y).
struct AxpyArgs {
  double* x;
  const double* z;
  int64_t n;
  const SmallState* st;
};
struct AxpyBody {
  typedef AxpyArgs Args;
  static constexpr int kThreads = 256;
  static constexpr int kMinWaves = 1;
  static __device__ void run(const AxpyArgs& a, int bid, int) {
    if (G(a.st)->h.done || G(a.st)->h.redo) return;
    const int64_t i = (int64_t)bid * kThreads + threadIdx.x;
    if (i < a.n) G(a.x)[i] += G(a.z)[i];
  }
};

}  // namespace tsg
