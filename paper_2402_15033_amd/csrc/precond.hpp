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
//             increasing order.  The first launch writes z over all rows (color-0 rows
//             w_i / a_ii, every other row 0), then one launch per color c >= 1 over that
//             color's rows: z_i = (w_i - sum_{j != i} a_ij z_j) / a_ii.
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

// ------------------------------------------------------------------ sweeps (per request)
struct GsArgs {
  const int32_t* row_ptr;  // CSR of A (FP64 values)
  const int32_t* col;
  const double* val;
  const int32_t* colors;   // first sweep: the row colors
  const int32_t* rows;     // color sweep: this color's rows (a slice of the color permutation)
  const double* w;         // right-hand side of the sweep
  double* z;               // result
  int64_t n;               // first sweep: rows; color sweep: rows of this color
  const SmallState* st;
  int32_t panel;           // -1: gate on the solve's end only; else also on stop_panel
  int32_t pad;
};

__device__ __forceinline__ bool gs_gated(const GsArgs& a) {
  gbl<const SmallState>* st = G(a.st);
  return st->h.done || a.panel > st->h.stop_panel;
}

// z_i = w_i / a_ii on color-0 rows, 0 elsewhere (every row, natural order).
__device__ __forceinline__ void gs_first_row(const GsArgs& a, int64_t i) {
  gbl<double>* z = G(a.z);
  if (G(a.colors)[i] != 0) {
    z[i] = 0.0;
    return;
  }
  gbl<const int32_t>* rp = G(a.row_ptr);
  gbl<const int32_t>* cl = G(a.col);
  double d = 0.0;
  for (int p = rp[i]; p < rp[i + 1]; ++p)
    if (cl[p] == i) d = G(a.val)[p];
  z[i] = G(a.w)[i] / d;
}

// One color c >= 1: z_i = (w_i - sum_{j != i} a_ij z_j) / a_ii for its rows (CSR order).
__device__ __forceinline__ void gs_color_row(const GsArgs& a, int64_t t) {
#pragma clang fp contract(off)
  const int64_t i = G(a.rows)[t];
  gbl<const int32_t>* rp = G(a.row_ptr);
  gbl<const int32_t>* cl = G(a.col);
  gbl<const double>* v = G(a.val);
  gbl<double>* z = G(a.z);
  double s = 0.0, d = 0.0;
  for (int p = rp[i]; p < rp[i + 1]; ++p) {
    const int32_t j = cl[p];
    if (j == i) d = v[p];
    else s += v[p] * z[j];
  }
  z[i] = (G(a.w)[i] - s) / d;
}

struct GsFirstBody {
  typedef GsArgs Args;
  static constexpr int kThreads = 256;
  static constexpr int kMinWaves = 1;
  static __device__ void run(const GsArgs& a, int bid, int) {
    if (gs_gated(a)) return;
    const int64_t i = (int64_t)bid * kThreads + threadIdx.x;
    if (i < a.n) gs_first_row(a, i);
  }
};
struct GsColorBody {
  typedef GsArgs Args;
  static constexpr int kThreads = 256;
  static constexpr int kMinWaves = 1;
  static __device__ void run(const GsArgs& a, int bid, int) {
    if (gs_gated(a)) return;
    const int64_t t = (int64_t)bid * kThreads + threadIdx.x;
    if (t < a.n) gs_color_row(a, t);
  }
};

// Stand-alone sweep launches (no request state).
__global__ __launch_bounds__(256) void gs_first_kernel(GsArgs a) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < a.n) gs_first_row(a, i);
}
__global__ __launch_bounds__(256) void gs_color_kernel(GsArgs a) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t < a.n) gs_color_row(a, t);
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
    if (G(a.st)->h.done) return;
    const int64_t i = (int64_t)bid * kThreads + threadIdx.x;
    if (i < a.n) G(a.x)[i] += G(a.z)[i];
  }
};

}  // namespace tsg
