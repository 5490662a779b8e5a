// Device helpers shared by the kernels of the tsgmres library (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tsg {

constexpr int kWave = 64;
constexpr int kLd = 64;      // leading dimension of every small matrix in SmallState
constexpr int kMaxCols = 64; // max basis columns (m + 1) and max tall-skinny block width
constexpr int kMaxS = 16;    // max step size
constexpr int kGroup = 16;   // blocks per first-level group of the two-level reduction

// Relative pivot threshold of the Cholesky factorizations inside a restart cycle:
// a pivot d_j <= tol * ref_j (ref = diagonal of the raw Gram matrix) is treated as a
// numerically dependent column (breakdown).  FP64 and FP32 bases.
constexpr double kPivotTolF64 = 1e-12;
constexpr double kPivotTolF32 = 1e-5;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

__device__ __forceinline__ void fence_release() { __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent"); }
__device__ __forceinline__ void fence_acquire() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent"); }

__device__ __forceinline__ unsigned atomic_ticket(unsigned* p) {
  return __hip_atomic_fetch_add(p, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void atomic_reset(unsigned* p) {
  __hip_atomic_store(p, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Blocks are dispatched round-robin over the 8 XCDs (block b runs on XCD b % 8).
// Map the hardware block index to a logical tile so that each XCD walks one
// contiguous range of tiles: neighbouring rows then share that XCD's L2 (the SpMV
// gathers x from rows +-1 and +-N).
__device__ __forceinline__ int xcd_tile(int b, int nb) {
  const int nx = 8;
  int per = nb / nx, rem = nb % nx;
  int x = b % nx, j = b / nx;
  return x * per + (x < rem ? x : rem) + j;
}

// Deterministic two-level "last block" reduction.
//   Every block has written its E partial sums to part1[blockIdx.x * E + e] (all
//   threads of the block may have written some).  Blocks are grouped by kGroup
//   consecutive indices.  The last block of each group to arrive sums its group's
//   partials in block order into part2[group * E + e]; the last group reducer sums
//   part2 in group order into out[e] (any address space) and returns true.  Every
//   other block returns false.  Counters: cnt[0] for level 2, cnt[1 + group] for
//   level 1; each is reset to zero by the block that consumed it, so the same counter
//   array serves every launch on one stream.  Must be called by all threads.
template <typename OutFn>
__device__ bool last_block_reduce(const double* part1, double* part2, unsigned* cnt, int E,
                                  int nblocks, OutFn out) {
  __shared__ int s_flag;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int group = blockIdx.x / kGroup;
  const int g0 = group * kGroup;
  const int gsz = min(kGroup, nblocks - g0);
  const int ngroups = (nblocks + kGroup - 1) / kGroup;
  fence_release();
  __syncthreads();
  if (tid == 0) s_flag = (atomic_ticket(&cnt[1 + group]) == (unsigned)(gsz - 1));
  __syncthreads();
  if (!s_flag) return false;
  fence_acquire();
  for (int e = tid; e < E; e += nt) {
    double acc = 0.0;
    for (int b = 0; b < gsz; ++b) acc += part1[(size_t)(g0 + b) * E + e];
    part2[(size_t)group * E + e] = acc;
  }
  if (tid == 0) atomic_reset(&cnt[1 + group]);
  fence_release();
  __syncthreads();
  if (tid == 0) s_flag = (atomic_ticket(&cnt[0]) == (unsigned)(ngroups - 1));
  __syncthreads();
  if (!s_flag) return false;
  fence_acquire();
  for (int e = tid; e < E; e += nt) {
    double acc = 0.0;
    for (int g = 0; g < ngroups; ++g) acc += part2[(size_t)g * E + e];
    out(e, acc);
  }
  if (tid == 0) atomic_reset(&cnt[0]);
  __syncthreads();
  return true;
}

}  // namespace tsg
