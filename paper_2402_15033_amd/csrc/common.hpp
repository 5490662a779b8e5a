// Device helpers shared by the kernels of the tsgmres library (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tsg {

constexpr int kWave = 64;
constexpr int kLd = 64;      // leading dimension of every small matrix in SmallState
constexpr int kMaxCols = 64; // max basis columns (m + 1) and max tall-skinny block width
constexpr int kMaxS = 16;    // max step size
constexpr int kMaxNz = 32;   // max right-hand columns of a lean Gram reduction (2 kMaxS)
constexpr int kTailThreads = 1024;  // threads of the one-block tail kernels

// Relative pivot threshold of the Cholesky factorizations inside a restart cycle:
// a pivot d_j <= tol * ref_j (ref = diagonal of the raw Gram matrix) is treated as a
// numerically dependent column (breakdown).  FP64 and FP32 bases.
constexpr double kPivotTolF64 = 1e-12;
constexpr double kPivotTolF32 = 1e-5;
// Two-stage stage 1 in FP64: a relative pivot of the one-reduction pass (BCGS-PIP) at most
// this takes the explicit second pass.  Sec. IV-C: the Pythagorean Gram G_W - P^T P is
// accurate only while kappa([Q, W])^2 eps stays well below 1; its pivots near kPivotTolF64
// are at the rounding level of the subtraction (measured on the monomial basis at s = 10:
// pivots of 5e-12 .. 1.5e-9 off by up to 2e-9), so the pass is taken below 1e-8, where the
// decision has a wide margin.  Bases with s <= 5 (relative pivots >= 2e-6) never reach it.
// The mixed form keeps kPivotTolF32.
constexpr double kPipTolF64 = 1e-8;

// Device (global) memory as the compiler's address space 1.  The kernels take their
// pointers from a per-launch argument table in memory, so to the compiler they are
// generic pointers and their accesses would be flat instructions (which also count
// against the LDS wait counter, and never become scalar loads).  Every pointer of the
// table points to device memory; the hot loops access it through gbl<T>* pointers,
// which compile to global loads and stores, and to scalar loads for wave-uniform
// addresses.
template <typename T>
using gbl = __attribute__((address_space(1))) T;
template <typename T>
__device__ __forceinline__ gbl<T>* G(T* p) {
  return (gbl<T>*)p;
}
// The same wave-uniform pointer as a generic one that the compiler knows to point to device
// memory: a round trip through address space 1, kept from folding away by an empty asm on
// the scalar registers holding it.  Code that takes plain pointers derived from it (struct
// members, helper arguments) then compiles its accesses to global loads and stores instead
// of flat ones.
// (The pointer is wave-uniform by contract; reading it from the first active lane makes that
// explicit where the compiler holds it in vector registers.)
template <typename T>
__device__ __forceinline__ T* Gp(T* p) {
  const uint64_t u = (uint64_t)p;
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)u);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(u >> 32));
  gbl<T>* q = (gbl<T>*)(((uint64_t)hi << 32) | lo);
  __asm__ volatile("" : "+s"(q));
  return (T*)q;
}

// Wave-level synchronization of LDS traffic (workgroup-scope fences only: no cache
// write-back, just ordering of this wave's LDS accesses).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// A wave-uniform value (say, a kernel's argument block) read from the first active lane, one
// 32-bit word at a time: scalar registers instead of vector ones wherever the compiler had
// loaded it with vector loads.
template <typename T>
__device__ __forceinline__ T wave_uniform(const T& v) {
  static_assert(sizeof(T) % 4 == 0, "whole 32-bit words");
  uint32_t w[sizeof(T) / 4];
  __builtin_memcpy(w, &v, sizeof(T));
#pragma unroll
  for (int i = 0; i < (int)(sizeof(T) / 4); ++i) w[i] = (uint32_t)__builtin_amdgcn_readfirstlane((int)w[i]);
  T r;
  __builtin_memcpy(&r, w, sizeof(T));
  return r;
}

// Lane `src`'s value (src uniform) in every lane of the wave.
__device__ __forceinline__ double wave_bcast(double v, int src) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, src);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), src);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

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

// sum_{b < count} p[b * stride] in the order b = 0, 1, ...; the loads go in groups of 32,
// then of 8, issued before their adds (one memory round trip per group instead of one per
// term: a tail summing 32 first-level partials waits for one).
__device__ __forceinline__ double sum_strided(const double* p_, size_t stride, int count) {
  gbl<const double>* __restrict__ p = G(p_);
  double acc = 0.0;
  int b = 0;
  for (; b + 32 <= count; b += 32) {
    double v[32];
#pragma unroll
    for (int u = 0; u < 32; ++u) v[u] = p[(size_t)(b + u) * stride];
#pragma unroll
    for (int u = 0; u < 32; ++u) acc += v[u];
  }
  for (; b + 8 <= count; b += 8) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = p[(size_t)(b + u) * stride];
#pragma unroll
    for (int u = 0; u < 8; ++u) acc += v[u];
  }
  for (; b < count; ++b) acc += p[(size_t)b * stride];
  return acc;
}

// Deterministic cross-block reduction, run by ONE block of a separate "tail" kernel
// (the kernel boundary makes the partials of the streaming kernel visible; no
// device-scope fence is executed -- on gfx950 such a fence writes back the L2 of
// the XCD, which per block of a streaming kernel costs far more than a launch).
//   out[e] = sum_{b < nblocks} part1[b * E + e]   for e < E,
// with G = min(nt / E, nblocks) threads per entry each summing a contiguous range of
// blocks, then the G partial sums combined in group order: the summation order
// depends only on (E, nblocks, blockDim), never on timing.  scratch: >= blockDim
// doubles of LDS.  Must be called by all threads; ends with a barrier.
__device__ void block_sum_partials(const double* __restrict__ part1, int E, int nblocks,
                                   double* out, double* scratch) {
  const int tid = threadIdx.x, nt = blockDim.x;
  if (E >= nt || nblocks == 1) {
    for (int e = tid; e < E; e += nt) out[e] = sum_strided(part1 + e, E, nblocks);
    __syncthreads();
    return;
  }
  const int G = min(nt / E, nblocks);
  const int chunk = (nblocks + G - 1) / G;
  if (tid < G * E) {
    const int e = tid % E, g = tid / E;
    const int b0 = g * chunk, b1 = min(nblocks, b0 + chunk);
    scratch[g * E + e] = sum_strided(part1 + (size_t)b0 * E + e, E, b1 - b0);
  }
  __syncthreads();
  for (int e = tid; e < E; e += nt) {
    double acc = 0.0;
    for (int g = 0; g < G; ++g) acc += scratch[g * E + e];
    out[e] = acc;
  }
  __syncthreads();
}

// block_sum_partials for the tail kernels, inline: the same thread groups, block ranges and
// summation order, the loads in unconditional groups of 16 (rows clamped to the range, so a
// branch never waits on a load) to bound the registers held in flight.
__device__ __forceinline__ double strided_sum16(gbl<const double>* p, int E, int e, int b0, int b1) {
  double acc = 0.0;
  for (int b = b0; b < b1; b += 16) {
    double v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) v[u] = p[(size_t)min(b + u, b1 - 1) * E + e];
#pragma unroll
    for (int u = 0; u < 16; ++u)
      if (b + u < b1) acc += v[u];
  }
  return acc;
}
__device__ __forceinline__ void tail_sum_partials(const double* part1, int E, int nblocks, double* out,
                                                  double* scratch) {
  const int tid = threadIdx.x, nt = blockDim.x;
  gbl<const double>* p = G(part1);
  if (E >= nt || nblocks == 1) {
    for (int e = tid; e < E; e += nt) out[e] = strided_sum16(p, E, e, 0, nblocks);
    __syncthreads();
    return;
  }
  const int ng = min(nt / E, nblocks), chunk = (nblocks + ng - 1) / ng;
  if (tid < ng * E) {
    const int e = tid % E, g = tid / E;
    const int b0 = g * chunk, b1 = min(nblocks, b0 + chunk);
    scratch[g * E + e] = strided_sum16(p, E, e, b0, b1);
  }
  __syncthreads();
  for (int e = tid; e < E; e += nt) {
    double acc = 0.0;
    for (int g = 0; g < ng; ++g) acc += scratch[g * E + e];
    out[e] = acc;
  }
  __syncthreads();
}

// The same sum in two halves when every thread's share is at most 16 partials (E < blockDim.x
// and a block range of at most 16): partials_load issues all of this thread's loads at once,
// so that the caller can wait for other memory together with them, and partials_sum adds
// them in the same order.  partials_load returns false (nothing loaded) in other cases.
struct PartialLoads {
  double v[16];
};
__device__ __forceinline__ bool partials_load(const double* part1, int E, int nblocks, PartialLoads& pl) {
  const int tid = threadIdx.x, nt = blockDim.x;
  if (E >= nt || nblocks <= 1 || E <= 0) return false;
  const int ng = min(nt / E, nblocks), chunk = (nblocks + ng - 1) / ng;
  if (chunk > 16) return false;
  const int e = tid % E, g = tid / E;
  const int b0 = min(g * chunk, nblocks - 1);
  // unconditional loads, rows clamped to the last block (in bounds for every thread);
  // partials_sum adds only this thread's own rows
  gbl<const double>* __restrict__ p = G(part1);
#pragma unroll
  for (int u = 0; u < 16; ++u) pl.v[u] = p[(size_t)min(b0 + u, nblocks - 1) * E + e];
  return true;
}
__device__ __forceinline__ void partials_sum(const PartialLoads& pl, int E, int nblocks, double* out,
                                             double* scratch) {
  const int tid = threadIdx.x, nt = blockDim.x;
  const int ng = min(nt / E, nblocks), chunk = (nblocks + ng - 1) / ng;
  const int e = tid % E, g = tid / E;
  const int b0 = g * chunk, b1 = min(nblocks, b0 + chunk);
  double acc = 0.0;
#pragma unroll
  for (int u = 0; u < 16; ++u)
    if (b0 + u < b1) acc += pl.v[u];
  if (tid < ng * E) scratch[g * E + e] = acc;
  __syncthreads();
  for (int x = tid; x < E; x += nt) {
    double t = 0.0;
    for (int q = 0; q < ng; ++q) t += scratch[q * E + x];
    out[x] = t;
  }
  __syncthreads();
}

}  // namespace tsg
