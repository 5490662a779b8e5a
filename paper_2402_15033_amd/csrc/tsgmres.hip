// C ABI and host driver of the tsgmres library (s-step GMRES with two-stage block
// orthogonalization, arXiv:2402.15033) for AMD MI355X (gfx950).
//
// The host only enqueues kernels on the caller's stream and, once per restart cycle,
// reads back the 64-byte StateHead; every numerical decision (convergence, breakdown,
// truncation) is taken on the device by the tails of the reduction kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/tsgmres.h"
#include "kernels.hpp"
#include "stream.hpp"

using namespace tsg;

struct tsg_csr_s {
  int64_t n, nnz;
  const int32_t* row_ptr;
  const int32_t* col;
  const double* val;
  double lo, hi;
  double* dev;  // 4 KiB: Gershgorin partials scratch of the final reduce
};

namespace {

thread_local std::string g_err;

tsg_status fail(tsg_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

#define HIP_TRY(expr)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess) return fail(TSG_ERR_HIP, "%s failed: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

#define HIP_LAUNCH_CHECK()                                                              \
  do {                                                                                  \
    hipError_t e_ = hipGetLastError();                                                  \
    if (e_ != hipSuccess) return fail(TSG_ERR_HIP, "kernel launch failed: %s", hipGetErrorString(e_)); \
  } while (0)

constexpr size_t kAlign = 256;
inline size_t align_up(size_t x, size_t a = kAlign) { return (x + a - 1) / a * a; }
inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Leading dimension of a basis with n rows: a multiple of 64 elements; a column
// stride that is a multiple of 64 KiB elements gets 64 more so that the 8 columns
// read side by side by one block do not all start on the same HBM channel.
int64_t basis_ld(int64_t n) {
  int64_t ld = (n + 63) / 64 * 64;
  if (ld % 65536 == 0) ld += 64;
  return ld;
}

constexpr int kMaxReduceBlocks = 512;  // largest grid of any reduction kernel (MFMA Gram)

// Workspace carving shared by solve and orthogonalize.
struct Carve {
  char* base;
  size_t off = 0;
  template <typename T>
  T* take(size_t count) {
    T* p = reinterpret_cast<T*>(base + off);
    off = align_up(off + count * sizeof(T));
    return p;
  }
};

constexpr int kReduceGroups = 32;  // first-level groups of the two-level cross-block reduction

struct Common {
  SmallState* st;
  double* part1;  // per-block partial sums of the streaming kernels
  double* part2;  // per-group partial sums (two-level reduction)
  size_t part1_n;
};

size_t part1_count(int64_t n) {
  return std::max<size_t>((size_t)kMaxReduceBlocks * kMaxCols * kMaxNz, (size_t)cdiv(n, kRowBlock));
}

size_t common_bytes(int64_t n) {
  return align_up(sizeof(SmallState)) + align_up(part1_count(n) * sizeof(double)) +
         align_up((size_t)kReduceGroups * kMaxCols * kMaxNz * sizeof(double));
}

Common carve_common(Carve& cv, int64_t n) {
  Common c;
  c.part1_n = part1_count(n);
  c.st = cv.take<SmallState>(1);
  c.part1 = cv.take<double>(c.part1_n);
  c.part2 = cv.take<double>((size_t)kReduceGroups * kMaxCols * kMaxNz);
  return c;
}
__global__ void zero_f64_kernel(double* p, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

#define TRY(x)                  \
  do {                          \
    tsg_status s_ = (x);        \
    if (s_ != TSG_OK) return s_; \
  } while (0)

// ------------------------------------------------------------------ timing
// Per kernel class (TSG_KC_*): HIP events around every launch on the solve's stream,
// folded into totals after each per-cycle synchronization.
struct Timer {
  bool on = false;  // time the launches enqueued now
  struct Pair {
    int cls;
    double bytes;
    hipEvent_t b, e;
  };
  std::vector<Pair> pairs;  // launches of the current enqueue (one cycle, or the captured graph)
  std::vector<hipEvent_t> spare;
  double ms[16] = {0};
  int64_t count[16] = {0};
  double bytes[16] = {0};
  hipError_t err = hipSuccess;  // first failed event call (reported by the caller)
  ~Timer() {
    for (auto& p : pairs) {
      (void)hipEventDestroy(p.b);
      (void)hipEventDestroy(p.e);
    }
    for (auto e : spare) (void)hipEventDestroy(e);
  }
  hipEvent_t make() {
    if (!spare.empty()) {
      hipEvent_t e = spare.back();
      spare.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
  void begin(hipStream_t s, int c, double nbytes) {
    if (!on) return;
    Pair p{c, nbytes, make(), make()};
    if (!p.b || !p.e) {
      if (err == hipSuccess) err = hipErrorOutOfMemory;
      (void)hipGetLastError();
    } else {
      note(hipEventRecord(p.b, s));
    }
    pairs.push_back(p);
  }
  void end(hipStream_t s) {
    if (!on || pairs.empty()) return;
    if (pairs.back().e) note(hipEventRecord(pairs.back().e, s));
  }
  void note(hipError_t e) {
    if (e == hipSuccess) return;
    if (err == hipSuccess) err = e;
    (void)hipGetLastError();  // keep the launch checks about launches
  }
  // after a stream synchronization: fold the pairs' elapsed times into the totals
  void harvest() {
    for (auto& p : pairs) {
      float t = 0.f;
      if (p.b && p.e && hipEventElapsedTime(&t, p.b, p.e) == hipSuccess) ms[p.cls] += t;
      count[p.cls] += 1;
      bytes[p.cls] += p.bytes;
      if (p.b) spare.push_back(p.b);
      if (p.e) spare.push_back(p.e);
    }
    pairs.clear();
  }
};

// ------------------------------------------------------------------ panel launchers
struct PanelCtx {
  void* V;
  int64_t ld, n;
  int elem;  // sizeof(T)
  bool f32;
  Common c;
  hipStream_t stream;
  Timer* timer;
  int standalone;
};

// Round a panel width up to an instantiated template width.
int s_template(int sw) { return sw <= 6 ? sw : (sw <= 8 ? 8 : (sw <= 10 ? 10 : (sw <= 12 ? 12 : 16))); }
constexpr int kMaxGramNz = kMaxNz;  // widest lean reduction (two 16-wide MFMA tiles)
constexpr int kMaxMfmaBlocks = 512;  // two 8-wave blocks per CU
static_assert(kMaxMfmaBlocks <= kMaxReduceBlocks,
              "reduction partial buffer too small");

// Panel widths with a fused-kernel instantiation (a panel runs in the smallest one >= sw).
int fused_s(int sw) { return sw <= 1 ? 1 : sw <= 2 ? 2 : sw <= 4 ? 4 : sw <= 5 ? 5 : sw <= 8 ? 8 : sw <= 10 ? 10 : 16; }
// Columns staged by the fused kernel (Q only when the step projects or reduces against it).
template <typename T, int MT>
void launch_fused_mt(const PanelArgs& a, int nb, hipStream_t s) {
  switch (fused_s(a.sw)) {
    case 1: hipLaunchKernelGGL((panel_mfma_kernel<T, MT, 1>), dim3(nb), dim3(512), 0, s, a); break;
    case 2: hipLaunchKernelGGL((panel_mfma_kernel<T, MT, 2>), dim3(nb), dim3(512), 0, s, a); break;
    case 4: hipLaunchKernelGGL((panel_mfma_kernel<T, MT, 4>), dim3(nb), dim3(512), 0, s, a); break;
    case 5: hipLaunchKernelGGL((panel_mfma_kernel<T, MT, 5>), dim3(nb), dim3(512), 0, s, a); break;
    case 8: hipLaunchKernelGGL((panel_mfma_kernel<T, MT, 8>), dim3(nb), dim3(512), 0, s, a); break;
    case 10: hipLaunchKernelGGL((panel_mfma_kernel<T, MT, 10>), dim3(nb), dim3(512), 0, s, a); break;
    default: hipLaunchKernelGGL((panel_mfma_kernel<T, MT, 16>), dim3(nb), dim3(512), 0, s, a); break;
  }
}
// ncolA: columns on the A side of the fused kernel's Gram ([Q, q] or q alone)
template <typename T>
void launch_fused(const PanelArgs& a, int ncolA, int nb, hipStream_t s) {
  switch ((ncolA + 15) / 16) {
    case 1: launch_fused_mt<T, 1>(a, nb, s); break;
    case 2: launch_fused_mt<T, 2>(a, nb, s); break;
    case 3: launch_fused_mt<T, 3>(a, nb, s); break;
    default: launch_fused_mt<T, 4>(a, nb, s); break;
  }
}
template <typename T, int MT>
void launch_gram_mt(const PanelArgs& a, int nb, hipStream_t s) {
  if (a.nz <= 16) hipLaunchKernelGGL((gram_mfma_kernel<T, MT, 1>), dim3(nb), dim3(512), 0, s, a);
  else hipLaunchKernelGGL((gram_mfma_kernel<T, MT, 2>), dim3(nb), dim3(512), 0, s, a);
}
template <typename T>
void launch_gram(const PanelArgs& a, int nb, hipStream_t s) {
  switch ((a.k + a.sw + 15) / 16) {
    case 1: launch_gram_mt<T, 1>(a, nb, s); break;
    case 2: launch_gram_mt<T, 2>(a, nb, s); break;
    case 3: launch_gram_mt<T, 3>(a, nb, s); break;
    default: launch_gram_mt<T, 4>(a, nb, s); break;
  }
}
template <typename T>
void launch_update(const PanelArgs& a, int nb, hipStream_t s) {
  switch (s_template(a.sw)) {
    case 1: hipLaunchKernelGGL((update_kernel<T, 1>), dim3(nb), dim3(256), 0, s, a); break;
    case 2: hipLaunchKernelGGL((update_kernel<T, 2>), dim3(nb), dim3(256), 0, s, a); break;
    case 3: hipLaunchKernelGGL((update_kernel<T, 3>), dim3(nb), dim3(256), 0, s, a); break;
    case 4: hipLaunchKernelGGL((update_kernel<T, 4>), dim3(nb), dim3(256), 0, s, a); break;
    case 5: hipLaunchKernelGGL((update_kernel<T, 5>), dim3(nb), dim3(256), 0, s, a); break;
    case 6: hipLaunchKernelGGL((update_kernel<T, 6>), dim3(nb), dim3(256), 0, s, a); break;
    case 8: hipLaunchKernelGGL((update_kernel<T, 8>), dim3(nb), dim3(256), 0, s, a); break;
    case 10: hipLaunchKernelGGL((update_kernel<T, 10>), dim3(nb), dim3(256), 0, s, a); break;
    case 12: hipLaunchKernelGGL((update_kernel<T, 12>), dim3(nb), dim3(256), 0, s, a); break;
    default: hipLaunchKernelGGL((update_kernel<T, 16>), dim3(nb), dim3(256), 0, s, a); break;
  }
}

enum PanelKind { PK_GRAM, PK_UPDATE, PK_FUSED };

struct Step {
  PanelKind kind;
  int k, wcol, sw;
  int nprev = 0;      // PK_GRAM: previous-panel columns reduced along (stage-2 Gram block)
  int flags = 0;
  int tail = TAIL_NONE;
  int panel = 0, kkeep = 0, gate = 1;
  int kclass = -1;
};

// One panel step: the streaming kernel and, when it reduces, the one-block tail kernel.
tsg_status run_step(const PanelCtx& p, const Step& st) {
  PanelArgs a{};
  a.V = p.V;
  a.ld = p.ld;
  a.n = p.n;
  a.k = st.k;
  a.wcol = st.wcol;
  a.sw = st.sw;
  a.flags = st.flags;
  a.tail = st.tail;
  a.gate = st.gate;
  a.standalone = p.standalone;
  a.kkeep = st.kkeep;
  a.panel = st.panel;
  a.st = p.c.st;
  a.part1 = p.c.part1;
  bool reduces = false;
  int nb = 0;
  double cols = 0;
  int kc = st.kclass;
  if (st.kind == PK_UPDATE) {
    a.nz = st.sw;
    nb = (int)cdiv(p.n, 256);
    a.rows_per_block = 256;
    a.nblocks = nb;
    cols = ((st.flags & PF_HAS_P) ? st.k : 0) + 2.0 * st.sw;
    if (kc < 0) kc = TSG_KC_UPDATE;
  } else {
    const bool gram = st.kind == PK_GRAM;
    a.nz = gram ? st.nprev + st.sw : st.sw;
    const int rpl = p.f32 ? tile_rows_per_lane<float>() : tile_rows_per_lane<double>();
    const bool loadQ = (st.flags & (PF_HAS_P | PF_GRAM_Q)) != 0;
    const int staged = gram ? st.k + st.sw : (loadQ ? st.k : 0) + st.sw;
    const int br = kWave * rpl * (kTileItems / staged);  // the MFMA kernels' batch height
    int64_t tiles = cdiv(p.n, br);
    nb = (int)std::min<int64_t>(tiles, kMaxMfmaBlocks);
    a.rows_per_block = cdiv(cdiv(p.n, nb), br) * br;
    nb = (int)cdiv(p.n, a.rows_per_block);
    a.nblocks = nb;
    if (gram) {
      reduces = true;
      cols = st.k + st.sw;
      if (kc < 0) kc = st.nprev > 0 ? TSG_KC_GRAM : TSG_KC_GRAM_FIRST;
    } else {
      reduces = true;
      cols = staged + ((st.flags & PF_STORE) ? st.sw : 0);
      if (kc < 0) kc = TSG_KC_FUSED;
    }
  }
  if (a.nz > kMaxGramNz || st.k + st.sw > kMaxCols)
    return fail(TSG_ERR_UNSUPPORTED, "internal: reduction of %d x %d columns", st.k + st.sw, a.nz);
  if (reduces && (size_t)nb * (size_t)((st.k + st.sw) * a.nz) > p.c.part1_n)
    return fail(TSG_ERR_WORKSPACE, "internal: reduction partials (%d blocks x %d) exceed the buffer", nb,
                (st.k + st.sw) * a.nz);
  const bool fb = kc == TSG_KC_FALLBACK;
  if (p.timer) p.timer->begin(p.stream, kc, fb ? 0.0 : cols * (double)p.n * p.elem);
  switch (st.kind) {
    case PK_GRAM:
      if (p.f32) launch_gram<float>(a, nb, p.stream);
      else launch_gram<double>(a, nb, p.stream);
      break;
    case PK_UPDATE:
      if (p.f32) launch_update<float>(a, nb, p.stream);
      else launch_update<double>(a, nb, p.stream);
      break;
    case PK_FUSED: {
      const int ncolA = (st.flags & PF_GRAM_Q) ? st.k + st.sw : st.sw;
      if (p.f32) launch_fused<float>(a, ncolA, nb, p.stream);
      else launch_fused<double>(a, ncolA, nb, p.stream);
    } break;
  }
  if (p.timer) p.timer->end(p.stream);
  HIP_LAUNCH_CHECK();
  if (reduces) {
    if (p.timer) p.timer->begin(p.stream, fb ? TSG_KC_FALLBACK : TSG_KC_TAIL, 0.0);
    PanelArgs at = a;
    if (nb > 2 * kReduceGroups) {  // two-level: many blocks sum the partials first
      const int chunk = (int)cdiv(nb, kReduceGroups);
      const int ng = (int)cdiv(nb, chunk);
      hipLaunchKernelGGL(partial_reduce_kernel, dim3(ng), dim3(256), 0, p.stream, a, p.c.part2, chunk);
      at.part1 = p.c.part2;
      at.nblocks = ng;
    }
    hipLaunchKernelGGL(panel_tail_kernel, dim3(1), dim3(kTailThreads), 0, p.stream, at);
    if (p.timer) p.timer->end(p.stream);
    HIP_LAUNCH_CHECK();
  }
  return TSG_OK;
}

// A reduction over the k + sw columns (lean kernel when it fits, else the fused kernel in
// reduce-only mode).
Step gram_step(int k, int wcol, int sw, int nprev, int tail, int panel, int kkeep, int gate = 1) {
  Step st{};
  st.kind = PK_GRAM;
  st.nprev = nprev;
  st.k = k;
  st.wcol = wcol;
  st.sw = sw;
  st.tail = tail;
  st.panel = panel;
  st.kkeep = kkeep;
  st.gate = gate;
  return st;
}
Step upd_step(PanelKind kind, int k, int wcol, int sw, int flags, int tail, int panel, int kkeep) {
  Step st{};
  st.kind = kind;
  st.k = k;
  st.wcol = wcol;
  st.sw = sw;
  st.flags = flags;
  st.tail = tail;
  st.panel = panel;
  st.kkeep = kkeep;
  return st;
}

// The kernel sequence of one panel (columns wcol .. wcol+sw-1 against the k before them).
//   two_stage: stage-1 BCGS-PIP; the reduction also covers the previous panel's stage-2
//              Gram block column when nprev > 0; the last panel's update is fused with
//              its own stage-2 Gram block column.
//   others:    as in the paper's figures, with fused passes where the next reduction
//              reads exactly the columns just written.
tsg_status panel_sequence(const PanelCtx& p, int ortho, int k, int sw, int nprev, bool fuse_update, int j,
                          int kkeep) {
  const int c0 = k;
  switch (ortho) {
    case TSG_ORTHO_TWO_STAGE: {
      // stage-1 BCGS-PIP; in solver mode followed by the explicit second pass, whose
      // launches return at entry unless this panel's PIP pivot failed (gate 2)
      const int passes = p.standalone ? 1 : 2;
      for (int pass = 0; pass < passes; ++pass) {
        const int gate = pass == 0 ? 1 : 2;
        Step g = gram_step(k, c0, sw, pass == 0 ? nprev : 0, pass == 0 ? TAIL_PIP : TAIL_PIP_FB, j,
                           kkeep, gate);
        if (pass == 1) g.kclass = TSG_KC_FALLBACK;
        TRY(run_step(p, g));
        Step u = fuse_update ? upd_step(PK_FUSED, k, c0, sw, PF_HAS_P | PF_HAS_T | PF_STORE | PF_GRAM_Q | PF_GRAM_W,
                                        TAIL_G2COL, j, kkeep)
                             : upd_step(PK_UPDATE, k, c0, sw, PF_HAS_P | PF_HAS_T | PF_STORE, TAIL_NONE, j, kkeep);
        u.gate = gate;
        if (pass == 1) u.kclass = TSG_KC_FALLBACK;
        TRY(run_step(p, u));
      }
    } break;
    case TSG_ORTHO_BCGS_PIP2:
      TRY(run_step(p, gram_step(k, c0, sw, 0, TAIL_PIP2_A, j, kkeep)));
      TRY(run_step(p, upd_step(PK_FUSED, k, c0, sw, PF_HAS_P | PF_HAS_T | PF_STORE | PF_GRAM_Q | PF_GRAM_W,
                               TAIL_PIP2_B, j, kkeep)));
      TRY(run_step(p, upd_step(PK_UPDATE, k, c0, sw, PF_HAS_P | PF_HAS_T | PF_STORE, TAIL_NONE, j, kkeep)));
      break;
    case TSG_ORTHO_BCGS2_CHOLQR2:
      TRY(run_step(p, gram_step(k, c0, sw, 0, TAIL_BC_P1, j, kkeep)));
      TRY(run_step(p, upd_step(PK_FUSED, k, c0, sw, PF_HAS_P | PF_STORE | PF_GRAM_W, TAIL_BC_A1, j, kkeep)));
      TRY(run_step(p, upd_step(PK_FUSED, 0, c0, sw, PF_HAS_T | PF_STORE | PF_GRAM_W, TAIL_BC_A2, j, kkeep)));
      TRY(run_step(p, upd_step(PK_FUSED, k, c0, sw, PF_HAS_T | PF_STORE | PF_GRAM_Q | PF_GRAM_W, TAIL_BC_P2, j,
                               kkeep)));
      TRY(run_step(p, upd_step(PK_FUSED, k, c0, sw, PF_HAS_P | PF_STORE | PF_GRAM_W, TAIL_BC_C, j, kkeep)));
      TRY(run_step(p, upd_step(PK_UPDATE, 0, c0, sw, PF_HAS_T | PF_STORE, TAIL_NONE, j, kkeep)));
      break;
    case TSG_ORTHO_CGS2:
      TRY(run_step(p, gram_step(k, c0, 1, 0, TAIL_CGS_H1, j, kkeep)));
      TRY(run_step(p, upd_step(PK_FUSED, k, c0, 1, PF_HAS_P | PF_STORE | PF_GRAM_Q | PF_GRAM_W, TAIL_CGS_H2, j,
                               kkeep)));
      TRY(run_step(p, upd_step(PK_UPDATE, k, c0, 1, PF_HAS_P | PF_HAS_T | PF_STORE, TAIL_NONE, j, kkeep)));
      break;
  }
  return TSG_OK;
}


}  // namespace

// =================================================================== C ABI
// (the entry points keep the C linkage of their declarations in tsgmres.h)

const char* tsg_status_string(tsg_status st) {
  switch (st) {
    case TSG_OK: return "ok";
    case TSG_NOT_CONVERGED: return "not converged";
    case TSG_BREAKDOWN: return "breakdown";
    case TSG_ERR_INVALID_ARG: return "invalid argument";
    case TSG_ERR_HIP: return "HIP runtime error";
    case TSG_ERR_WORKSPACE: return "workspace too small or misaligned";
    case TSG_ERR_UNSUPPORTED: return "unsupported";
  }
  return "unknown status";
}

const char* tsg_last_error(void) { return g_err.c_str(); }

tsg_status tsg_csr_create(int64_t n, int64_t nnz, const int32_t* row_ptr, const int32_t* col,
                          const double* val, void* stream, tsg_csr* out) {
  if (!out) return fail(TSG_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (n < 1 || nnz < 0 || nnz >= (int64_t(1) << 31) || n >= (int64_t(1) << 31))
    return fail(TSG_ERR_INVALID_ARG, "bad sizes n=%lld nnz=%lld", (long long)n, (long long)nnz);
  if (!row_ptr || (nnz > 0 && (!col || !val)))
    return fail(TSG_ERR_INVALID_ARG, "NULL CSR array");
  hipStream_t s = (hipStream_t)stream;
  tsg_csr A = new (std::nothrow) tsg_csr_s();
  if (!A) return fail(TSG_ERR_INVALID_ARG, "out of host memory");
  A->n = n;
  A->nnz = nnz;
  A->row_ptr = row_ptr;
  A->col = col;
  A->val = val;
  int nb = (int)cdiv(n, kRowBlock);
  double* part = nullptr;
  hipError_t e = hipMalloc(&A->dev, 4096);
  if (e == hipSuccess) e = hipMallocAsync(&part, sizeof(double) * 2 * nb, s);
  if (e != hipSuccess) {
    if (A->dev) (void)hipFree(A->dev);
    delete A;
    return fail(TSG_ERR_HIP, "allocation failed: %s", hipGetErrorString(e));
  }
  hipLaunchKernelGGL(gershgorin_kernel, dim3(nb), dim3(kRowBlock), 0, s, row_ptr, col, val, n, part);
  hipLaunchKernelGGL(minmax_final_kernel, dim3(1), dim3(kRowBlock), 0, s, part, nb, A->dev);
  double lohi[2] = {0, 0};
  e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpyAsync(lohi, A->dev, sizeof(lohi), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipFreeAsync(part, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    (void)hipFree(A->dev);
    delete A;
    return fail(TSG_ERR_HIP, "Gershgorin pass failed: %s", hipGetErrorString(e));
  }
  A->lo = lohi[0];
  A->hi = lohi[1];
  *out = A;
  return TSG_OK;
}

tsg_status tsg_csr_destroy(tsg_csr A) {
  if (!A) return TSG_OK;
  hipError_t e = hipFree(A->dev);
  delete A;
  if (e != hipSuccess) return fail(TSG_ERR_HIP, "hipFree: %s", hipGetErrorString(e));
  return TSG_OK;
}

tsg_status tsg_csr_gershgorin(tsg_csr A, double* lo, double* hi) {
  if (!A || !lo || !hi) return fail(TSG_ERR_INVALID_ARG, "NULL argument");
  *lo = A->lo;
  *hi = A->hi;
  return TSG_OK;
}

tsg_status tsg_spmv(tsg_csr A, const double* x, double* y, void* stream) {
  if (!A || !x || !y) return fail(TSG_ERR_INVALID_ARG, "NULL argument");
  int nb = (int)cdiv(A->n, kRowBlock);
  hipLaunchKernelGGL(spmv_f64_kernel, dim3(nb), dim3(kRowBlock), 0, (hipStream_t)stream,
                     A->row_ptr, A->col, A->val, x, y, A->n);
  HIP_LAUNCH_CHECK();
  return TSG_OK;
}

static tsg_status validate_params(int64_t n, const tsg_solve_params* p) {
  if (!p) return fail(TSG_ERR_INVALID_ARG, "params is NULL");
  if (p->m < 1 || p->m + 1 > kMaxCols) return fail(TSG_ERR_INVALID_ARG, "m=%d outside [1, 63]", p->m);
  if (p->m + 1 > n) return fail(TSG_ERR_INVALID_ARG, "m+1=%d exceeds n=%lld", p->m + 1, (long long)n);
  if (p->ortho < 0 || p->ortho > 3) return fail(TSG_ERR_INVALID_ARG, "bad ortho %d", p->ortho);
  if (p->ortho != TSG_ORTHO_CGS2) {
    if (p->s < 1 || p->s > kMaxS) return fail(TSG_ERR_INVALID_ARG, "s=%d outside [1, 16]", p->s);
    if (p->m % p->s != 0) return fail(TSG_ERR_INVALID_ARG, "s=%d does not divide m=%d", p->s, p->m);
  }
  if (p->s_hat != 0 && p->s_hat != p->m)
    return fail(TSG_ERR_UNSUPPORTED, "s_hat=%d: only s_hat = m is built", p->s_hat);
  if (p->basis < 0 || p->basis > 2) return fail(TSG_ERR_INVALID_ARG, "bad basis %d", p->basis);
  if (p->basis == TSG_BASIS_NEWTON && !p->newton_shifts)
    return fail(TSG_ERR_INVALID_ARG, "newton basis needs newton_shifts");
  if (p->precision < 0 || p->precision > 1) return fail(TSG_ERR_INVALID_ARG, "bad precision");
  if (!(p->tol >= 0.0)) return fail(TSG_ERR_INVALID_ARG, "bad tol");
  if (p->max_iters < 0) return fail(TSG_ERR_INVALID_ARG, "bad max_iters");
  if (p->timing < 0) return fail(TSG_ERR_INVALID_ARG, "bad timing %d", p->timing);
  if (p->flags & ~TSG_FLAG_EAGER) return fail(TSG_ERR_INVALID_ARG, "unknown flags 0x%x", p->flags);
  return TSG_OK;
}

size_t tsg_solve_workspace_bytes(int64_t n, int64_t nnz, const tsg_solve_params* p) {
  if (n < 1 || !p || validate_params(n, p) != TSG_OK) return 0;
  size_t cb = common_bytes(n);
  if (cb == (size_t)-1) return 0;
  size_t elem = p->precision == TSG_PREC_FP32_IR ? 4 : 8;
  size_t basis = align_up((size_t)basis_ld(n) * (p->m + 1) * elem);
  size_t v32 = p->precision == TSG_PREC_FP32_IR ? align_up((size_t)nnz * 4) : 0;
  return cb + basis + v32 + kAlign;
}

namespace {

template <typename T, typename VT>
tsg_status run_solve(tsg_csr A, const double* b, double* x, const tsg_solve_params* p,
                     const Common& c, T* V, int64_t ld, const VT* val, hipStream_t s,
                     tsg_solve_info* info) {
  const int64_t n = A->n;
  const int m = p->m;
  const int ortho = p->ortho;
  const int sstep = (ortho == TSG_ORTHO_CGS2) ? 1 : p->s;
  const int J = m / sstep;
  const bool two = ortho == TSG_ORTHO_TWO_STAGE;
  const bool f32 = sizeof(T) == 4;
  Timer timer;
  const bool timing = p->timing != 0;
  const int64_t stride = p->timing > 1 ? p->timing : 1;  // time every stride-th cycle
  PanelCtx pc{V, ld, n, (int)sizeof(T), f32, c, s, &timer, 0};

  // basis parameters from the Gershgorin interval (Sec. VI uses the monomial basis)
  std::vector<double> theta(sstep), sigma(sstep);
  const double lo = A->lo, hi = A->hi;
  for (int i = 0; i < sstep; ++i) {
    if (ortho == TSG_ORTHO_CGS2) {
      theta[i] = 0.0;
      sigma[i] = 1.0;
    } else if (p->basis == TSG_BASIS_MONOMIAL) {
      theta[i] = 0.0;
      sigma[i] = std::max(std::fabs(lo), std::fabs(hi));
    } else if (p->basis == TSG_BASIS_SHIFTED) {
      theta[i] = 0.5 * (lo + hi);
      sigma[i] = 0.5 * (hi - lo);
    } else {
      theta[i] = p->newton_shifts[i];
      sigma[i] = 0.5 * (hi - lo);
    }
    if (!(sigma[i] > 0.0)) sigma[i] = 1.0;
  }

  // parameters -> device state (head + parameter block only)
  SmallState* hs = new (std::nothrow) SmallState();
  if (!hs) return fail(TSG_ERR_INVALID_ARG, "out of host memory");
  std::memset(hs, 0, sizeof(SmallState));
  hs->h.stop_panel = 1 << 30;
  hs->m = m;
  hs->s = sstep;
  hs->ortho = ortho;
  hs->prec = p->precision;
  hs->max_iters = p->max_iters;
  hs->tol = p->tol;
  hs->pivot_tol = f32 ? kPivotTolF32 : kPivotTolF64;
  for (int i = 0; i < sstep; ++i) {
    hs->theta[i] = theta[i];
    hs->sigma[i] = sigma[i];
  }
  const size_t head_bytes = offsetof(SmallState, Hh);
  hipError_t e = hipMemcpyAsync(c.st, hs, head_bytes, hipMemcpyHostToDevice, s);
  delete hs;
  HIP_TRY(e);
  const int nbr = (int)cdiv(n, kRowBlock);
  hipLaunchKernelGGL(norm_kernel, dim3(nbr), dim3(kRowBlock), 0, s, b, n, c.part1);
  hipLaunchKernelGGL(norm_tail_kernel, dim3(1), dim3(kTailThreads), 0, s, c.st, (const double*)c.part1, nbr);
  HIP_LAUNCH_CHECK();
  double bnorm = 0.0;
  HIP_TRY(hipMemcpyAsync(&bnorm, &c.st->bnorm, sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (bnorm == 0.0) {  // b = 0: x = 0 is the solution
    hipLaunchKernelGGL(zero_f64_kernel, dim3(nbr), dim3(kRowBlock), 0, s, x, n);
    HIP_TRY(hipStreamSynchronize(s));
    if (info) {
      std::memset(info, 0, sizeof(*info));
      info->status = TSG_OK;
    }
    return TSG_OK;
  }

  StateHead* head = nullptr;
  HIP_TRY(hipHostMalloc((void**)&head, sizeof(StateHead), hipHostMallocDefault));
  const double spmv_bytes = (double)(n + 1) * 4 + (double)A->nnz * (4 + sizeof(VT)) + 2.0 * n * sizeof(T);
  const double resid_bytes = (double)(n + 1) * 4 + (double)A->nnz * 12 + 2.0 * n * 8 + n * sizeof(T);
  hipEvent_t t0 = nullptr, t1 = nullptr;
  if (timing) {
    HIP_TRY(hipEventCreate(&t0));
    HIP_TRY(hipEventCreate(&t1));
    HIP_TRY(hipEventRecord(t0, s));
  }


  const bool g00_here = two && 1 + sstep > kMaxGramNz;
  // Every launch of a restart cycle has the same arguments in every cycle (what changes --
  // convergence, truncation after a breakdown, the iteration count -- lives in the device
  // state), so one cycle is enqueued on stream q either directly or into a graph.
  auto enqueue_cycle = [&](hipStream_t q) -> tsg_status {
    pc.stream = q;
    // ---- restart residual r = b - A x, beta, convergence test (explicit, FP64)
    timer.begin(q, TSG_KC_RESIDUAL, resid_bytes);
    hipLaunchKernelGGL((residual_kernel<T>), dim3(nbr), dim3(kRowBlock), 0, q, A->row_ptr, A->col,
                       A->val, x, b, V, n, c.st, c.part1);
    hipLaunchKernelGGL(residual_tail_kernel, dim3(1), dim3(kTailThreads), 0, q, c.st,
                       (const double*)c.part1, nbr);
    timer.end(q);
    HIP_LAUNCH_CHECK();
    // ---- qhat_1 = r / beta (two-stage: its G2(0,0) comes with the first panel's reduction
    //      when column 0 and the panel fit one lean reduction, else from this pass)
    {
      Step sc = upd_step(g00_here ? PK_FUSED : PK_UPDATE, 0, 0, 1,
                         PF_HAS_T | PF_STORE | (g00_here ? PF_GRAM_W : 0), g00_here ? TAIL_NORM0 : TAIL_NONE,
                         -1, 0);
      sc.kclass = TSG_KC_SCALE;
      TRY(run_step(pc, sc));
    }
    for (int j = 0; j < J; ++j) {
      const int k = j * sstep + 1;
      for (int i = 0; i < sstep; ++i) {
        timer.begin(q, TSG_KC_MPK, spmv_bytes);
        hipLaunchKernelGGL((mpk_step_kernel<T, VT>), dim3(nbr), dim3(kRowBlock), 0, q, A->row_ptr, A->col,
                           val, V + (int64_t)(k - 1 + i) * ld, V + (int64_t)(k + i) * ld, n, theta[i],
                           sigma[i], c.st, j);
        timer.end(q);
        HIP_LAUNCH_CHECK();
      }
      // two-stage: the next panel's reduction covers this panel's stage-2 Gram block column
      // when both panels fit one lean reduction; otherwise the update is fused with it
      const bool lean2 = 2 * sstep <= kMaxGramNz;
      const bool covered = j < J - 1 && lean2;
      // previous panel's columns reduced along: column 0 for the first panel, else s
      const int nprev = !two ? 0 : (j == 0 ? (g00_here ? 0 : 1) : (lean2 ? sstep : 0));
      TRY(panel_sequence(pc, ortho, k, sstep, nprev, !covered, j, k - 1));
    }
    // ---- stage 2 (two-stage) / projected least squares; counters
    timer.begin(q, TSG_KC_CYCLE_END, 0.0);
    hipLaunchKernelGGL(cycle_end_kernel, dim3(1), dim3(256), 0, q, c.st, two ? 1 : 0);
    timer.end(q);
    HIP_LAUNCH_CHECK();
    // ---- x += V(:, 0:k_used) coef
    timer.begin(q, TSG_KC_XUPDATE, (double)m * n * sizeof(T) + 16.0 * n);
    hipLaunchKernelGGL((xupdate_kernel<T>), dim3(nbr), dim3(kRowBlock), 0, q, x, V, ld, n, c.st);
    timer.end(q);
    HIP_LAUNCH_CHECK();
    return TSG_OK;
  };

  // graph mode: capture one cycle on a private stream, replay it on s.  A timed cycle is
  // enqueued directly (its events bracket each launch; same kernels and arguments).
  const bool use_graph = (p->flags & TSG_FLAG_EAGER) == 0;
  hipStream_t cs = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  tsg_status result = TSG_OK;
  if (use_graph) {
    hipError_t ge = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (ge == hipSuccess) ge = hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed);
    if (ge == hipSuccess) {
      timer.on = false;
      tsg_status cst = enqueue_cycle(cs);
      ge = hipStreamEndCapture(cs, &graph);
      if (cst != TSG_OK) result = cst;
    }
    if (ge == hipSuccess && result == TSG_OK) ge = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (ge != hipSuccess && result == TSG_OK)
      result = fail(TSG_ERR_HIP, "capture of a restart cycle failed: %s", hipGetErrorString(ge));
  }
  int64_t timed_cycles = 0;
  for (int64_t cyc = 0; result == TSG_OK; ++cyc) {
    timer.on = timing && cyc % stride == 0;
    if (use_graph && !timer.on) {
      e = hipGraphLaunch(exec, s);
      if (e != hipSuccess) {
        result = fail(TSG_ERR_HIP, "hipGraphLaunch: %s", hipGetErrorString(e));
        break;
      }
    } else {
      result = enqueue_cycle(s);
      if (result != TSG_OK) break;
      timed_cycles += timer.on ? 1 : 0;
    }
    e = hipMemcpyAsync(head, &c.st->h, sizeof(StateHead), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
      result = fail(TSG_ERR_HIP, "cycle sync failed: %s", hipGetErrorString(e));
      break;
    }
    if (timer.err != hipSuccess) {
      result = fail(TSG_ERR_HIP, "timing event: %s", hipGetErrorString(timer.err));
      break;
    }
    timer.harvest();
    if (head->done) break;
  }
  if (exec) (void)hipGraphExecDestroy(exec);
  if (graph) (void)hipGraphDestroy(graph);
  if (cs) (void)hipStreamDestroy(cs);
  if (timing && result == TSG_OK) {
    (void)hipEventRecord(t1, s);
    (void)hipEventSynchronize(t1);
    float tot = 0.f;
    (void)hipEventElapsedTime(&tot, t0, t1);
    if (info) info->ms_total = tot;
  }
  if (t0) (void)hipEventDestroy(t0);
  if (t1) (void)hipEventDestroy(t1);
  StateHead h = *head;
  (void)hipHostFree(head);
  if (result != TSG_OK) return result;
  tsg_status st = h.status == 0 ? TSG_OK : (h.status == 1 ? TSG_NOT_CONVERGED : TSG_BREAKDOWN);
  if (info) {
    double ms_total = info->ms_total;
    std::memset(info, 0, sizeof(*info));
    info->iters = h.iters;
    info->cycles = h.cycles;
    info->relres = h.relres;
    info->relres_est = h.est;
    info->status = st;
    info->truncated_cycles = h.truncated;
    info->pip_fallbacks = h.fallbacks;
    if (timing) {
      info->ms_total = ms_total;
      info->timed_cycles = timed_cycles;
      auto& T_ = timer;
      info->ms_spmv = T_.ms[TSG_KC_MPK];
      info->ms_ortho_reduce = T_.ms[TSG_KC_GRAM] + T_.ms[TSG_KC_GRAM_FIRST];
      info->ms_ortho_update = T_.ms[TSG_KC_UPDATE] + T_.ms[TSG_KC_FUSED];
      info->ms_small = T_.ms[TSG_KC_TAIL] + T_.ms[TSG_KC_CYCLE_END];
      info->ms_xupdate = T_.ms[TSG_KC_XUPDATE];
      info->ms_residual = T_.ms[TSG_KC_RESIDUAL] + T_.ms[TSG_KC_SCALE];
      info->n_ortho_reduce = T_.count[TSG_KC_GRAM] + T_.count[TSG_KC_GRAM_FIRST];
      info->n_ortho_update = T_.count[TSG_KC_UPDATE] + T_.count[TSG_KC_FUSED];
      info->n_spmv = T_.count[TSG_KC_MPK];
      info->bytes_ortho_reduce = T_.bytes[TSG_KC_GRAM] + T_.bytes[TSG_KC_GRAM_FIRST];
      info->bytes_ortho_update = T_.bytes[TSG_KC_UPDATE] + T_.bytes[TSG_KC_FUSED];
      info->bytes_spmv = T_.bytes[TSG_KC_MPK];
      for (int i = 0; i < TSG_KC_COUNT; ++i) {
        info->kc_ms[i] = T_.ms[i];
        info->kc_launches[i] = T_.count[i];
        info->kc_bytes[i] = T_.bytes[i];
      }
    }
  }
  return st;
}

}  // namespace

tsg_status tsg_solve(tsg_csr A, const double* b, double* x, const tsg_solve_params* p, void* workspace,
                     size_t ws_bytes, void* stream, tsg_solve_info* info) {
  if (!A || !b || !x) return fail(TSG_ERR_INVALID_ARG, "NULL argument");
  TRY(validate_params(A->n, p));
  if (!workspace) return fail(TSG_ERR_INVALID_ARG, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(workspace) % kAlign != 0)
    return fail(TSG_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  size_t need = tsg_solve_workspace_bytes(A->n, A->nnz, p);
  if (need == 0) return fail(TSG_ERR_INVALID_ARG, "problem too large for the reduction buffers");
  if (ws_bytes < need) return fail(TSG_ERR_WORKSPACE, "workspace %zu < required %zu", ws_bytes, need);
  hipStream_t s = (hipStream_t)stream;
  Carve cv{(char*)workspace};
  Common c = carve_common(cv, A->n);
  const int64_t ld = basis_ld(A->n);
  if (p->precision == TSG_PREC_FP32_IR) {
    float* V = cv.take<float>((size_t)ld * (p->m + 1));
    float* v32 = cv.take<float>((size_t)std::max<int64_t>(A->nnz, 1));
    if (A->nnz > 0) {
      hipLaunchKernelGGL(to_f32_kernel, dim3(cdiv(A->nnz, kRowBlock)), dim3(kRowBlock), 0, s, A->val, v32,
                         A->nnz);
      HIP_LAUNCH_CHECK();
    }
    return run_solve<float, float>(A, b, x, p, c, V, ld, v32, s, info);
  }
  double* V = cv.take<double>((size_t)ld * (p->m + 1));
  return run_solve<double, double>(A, b, x, p, c, V, ld, A->val, s, info);
}

size_t tsg_orthogonalize_workspace_bytes(int64_t n, int32_t k, int32_t s) {
  if (n < 1 || k < 1 || k > kMaxCols || s < 1 || s > kMaxS) return 0;
  size_t cb = common_bytes(n);
  if (cb == (size_t)-1) return 0;
  return cb + kAlign;
}

tsg_status tsg_orthogonalize(int64_t n, int32_t k, double* X, int64_t ldx, double* R, int32_t ldr,
                             int32_t s, int32_t s_hat, int32_t algo, void* workspace, size_t ws_bytes,
                             void* stream, double* orth_err) {
  if (!X || !R || !workspace) return fail(TSG_ERR_INVALID_ARG, "NULL argument");
  if (n < 1 || k < 1 || k > kMaxCols || k > n)
    return fail(TSG_ERR_INVALID_ARG, "need 1 <= k <= min(n, 64): n=%lld k=%d", (long long)n, k);
  if (ldx < n || ldr < k) return fail(TSG_ERR_INVALID_ARG, "leading dimension too small");
  if (s < 1 || s > kMaxS) return fail(TSG_ERR_INVALID_ARG, "s=%d outside [1, 16]", s);
  if (algo != TSG_ORTHO_TWO_STAGE && algo != TSG_ORTHO_BCGS_PIP2 && algo != TSG_ORTHO_BCGS2_CHOLQR2)
    return fail(TSG_ERR_INVALID_ARG, "bad algo %d", algo);
  if (algo == TSG_ORTHO_TWO_STAGE && s_hat != 0 && s_hat != k - 1)
    return fail(TSG_ERR_UNSUPPORTED, "s_hat=%d: only one big panel (s_hat = k-1) is built", s_hat);
  if (reinterpret_cast<uintptr_t>(workspace) % kAlign != 0)
    return fail(TSG_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  size_t need = tsg_orthogonalize_workspace_bytes(n, k, s);
  if (need == 0) return fail(TSG_ERR_INVALID_ARG, "problem too large for the reduction buffers");
  if (ws_bytes < need) return fail(TSG_ERR_WORKSPACE, "workspace %zu < required %zu", ws_bytes, need);
  hipStream_t st = (hipStream_t)stream;
  Carve cv{(char*)workspace};
  Common c = carve_common(cv, n);
  const bool two = algo == TSG_ORTHO_TWO_STAGE;

  SmallState* hs = new (std::nothrow) SmallState();
  if (!hs) return fail(TSG_ERR_INVALID_ARG, "out of host memory");
  std::memset(hs, 0, sizeof(SmallState));
  hs->h.stop_panel = 1 << 30;
  hs->pivot_tol = 0.0;  // stand-alone: fail only when a Gram is not positive definite
  hipError_t e = hipMemcpyAsync(c.st, hs, offsetof(SmallState, Hh), hipMemcpyHostToDevice, st);
  delete hs;
  HIP_TRY(e);
  hipLaunchKernelGGL(zero_f64_kernel, dim3(cdiv(kLd * kLd, 256)), dim3(256), 0, st, c.st->Hh,
                     (int64_t)kLd * kLd);
  hipLaunchKernelGGL(zero_f64_kernel, dim3(cdiv(kLd * kLd, 256)), dim3(256), 0, st, c.st->G2,
                     (int64_t)kLd * kLd);
  HIP_LAUNCH_CHECK();
  PanelCtx pc{X, ldx, n, 8, false, c, st, nullptr, 1};
  // column 1 alone
  TRY(run_step(pc, gram_step(0, 0, 1, 0, TAIL_SA_NORM, -1, 0)));
  // two-stage with panels: G2(0,0) comes with the first panel's reduction when column 0 and
  // the first panel fit one lean reduction
  const bool g00 = two && (k == 1 || 1 + std::min(s, k - 1) > kMaxGramNz);
  TRY(run_step(pc, upd_step(g00 ? PK_FUSED : PK_UPDATE, 0, 0, 1, PF_HAS_T | PF_STORE | (g00 ? PF_GRAM_W : 0),
                            g00 ? TAIL_NORM0 : TAIL_NONE, -1, 0)));
  const bool lean2 = 2 * s <= kMaxGramNz;
  for (int c0 = 1; c0 < k; c0 += s) {
    const int sw = std::min(s, k - c0);
    const bool last = c0 + sw >= k;
    // previous columns reduced along: column 0 for the first panel, else the previous panel
    // (panels before the last have width s)
    const int nprev = !two ? 0 : (c0 == 1 ? (g00 ? 0 : 1) : (lean2 ? s : 0));
    TRY(panel_sequence(pc, algo, c0, sw, nprev, last || !lean2, 0, 0));
  }
  if (two) {
    // stage 2: one CholQR over all k columns, then Q = Qhat R2^{-1}
    hipLaunchKernelGGL(sa_stage2_kernel, dim3(1), dim3(256), 0, st, c.st, k);
    HIP_LAUNCH_CHECK();
    const int nb = (int)cdiv(n, kRowBlock);
    // rows are independent; the kernel returns early when the solve is done (breakdown)
    hipLaunchKernelGGL((apply_rinv_kernel<kMaxCols>), dim3(nb), dim3(kRowBlock), 0, st, X, ldx, n, k,
                       (const double*)c.st->Wk);
    HIP_LAUNCH_CHECK();
    hipLaunchKernelGGL(copy_r_kernel, dim3(1), dim3(256), 0, st, c.st, 1, k, R, ldr);
  } else {
    hipLaunchKernelGGL(copy_r_kernel, dim3(1), dim3(256), 0, st, c.st, 0, k, R, ldr);
  }
  HIP_LAUNCH_CHECK();
  if (orth_err) {
    for (int c0 = 0; c0 < k; c0 += kMaxS) {
      const int sw = std::min(kMaxS, k - c0);
      TRY(run_step(pc, gram_step(c0, c0, sw, 0, TAIL_GRAM_OUT, 0, 0, 0)));
    }
    hipLaunchKernelGGL(orth_err_kernel, dim3(1), dim3(256), 0, st, c.st, k);
    HIP_LAUNCH_CHECK();
    HIP_TRY(hipMemcpyAsync(orth_err, &c.st->beta, sizeof(double), hipMemcpyDeviceToHost, st));
  }
  StateHead h{};
  HIP_TRY(hipMemcpyAsync(&h, &c.st->h, sizeof(StateHead), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (h.status == 2) return fail(TSG_BREAKDOWN, "a Gram matrix was not positive definite");
  return TSG_OK;
}
