// C ABI and host-side code of the tsgmres library (s-step GMRES with two-stage block
// orthogonalization, arXiv:2402.15033) for AMD MI355X (gfx950).
//
// The host only enqueues kernels on the caller's stream and, once per restart cycle,
// reads back the 80-byte StateHead; every numerical decision (convergence, breakdown,
// truncation) is taken on the device by the tails of the reduction kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
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
  bool dev_owned = true;  // false for the reordered system of a preconditioner set-up
  std::vector<int32_t> blk_maxw;  // largest row length of each block of kGsBlock rows
  // SELL-64 plan (computed at create) and, once tsg_csr_pack ran, the packed arrays
  int64_t nslices = 0, sell_total = 0;
  int sell_fmt = 0;  // FMT_SELL16 or FMT_SELL32
  std::vector<int64_t> soff_host;
  const int64_t* soff = nullptr;
  const double* v64 = nullptr;
  const float* v32 = nullptr;
  const void* scol = nullptr;
  int packed = 0;
  // multicolor Gauss-Seidel (tsg_csr_precond): row colors and the sweep layout
  int ncolors = 0;
  const int32_t* colors = nullptr;
  // the reordered system P A P^T the preconditioned solve runs on (rows by block, then by
  // color: its own handle with the sweep layout), the permutation and its scratch; all in
  // the caller's buffer of tsg_csr_precond
  tsg_csr_s* pa = nullptr;
  const int32_t* perm = nullptr;  // position p of P A P^T holds row perm[p] of A
  double* gs_tmp = nullptr;       // 2 n doubles for tsg_precond_apply
  const int32_t* gs_prow = nullptr;
  const double* gs_diag = nullptr;
  const double* gs_val = nullptr;
  const int32_t* gs_col = nullptr;
  const int64_t* gs_eoff = nullptr;
  const int32_t* gs_width = nullptr;
  std::vector<int64_t> gs_sloff;  // color c holds slices gs_sloff[c] .. gs_sloff[c+1]-1
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
// stride that is a multiple of 64 Ki elements gets 512 more (4 KiB) so that the columns
// read side by side by one block do not all start on the same HBM channel (measured on
// n = 4194304: 512 beats 64, 128, 256 and 1024 for the panel updates by 2-4%, and the
// solve's orthogonalization by 0.5%).
int64_t basis_ld(int64_t n) {
  int64_t ld = (n + 63) / 64 * 64;
  if (ld % 65536 == 0) ld += 512;
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
#define TRY_OR(x, cleanup)                \
  do {                                    \
    tsg_status s_ = (x);                  \
    if (s_ != TSG_OK) return cleanup(s_); \
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

// ------------------------------------------------------------------ launch programs
// A restart cycle (or a stand-alone orthogonalization) is a fixed sequence of phases; every
// phase is one launch of batched_kernel<Body> over a batch of requests (one request for
// tsg_solve / tsg_orthogonalize, many for the server).  A Program holds the phases and a
// host image of every launch's per-request arguments and block starts; the image is
// copied to the device once, and executing the program only launches kernels, so it can
// be replayed cycle after cycle (or captured into a graph).

// Round a panel width up to an instantiated template width.
int s_template(int sw) { return sw <= 6 ? sw : (sw <= 8 ? 8 : (sw <= 10 ? 10 : (sw <= 12 ? 12 : 16))); }
constexpr int kMaxGramNz = kMaxNz;   // widest lean reduction (two 16-wide MFMA tiles)
constexpr int kMaxMfmaBlocks = 512;  // two 8-wave blocks per CU
// the fused step's registers (two groups of operands in flight) allow one 8-wave block per CU
constexpr int kMaxFusedBlocks = 256;
constexpr int64_t kGsBlock = 8192;   // rows per block of the preconditioned system's order
static_assert(kMaxMfmaBlocks <= kMaxReduceBlocks, "reduction partial buffer too small");
// Device bytes reserved for the launch image of one request's program.
constexpr size_t kProgramBytesPerRequest = 512 * 1024;

enum Family : int {
  F_RESID, F_RTAIL, F_UPDATE, F_MPK, F_GRAM, F_PREDUCE, F_PTAIL, F_FUSED, F_CYCLE_END, F_XUPD, F_S2, F_RITZ,
  F_GSC, F_AXPY
};

struct Phase {
  Family f;
  int t1 = 0, t2 = 0;  // template selectors: S (update), MT/NT (gram), MT/S (fused)
  size_t aoff = 0, boff = 0;
  int blocks = 0;
  int tclass = -1;     // >= 0: a timing span of this kernel class starts at this phase
  double bytes = 0.0;  // algorithmic bytes of that span, all requests
};

struct Program {
  bool f32 = false;
  int nreq = 0;
  std::vector<char> blob;
  std::vector<Phase> phases;
  size_t put(const void* p, size_t bytes) {
    size_t off = align_up(blob.size(), 16);
    blob.resize(off + bytes);
    std::memcpy(blob.data() + off, p, bytes);
    return off;
  }
  template <typename A>
  void add(Family f, int t1, int t2, const std::vector<A>& args, const std::vector<int>& blocks, int tclass,
           double bytes) {
    std::vector<int> bs(args.size() + 1, 0);
    for (size_t r = 0; r < args.size(); ++r) bs[r + 1] = bs[r] + blocks[r];
    if (bs.back() == 0) return;  // no request has work in this phase
    Phase ph;
    ph.f = f;
    ph.t1 = t1;
    ph.t2 = t2;
    ph.aoff = put(args.data(), sizeof(A) * args.size());
    ph.boff = put(bs.data(), sizeof(int) * bs.size());
    ph.blocks = bs.back();
    ph.tclass = tclass;
    ph.bytes = bytes;
    phases.push_back(ph);
  }
};

template <typename Body>
void launch_b(const Phase& ph, const char* d, int nreq, hipStream_t s) {
  hipLaunchKernelGGL((batched_kernel<Body>), dim3(ph.blocks), dim3(Body::kThreads), 0, s,
                     reinterpret_cast<const typename Body::Args*>(d + ph.aoff),
                     reinterpret_cast<const int*>(d + ph.boff), nreq);
}
template <typename T, int B>
void launch_update(const Phase& ph, const char* d, int nreq, hipStream_t s) {
  switch (ph.t1) {
    case 1: launch_b<UpdateBody<T, 1, B>>(ph, d, nreq, s); break;
    case 2: launch_b<UpdateBody<T, 2, B>>(ph, d, nreq, s); break;
    case 3: launch_b<UpdateBody<T, 3, B>>(ph, d, nreq, s); break;
    case 4: launch_b<UpdateBody<T, 4, B>>(ph, d, nreq, s); break;
    case 5: launch_b<UpdateBody<T, 5, B>>(ph, d, nreq, s); break;
    case 6: launch_b<UpdateBody<T, 6, B>>(ph, d, nreq, s); break;
    case 8: launch_b<UpdateBody<T, 8, B>>(ph, d, nreq, s); break;
    case 10: launch_b<UpdateBody<T, 10, B>>(ph, d, nreq, s); break;
    case 12: launch_b<UpdateBody<T, 12, B>>(ph, d, nreq, s); break;
    default: launch_b<UpdateBody<T, 16, B>>(ph, d, nreq, s); break;
  }
}
// t1 = MA column tiles, t2 = NT right-hand tiles (MA >= NT)
template <typename T>
void launch_gram(const Phase& ph, const char* d, int nreq, hipStream_t s) {
  if (ph.t2 == 1) {
    switch (ph.t1) {
      case 1: launch_b<GramBody<T, 1, 1>>(ph, d, nreq, s); break;
      case 2: launch_b<GramBody<T, 2, 1>>(ph, d, nreq, s); break;
      case 3: launch_b<GramBody<T, 3, 1>>(ph, d, nreq, s); break;
      case 4: launch_b<GramBody<T, 4, 1>>(ph, d, nreq, s); break;
      default: launch_b<GramBody<T, 5, 1>>(ph, d, nreq, s); break;
    }
  } else {
    switch (ph.t1) {
      case 2: launch_b<GramBody<T, 2, 2>>(ph, d, nreq, s); break;
      case 3: launch_b<GramBody<T, 3, 2>>(ph, d, nreq, s); break;
      case 4: launch_b<GramBody<T, 4, 2>>(ph, d, nreq, s); break;
      default: launch_b<GramBody<T, 5, 2>>(ph, d, nreq, s); break;
    }
  }
}
template <typename T>
void launch_phase_t(const Phase& ph, const char* d, int nreq, hipStream_t s) {
  switch (ph.f) {
    case F_RESID:
      if (ph.t1 == FMT_SELL16) launch_b<ResidBody<T, FMT_SELL16>>(ph, d, nreq, s);
      else if (ph.t1 == FMT_SELL32) launch_b<ResidBody<T, FMT_SELL32>>(ph, d, nreq, s);
      else launch_b<ResidBody<T, FMT_CSR>>(ph, d, nreq, s);
      break;
    case F_RTAIL: launch_b<RTailBody>(ph, d, nreq, s); break;
    case F_MPK:
      if (ph.t1 == FMT_SELL16) launch_b<MpkBody<T, T, FMT_SELL16>>(ph, d, nreq, s);
      else if (ph.t1 == FMT_SELL32) launch_b<MpkBody<T, T, FMT_SELL32>>(ph, d, nreq, s);
      else launch_b<MpkBody<T, T, FMT_CSR>>(ph, d, nreq, s);
      break;
    case F_PREDUCE: launch_b<PReduceBody>(ph, d, nreq, s); break;
    case F_PTAIL: launch_b<PTailBody>(ph, d, nreq, s); break;
    case F_CYCLE_END: launch_b<CycleEndBody>(ph, d, nreq, s); break;
    case F_S2: launch_b<Stage2Body>(ph, d, nreq, s); break;
    case F_RITZ: launch_b<RitzBody>(ph, d, nreq, s); break;
    case F_GSC: launch_b<GsColorBody>(ph, d, nreq, s); break;
    case F_AXPY: launch_b<AxpyBody>(ph, d, nreq, s); break;
    case F_XUPD: launch_b<XupdBody<T>>(ph, d, nreq, s); break;
    case F_UPDATE:
      if (ph.t2) launch_update<T, 256>(ph, d, nreq, s);
      else launch_update<T, 128>(ph, d, nreq, s);
      break;
    case F_GRAM: launch_gram<T>(ph, d, nreq, s); break;
    case F_FUSED:
      switch (ph.t1) {
        case 1: launch_b<FusedBody<T, 1>>(ph, d, nreq, s); break;
        case 2: launch_b<FusedBody<T, 2>>(ph, d, nreq, s); break;
        case 3: launch_b<FusedBody<T, 3>>(ph, d, nreq, s); break;
        default: launch_b<FusedBody<T, 4>>(ph, d, nreq, s); break;
      }
      break;
  }
}

// Launch phases [first, last) of a program whose image is at d (device).
tsg_status exec_program(const Program& P, const char* d, hipStream_t s, Timer* timer, size_t first = 0,
                        size_t last = (size_t)-1) {
  last = std::min(last, P.phases.size());
  bool open = false;
  for (size_t i = first; i < last; ++i) {
    const Phase& ph = P.phases[i];
    if (timer && ph.tclass >= 0) {
      if (open) timer->end(s);
      timer->begin(s, ph.tclass, ph.bytes);
      open = true;
    }
    if (P.f32) launch_phase_t<float>(ph, d, P.nreq, s);
    else launch_phase_t<double>(ph, d, P.nreq, s);
    HIP_LAUNCH_CHECK();
  }
  if (timer && open) timer->end(s);
  return TSG_OK;
}

// One request of a program: its operator, vectors, basis and reduction buffers.
struct ReqCtx {
  int fmt = FMT_CSR;             // operator layout (OpFormat)
  const int32_t* row_ptr = nullptr;  // CSR row pointers, or the packed slice offsets
  const void* col = nullptr;     // CSR columns, or the packed column deltas / columns
  const double* val = nullptr;   // FP64 values (restart residual)
  const void* valT = nullptr;    // values of the basis type (MPK)
  int64_t nnz = 0;               // stored entries (packed: with padding)
  int64_t n_index = 0;           // row pointers or slice offsets (for the byte counts)
  const double* b = nullptr;
  double* x = nullptr;
  void* V = nullptr;
  int64_t ld = 0, n = 0;
  Common c{};
  double theta[kMaxS] = {0}, sigma[kMaxS] = {0};
  bool leja = false;             // Newton shifts from the Ritz values of a cycle
  // right preconditioning by multicolor Gauss-Seidel (NULL colors: none)
  const tsg_csr_s* A = nullptr;
  const int32_t* colors = nullptr;
  double* zp = nullptr;          // M^{-1} w of the current step; M^{-1} t of the cycle update
  double* tp = nullptr;          // V coef of the cycle update
  double* bp = nullptr;          // P b and P x (the solve runs on P A P^T)
  double* xp = nullptr;
};

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

// A reduction over the k + sw columns against the nprev previous-panel columns and W.
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

// Builds the phases of a batch of requests that share the basis type and every step
// parameter; each request keeps its own sizes, buffers and block decomposition.
// The sweep arguments of color c of A's multicolor Gauss-Seidel layout.
GsArgs gs_color_args(const tsg_csr_s* A, int c, const double* w, double* z, const SmallState* st, int panel) {
  const int64_t s0 = A->gs_sloff[c], ns = A->gs_sloff[c + 1] - s0;
  return GsArgs{A->gs_prow, A->gs_diag, A->gs_val, A->gs_col, A->gs_eoff, A->gs_width, s0, w, z, ns, st, panel, 0};
}

struct Builder {
  Program& P;
  std::vector<ReqCtx*> R;
  int standalone = 0;
  int shifted = 0;  // two-stage stage 1 holds the gated pass after a shifted Cholesky QR
  int fast = 0;     // two-stage stage 1 without the gated fallback passes (a failed PIP pivot
                    // asks the host to run the cycle again with the full program)
  int elem() const { return P.f32 ? 4 : 8; }
  // bytes of the operator's index arrays read by one SpMV (CSR: row pointers and int32
  // columns; packed: slice offsets and int16 deltas / int32 columns)
  static double index_bytes(const ReqCtx& q) {
    const double per = q.fmt == FMT_SELL16 ? 2.0 : 4.0;
    return (double)q.n_index * (q.fmt == FMT_CSR ? 4.0 : 8.0) + (double)q.nnz * per;
  }

  // One panel step: the streaming kernel and, when it reduces, the tail (after a
  // first-level reduction for requests with more than 64 blocks).
  tsg_status step(const Step& st) {
    const size_t nr = R.size();
    std::vector<PanelArgs> a(nr);
    std::vector<int> nb(nr);
    double bytes = 0.0;
    bool reduces = false;
    int kc = st.kclass;
    const bool gram = st.kind == PK_GRAM;
    const bool loadQ = (st.flags & (PF_HAS_P | PF_GRAM_Q)) != 0;
    const int nz = gram ? st.nprev + st.sw : st.sw;
    if (nz > kMaxGramNz || st.k + st.sw > kMaxCols)
      return fail(TSG_ERR_UNSUPPORTED, "internal: reduction of %d x %d columns", st.k + st.sw, nz);
    for (size_t r = 0; r < nr; ++r) {
      const ReqCtx& q = *R[r];
      PanelArgs& x = a[r];
      x = PanelArgs{};
      x.V = q.V;
      x.ld = q.ld;
      x.n = q.n;
      x.k = st.k;
      x.wcol = st.wcol;
      x.sw = st.sw;
      x.flags = st.flags;
      x.tail = st.tail;
      x.gate = st.gate;
      x.standalone = standalone;
      x.kkeep = st.kkeep;
      x.panel = st.panel;
      x.st = q.c.st;
      x.part1 = q.c.part1;
      x.nz = nz;
      x.shifted = shifted;
      x.fast = fast;
      double cols;
      if (st.kind == PK_UPDATE) {
        x.rows_per_block = st.gate >= 2 ? 256 : 128;  // the kernel's block (see UpdateBody)
        nb[r] = (int)cdiv(q.n, x.rows_per_block);
        cols = ((st.flags & PF_HAS_P) ? st.k : 0) + 2.0 * st.sw;
      } else if (gram) {
        const int ma = gram_tiles(st.k + st.sw, nz);
        const int64_t groups = cdiv(q.n, kGramGroupRows);
        const int b0 = (int)std::min<int64_t>(groups, gram_max_blocks(ma));
        x.rows_per_block = cdiv(cdiv(q.n, b0), kGramGroupRows) * kGramGroupRows;
        nb[r] = (int)cdiv(q.n, x.rows_per_block);
        cols = st.k + st.sw;
        reduces = true;
        if ((size_t)nb[r] * (size_t)((st.k + st.sw) * nz) > q.c.part1_n)
          return fail(TSG_ERR_WORKSPACE, "internal: reduction partials (%d blocks x %d) exceed the buffer", nb[r],
                      (st.k + st.sw) * nz);
      } else {
        const int staged = (st.flags & PF_BMAT) ? st.k + st.sw : (loadQ ? st.k : 0) + st.sw;
        const int64_t groups = cdiv(q.n, kFusedGroupRows);
        const int b0 = (int)std::min<int64_t>(groups, kMaxFusedBlocks);
        x.rows_per_block = cdiv(cdiv(q.n, b0), kFusedGroupRows) * kFusedGroupRows;
        nb[r] = (int)cdiv(q.n, x.rows_per_block);
        cols = staged + ((st.flags & PF_STORE) ? st.sw : 0);
        reduces = (st.flags & (PF_GRAM_Q | PF_GRAM_W)) != 0;
        if ((size_t)nb[r] * (size_t)((st.k + st.sw) * nz) > q.c.part1_n)
          return fail(TSG_ERR_WORKSPACE, "internal: reduction partials (%d blocks x %d) exceed the buffer", nb[r],
                      (st.k + st.sw) * nz);
      }
      x.nblocks = nb[r];
      bytes += cols * (double)q.n * elem();
    }
    if (kc < 0) kc = st.kind == PK_UPDATE ? TSG_KC_UPDATE : (gram ? (st.nprev > 0 ? TSG_KC_GRAM : TSG_KC_GRAM_FIRST) : TSG_KC_FUSED);
    const bool fb = kc == TSG_KC_FALLBACK;
    if (st.kind == PK_UPDATE) {
      P.add(F_UPDATE, s_template(st.sw), st.gate >= 2 ? 1 : 0, a, nb, kc, fb ? 0.0 : bytes);
    } else if (gram) {
      P.add(F_GRAM, gram_tiles(st.k + st.sw, nz), nz <= 16 ? 1 : 2, a, nb, kc, fb ? 0.0 : bytes);
    } else {
      const int staged = (st.flags & (PF_HAS_P | PF_GRAM_Q | PF_BMAT)) ? st.k + st.sw : st.sw;
      P.add(F_FUSED, (staged + 15) / 16, 0, a, nb, kc, fb ? 0.0 : bytes);
    }
    if (!reduces) return TSG_OK;
    // first level for requests with many blocks, then the tail.  The gated passes (which
    // almost always return at entry) skip the first level: their tail sums every block's
    // partial itself, one launch less per panel when they are off
    std::vector<RedArgs> ra(nr);
    std::vector<int> rb(nr, 0), one(nr, 1);
    std::vector<PanelArgs> at(a);
    for (size_t r = 0; r < nr; ++r) {
      ra[r] = RedArgs{a[r], R[r]->c.part2, 0, 0};
      if (nb[r] > 2 * kReduceGroups && st.gate < 2) {
        const int chunk = (int)cdiv(nb[r], kReduceGroups);
        rb[r] = (int)cdiv(nb[r], chunk);
        ra[r].chunk = chunk;
        at[r].part1 = R[r]->c.part2;
        at[r].nblocks = rb[r];
      }
    }
    const int tc = fb ? TSG_KC_FALLBACK : TSG_KC_TAIL;
    size_t before = P.phases.size();
    P.add(F_PREDUCE, 0, 0, ra, rb, tc, 0.0);
    P.add(F_PTAIL, 0, 0, at, one, P.phases.size() > before ? -1 : tc, 0.0);
    return TSG_OK;
  }

  // restart residual r = b - A x into column 0, beta, convergence test, cycle set-up.
  // One launch per operator layout present in the batch.
  void resid() {
    for (int fmt = FMT_CSR; fmt <= FMT_SELL32; ++fmt) {
      std::vector<ResidArgs> a;
      std::vector<int> nb;
      double bytes = 0.0;
      for (ReqCtx* q : R) {
        const bool mine = q->fmt == fmt;
        a.push_back(ResidArgs{q->row_ptr, q->col, q->val, q->x, q->b, q->V, q->n, q->c.st, q->c.part1});
        nb.push_back(mine ? (int)cdiv(q->n, kRowBlock) : 0);
        if (mine) bytes += index_bytes(*q) + (double)q->nnz * 8 + 2.0 * q->n * 8 + (double)q->n * elem();
      }
      P.add(F_RESID, fmt, 0, a, nb, TSG_KC_RESIDUAL, bytes);
    }
    std::vector<TailArgs> t;
    std::vector<int> one(R.size(), 1);
    for (ReqCtx* q : R) t.push_back(TailArgs{q->c.st, q->c.part1, (int)cdiv(q->n, kRowBlock), 0});
    P.add(F_RTAIL, 0, 0, t, one, -1, 0.0);
  }
  // z = M^{-1} w (one multicolor Gauss-Seidel sweep) for the preconditioned requests:
  // w(q), z(q) give each request's vectors; panel gates as the matrix-powers steps do
  template <typename FW, typename FZ>
  void gs(FW w_of, FZ z_of, int panel) {
    bool any = false;
    int maxc = 0;
    for (ReqCtx* q : R)
      if (q->colors) {
        any = true;
        maxc = std::max(maxc, q->A->ncolors);
      }
    if (!any) return;
    for (int c = 0; c < maxc; ++c) {
      std::vector<GsArgs> a;
      std::vector<int> nb;
      double bytes = 0.0;
      for (ReqCtx* q : R) {
        const bool on = q->colors != nullptr && c < q->A->ncolors;
        const GsArgs g = on ? gs_color_args(q->A, c, w_of(q), z_of(q), q->c.st, panel) : GsArgs{};
        a.push_back(g);
        nb.push_back(on ? (int)cdiv(g.n, 4) : 0);
        if (on) {  // slot rows and diagonals, w, z, and the lower-color entries (value,
                   // column, z gather): about half of the off-diagonals over the colors
          const int64_t s0 = q->A->gs_sloff[c], s1 = q->A->gs_sloff[c + 1];
          const double rows = (double)(s1 - s0) * kWave;
          bytes += rows * (4.0 + 8.0 + 8.0 + 8.0) + 10.0 * (double)(q->A->nnz - q->n) * rows / (double)q->n;
        }
      }
      P.add(F_GSC, 0, 0, a, nb, TSG_KC_PRECOND, bytes);
    }
  }
  // w_{i+1} = (A w_i - theta_i w_i + tau_i w_{i-1}) / sigma_i into column col_out
  // (preconditioned: A M^{-1} w_i, the sweep into zp first)
  void mpk(int col_in, int col_out, int i, int panel) {
    auto colp = [&](ReqCtx* q, int c) { return static_cast<char*>(q->V) + (size_t)c * q->ld * elem(); };
    gs([&](ReqCtx* q) { return reinterpret_cast<const double*>(colp(q, col_in)); }, [](ReqCtx* q) { return q->zp; },
       panel);
    for (int fmt = FMT_CSR; fmt <= FMT_SELL32; ++fmt) {
      std::vector<MpkArgs> a;
      std::vector<int> nb;
      double bytes = 0.0;
      for (ReqCtx* q : R) {
        const bool mine = q->fmt == fmt;
        char* V = static_cast<char*>(q->V);
        const void* win = V + (size_t)col_in * q->ld * elem();
        a.push_back(MpkArgs{q->row_ptr, q->col, q->valT, q->colors ? (const void*)q->zp : win,
                            V + (size_t)col_out * q->ld * elem(),
                            i > 0 ? V + (size_t)(col_in - 1) * q->ld * elem() : nullptr, win, q->n, q->c.st, i,
                            panel});
        nb.push_back(mine ? (int)cdiv(q->n, kRowBlock) : 0);
        if (mine) bytes += index_bytes(*q) + (double)q->nnz * elem() + 2.0 * q->n * elem();
      }
      P.add(F_MPK, fmt, 0, a, nb, TSG_KC_MPK, bytes);
    }
  }
  // stage 2 of big panel [b0, b1) (s_hat < m), then Y(:, b0:b1) <- Y(:, :b1) Bs in
  // 16-column chunks from the last to the first (a chunk reads only columns before its
  // end, none of which a later-launched chunk has overwritten)
  tsg_status big_stage2(int b0, int b1, int panel) {
    std::vector<S2Args> t;
    std::vector<int> one(R.size(), 1);
    for (ReqCtx* q : R) t.push_back(S2Args{q->c.st, b0, b1, panel, standalone ? 1 : 0});
    P.add(F_S2, 0, 0, t, one, TSG_KC_STAGE2, 0.0);
    const int nchunks = (b1 - b0 + 15) / 16;
    for (int ch = nchunks - 1; ch >= 0; --ch) {
      const int o0 = b0 + 16 * ch, sw = std::min(16, b1 - o0);
      Step ap = upd_step(PK_FUSED, o0, o0, sw, PF_BMAT | PF_STORE, TAIL_NONE, panel, 0);
      ap.kclass = TSG_KC_STAGE2;
      TRY(step(ap));
    }
    return TSG_OK;
  }
  void cycle_end(int two) {
    std::vector<TailArgs> t;
    std::vector<int> one(R.size(), 1);
    bool leja = false;
    for (ReqCtx* q : R) {
      t.push_back(TailArgs{q->c.st, nullptr, 0, two});
      leja = leja || q->leja;
    }
    P.add(F_CYCLE_END, 0, 0, t, one, TSG_KC_CYCLE_END, 0.0);
    // Newton shifts from this cycle's Ritz values (returns at entry unless pending)
    if (leja) P.add(F_RITZ, 0, 0, t, one, TSG_KC_CYCLE_END, 0.0);
  }
  // x += Q coef; preconditioned: t = Q coef, z = M^{-1} t, x += z
  void xupdate(int m) {
    std::vector<XupdArgs> a;
    std::vector<int> nb;
    double bytes = 0.0;
    bool any = false;
    for (ReqCtx* q : R) {
      a.push_back(XupdArgs{q->x, q->V, q->ld, q->n, q->c.st, q->colors ? q->tp : nullptr});
      nb.push_back((int)cdiv(q->n, kRowBlock));
      bytes += (double)m * q->n * elem() + 16.0 * q->n;
      any = any || q->colors;
    }
    P.add(F_XUPD, 0, 0, a, nb, TSG_KC_XUPDATE, bytes);
    if (!any) return;
    gs([](ReqCtx* q) { return (const double*)q->tp; }, [](ReqCtx* q) { return q->zp; }, -1);
    std::vector<AxpyArgs> x;
    std::vector<int> xb;
    double xbytes = 0.0;
    for (ReqCtx* q : R) {
      x.push_back(AxpyArgs{q->x, q->zp, q->n, q->c.st});
      xb.push_back(q->colors ? (int)cdiv(q->n, 256) : 0);
      if (q->colors) xbytes += 24.0 * q->n;
    }
    P.add(F_AXPY, 0, 0, x, xb, TSG_KC_XUPDATE, xbytes);
  }
};

// The kernel sequence of one panel (columns wcol .. wcol+sw-1 against the k before them).
//   two_stage: stage-1 BCGS-PIP; the reduction also covers the previous panel's stage-2
//              Gram block column when nprev > 0; the last panel's update is fused with
//              its own stage-2 Gram block column.
//   others:    as in the paper's figures, with fused passes where the next reduction
//              reads exactly the columns just written.
tsg_status panel_sequence(Builder& B, int ortho, int k, int sw, int nprev, bool fuse_update, int j, int kkeep) {
  const int c0 = k;
  switch (ortho) {
    case TSG_ORTHO_TWO_STAGE: {
      // stage-1 BCGS-PIP; in solver mode followed by the explicit second pass, whose
      // launches return at entry unless this panel's PIP pivot failed (gate 2), and where
      // enabled by the pass after a shifted Cholesky QR, which runs only when the explicit
      // pass failed too (gate 3)
      const int passes = (B.standalone || B.fast) ? 1 : (B.shifted ? 3 : 2);
      for (int pass = 0; pass < passes; ++pass) {
        const int gate = pass + 1;
        const int tail = pass == 0 ? TAIL_PIP : (pass == 1 ? TAIL_PIP_FB : TAIL_PIP_FB2);
        Step g = gram_step(k, c0, sw, pass == 0 ? nprev : 0, tail, j, kkeep, gate);
        if (pass >= 1) g.kclass = TSG_KC_FALLBACK;
        TRY(B.step(g));
        Step u = fuse_update ? upd_step(PK_FUSED, k, c0, sw, PF_HAS_P | PF_HAS_T | PF_STORE | PF_GRAM_Q | PF_GRAM_W,
                                        TAIL_G2COL, j, kkeep)
                             : upd_step(PK_UPDATE, k, c0, sw, PF_HAS_P | PF_HAS_T | PF_STORE, TAIL_NONE, j, kkeep);
        u.gate = gate;
        if (pass >= 1) u.kclass = TSG_KC_FALLBACK;
        TRY(B.step(u));
      }
    } break;
    case TSG_ORTHO_BCGS_PIP2:
      TRY(B.step(gram_step(k, c0, sw, 0, TAIL_PIP2_A, j, kkeep)));
      TRY(B.step(upd_step(PK_FUSED, k, c0, sw, PF_HAS_P | PF_HAS_T | PF_STORE | PF_GRAM_Q | PF_GRAM_W, TAIL_PIP2_B, j,
                          kkeep)));
      TRY(B.step(upd_step(PK_UPDATE, k, c0, sw, PF_HAS_P | PF_HAS_T | PF_STORE, TAIL_NONE, j, kkeep)));
      break;
    case TSG_ORTHO_BCGS2_CHOLQR2:
      TRY(B.step(gram_step(k, c0, sw, 0, TAIL_BC_P1, j, kkeep)));
      TRY(B.step(upd_step(PK_FUSED, k, c0, sw, PF_HAS_P | PF_STORE | PF_GRAM_W, TAIL_BC_A1, j, kkeep)));
      TRY(B.step(upd_step(PK_FUSED, 0, c0, sw, PF_HAS_T | PF_STORE | PF_GRAM_W, TAIL_BC_A2, j, kkeep)));
      TRY(B.step(upd_step(PK_FUSED, k, c0, sw, PF_HAS_T | PF_STORE | PF_GRAM_Q | PF_GRAM_W, TAIL_BC_P2, j, kkeep)));
      TRY(B.step(upd_step(PK_FUSED, k, c0, sw, PF_HAS_P | PF_STORE | PF_GRAM_W, TAIL_BC_C, j, kkeep)));
      TRY(B.step(upd_step(PK_UPDATE, 0, c0, sw, PF_HAS_T | PF_STORE, TAIL_NONE, j, kkeep)));
      break;
    case TSG_ORTHO_CGS2:
      TRY(B.step(gram_step(k, c0, 1, 0, TAIL_CGS_H1, j, kkeep)));
      TRY(B.step(upd_step(PK_FUSED, k, c0, 1, PF_HAS_P | PF_STORE | PF_GRAM_Q | PF_GRAM_W, TAIL_CGS_H2, j, kkeep)));
      TRY(B.step(upd_step(PK_UPDATE, k, c0, 1, PF_HAS_P | PF_HAS_T | PF_STORE, TAIL_NONE, j, kkeep)));
      break;
  }
  return TSG_OK;
}

// The phases of a two-stage restart cycle with big panels of s_hat < m columns (the first
// holds column 0 too): stage 1 per panel as with s_hat = m -- each reduction also carries
// the previous panel's stage-2 Gram block column when that panel is in the same big
// panel, and a panel that ends a big panel forms its own block column in its (fused)
// update -- then at the end of each big panel its stage 2 (tail + explicit Q).  A stage-1
// breakdown keeps the final columns of the completed big panels.
tsg_status build_cycle_big_panels(Builder& B, int m, int sstep, int s_hat) {
  const int J = m / sstep;
  B.resid();
  {
    Step sc = upd_step(PK_UPDATE, 0, 0, 1, PF_HAS_T | PF_STORE, TAIL_NONE, -1, 0);
    sc.kclass = TSG_KC_SCALE;
    TRY(B.step(sc));
  }
  int b0 = 0, b1 = 1 + s_hat;
  for (int j = 0; j < J; ++j) {
    const int k = j * sstep + 1;
    for (int i = 0; i < sstep; ++i) B.mpk(k - 1 + i, k + i, i, j);
    const bool first_in_big = (k == b0) || (b0 == 0 && k == 1);
    const int nprev = j == 0 ? 1 : (first_in_big ? 0 : sstep);
    const bool ends_big = k + sstep == b1;
    TRY(panel_sequence(B, TSG_ORTHO_TWO_STAGE, k, sstep, nprev, ends_big, j, b0 > 0 ? b0 - 1 : 0));
    if (ends_big) {
      TRY(B.big_stage2(b0, b1, j));
      b0 = b1;
      b1 = b0 + s_hat;
    }
  }
  B.cycle_end(0);  // least squares from the Givens factorization of the final H
  B.xupdate(m);
  return TSG_OK;
}

// The phases of one restart cycle of s-step GMRES(m) with the given orthogonalization.
tsg_status build_cycle(Builder& B, int m, int sstep, int ortho, int s_hat) {
  const bool two = ortho == TSG_ORTHO_TWO_STAGE;
  const int J = m / sstep;
  if (two && s_hat > 0 && s_hat < m) return build_cycle_big_panels(B, m, sstep, s_hat);
  B.resid();
  // qhat_1 = r / beta; two-stage: its G2(0,0) comes with the first panel's reduction when
  // column 0 and the panel fit one lean reduction, else from this pass
  const bool g00_here = two && 1 + sstep > kMaxGramNz;
  {
    Step sc = upd_step(g00_here ? PK_FUSED : PK_UPDATE, 0, 0, 1, PF_HAS_T | PF_STORE | (g00_here ? PF_GRAM_W : 0),
                       g00_here ? TAIL_NORM0 : TAIL_NONE, -1, 0);
    sc.kclass = TSG_KC_SCALE;
    TRY(B.step(sc));
  }
  const bool lean2 = 2 * sstep <= kMaxGramNz;
  for (int j = 0; j < J; ++j) {
    const int k = j * sstep + 1;
    for (int i = 0; i < sstep; ++i) B.mpk(k - 1 + i, k + i, i, j);
    // two-stage: the next panel's reduction covers this panel's stage-2 Gram block column
    // when both panels fit one lean reduction; otherwise the update is fused with it
    const bool covered = j < J - 1 && lean2;
    // previous panel's columns reduced along: column 0 for the first panel, else s
    const int nprev = !two ? 0 : (j == 0 ? (g00_here ? 0 : 1) : (lean2 ? sstep : 0));
    TRY(panel_sequence(B, ortho, k, sstep, nprev, !covered, j, k - 1));
  }
  B.cycle_end(two ? 1 : 0);
  B.xupdate(m);
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

namespace {

// Device bytes of the temporaries of create_impl (Gershgorin partials, slice analysis).
size_t create_tmp_bytes(int64_t n) {
  return align_up(sizeof(double) * 2 * (size_t)cdiv(n, kRowBlock)) + align_up(sizeof(int) * 2 * (size_t)cdiv(n, kWave));
}

// tsg_csr_create's work.  dev4k / tmp: the handle's 4 KiB block and the temporaries
// (create_tmp_bytes), both device memory of the caller (then nothing is allocated and the
// handle does not free dev4k), or NULL (allocated here: the block kept, the temporaries
// stream-ordered and freed before returning).
tsg_status create_impl(int64_t n, int64_t nnz, const int32_t* row_ptr, const int32_t* col, const double* val,
                       hipStream_t s, void* dev4k, void* tmp, tsg_csr* out) {
  *out = nullptr;
  tsg_csr A = new (std::nothrow) tsg_csr_s();
  if (!A) return fail(TSG_ERR_INVALID_ARG, "out of host memory");
  A->n = n;
  A->nnz = nnz;
  A->row_ptr = row_ptr;
  A->col = col;
  A->val = val;
  const int nb = (int)cdiv(n, kRowBlock);
  A->nslices = cdiv(n, kWave);
  double* part = nullptr;
  int* wf = nullptr;
  hipError_t e = hipSuccess;
  if (dev4k) {
    A->dev = static_cast<double*>(dev4k);
    A->dev_owned = false;
    Carve tc{static_cast<char*>(tmp)};
    part = tc.take<double>(2 * (size_t)nb);
    wf = tc.take<int>(2 * (size_t)A->nslices);
  } else {
    e = hipMalloc(&A->dev, 4096);
    if (e == hipSuccess) e = hipMallocAsync(&part, sizeof(double) * 2 * nb, s);
    if (e == hipSuccess) e = hipMallocAsync(&wf, sizeof(int) * 2 * A->nslices, s);
  }
  auto bail = [&](const char* what) {
    (void)hipStreamSynchronize(s);
    if (!dev4k) {
      if (part) (void)hipFree(part);
      if (wf) (void)hipFree(wf);
      if (A->dev) (void)hipFree(A->dev);
    }
    delete A;
    return fail(TSG_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
  };
  if (e != hipSuccess) return bail("allocation failed");
  // Gershgorin interval, then the SELL-64 plan: slice widths and the column-delta range,
  // offsets on the host
  hipLaunchKernelGGL(gershgorin_kernel, dim3(nb), dim3(kRowBlock), 0, s, row_ptr, col, val, n, part);
  hipLaunchKernelGGL(minmax_final_kernel, dim3(1), dim3(kRowBlock), 0, s, part, nb, A->dev);
  hipLaunchKernelGGL(sell_analyze_kernel, dim3(cdiv(A->nslices, kRowBlock / kWave)), dim3(kRowBlock), 0, s, row_ptr,
                     col, n, A->nslices, wf, wf + A->nslices);
  double lohi[2] = {0, 0};
  std::vector<int> wh(2 * A->nslices);
  e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpyAsync(lohi, A->dev, sizeof(lohi), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipMemcpyAsync(wh.data(), wf, sizeof(int) * 2 * A->nslices, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess && !dev4k) e = hipFreeAsync(part, s);
  if (e == hipSuccess && !dev4k) e = hipFreeAsync(wf, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return bail("operator analysis failed");
  A->lo = lohi[0];
  A->hi = lohi[1];
  A->soff_host.resize(A->nslices + 1);
  A->blk_maxw.assign((size_t)cdiv(n, kGsBlock), 0);
  int fits = 1;
  int64_t acc = 0;
  for (int64_t i = 0; i < A->nslices; ++i) {
    A->soff_host[i] = acc;
    acc += (int64_t)kWave * wh[i];
    fits &= wh[A->nslices + i];
    int32_t& bm = A->blk_maxw[(size_t)(i * kWave / kGsBlock)];
    bm = std::max(bm, (int32_t)wh[i]);
  }
  A->soff_host[A->nslices] = acc;
  A->sell_total = acc;
  A->sell_fmt = fits ? FMT_SELL16 : FMT_SELL32;
  *out = A;
  return TSG_OK;
}

}  // namespace

tsg_status tsg_csr_create(int64_t n, int64_t nnz, const int32_t* row_ptr, const int32_t* col,
                          const double* val, void* stream, tsg_csr* out) {
  if (!out) return fail(TSG_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (n < 1 || nnz < 0 || nnz >= (int64_t(1) << 31) || n >= (int64_t(1) << 31))
    return fail(TSG_ERR_INVALID_ARG, "bad sizes n=%lld nnz=%lld", (long long)n, (long long)nnz);
  if (!row_ptr || (nnz > 0 && (!col || !val)))
    return fail(TSG_ERR_INVALID_ARG, "NULL CSR array");
  return create_impl(n, nnz, row_ptr, col, val, (hipStream_t)stream, nullptr, nullptr, out);
}

size_t tsg_csr_pack_bytes(tsg_csr A) {
  if (!A) return 0;
  const size_t t = (size_t)A->sell_total;
  return align_up((A->nslices + 1) * sizeof(int64_t)) + align_up(t * 8) + align_up(t * 4) +
         align_up(t * (A->sell_fmt == FMT_SELL16 ? 2 : 4)) + kAlign;
}

tsg_status tsg_csr_pack(tsg_csr A, void* buf, size_t bytes, void* stream) {
  if (!A) return fail(TSG_ERR_INVALID_ARG, "NULL operator");
  hipStream_t s = (hipStream_t)stream;
  if (!buf) {  // back to the CSR arrays (after the stream's pending solves)
    HIP_TRY(hipStreamSynchronize(s));
    A->packed = 0;
    A->soff = nullptr;
    A->v64 = nullptr;
    A->v32 = nullptr;
    A->scol = nullptr;
    return TSG_OK;
  }
  if (reinterpret_cast<uintptr_t>(buf) % kAlign != 0) return fail(TSG_ERR_WORKSPACE, "buffer must be 256-byte aligned");
  if (bytes < tsg_csr_pack_bytes(A)) return fail(TSG_ERR_WORKSPACE, "buffer %zu < required %zu", bytes, tsg_csr_pack_bytes(A));
  Carve cv{(char*)buf};
  int64_t* soff = cv.take<int64_t>(A->nslices + 1);
  double* v64 = cv.take<double>((size_t)A->sell_total);
  float* v32 = cv.take<float>((size_t)A->sell_total);
  void* scol = A->sell_fmt == FMT_SELL16 ? (void*)cv.take<int16_t>((size_t)A->sell_total)
                                         : (void*)cv.take<int32_t>((size_t)A->sell_total);
  HIP_TRY(hipMemcpyAsync(soff, A->soff_host.data(), sizeof(int64_t) * (A->nslices + 1), hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(sell_fill_kernel, dim3(cdiv(A->nslices * kWave, kRowBlock)), dim3(kRowBlock), 0, s, A->row_ptr,
                     A->col, A->val, A->n, A->nslices, soff, v64, v32, scol, A->sell_fmt);
  HIP_LAUNCH_CHECK();
  A->soff = soff;
  A->v64 = v64;
  A->v32 = v32;
  A->scol = scol;
  A->packed = 1;
  return TSG_OK;
}

tsg_status tsg_csr_destroy(tsg_csr A) {
  if (!A) return TSG_OK;
  hipError_t e = A->dev_owned ? hipFree(A->dev) : hipSuccess;
  if (A->pa) (void)tsg_csr_destroy(A->pa);  // (its memory is the caller's buffer)
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

namespace {

// The regions of tsg_csr_precond's buffer, in bytes: coloring scratch, the reordered system
// and its vectors, its handle block and temporaries, its packed copy, the sweep layout and
// its plan.  The last three depend on the coloring; their sizes are upper bounds from the
// row lengths: with W_b the longest row of block b (kGsBlock rows) and W the longest of all,
//   * packed copy: every 64-row slice at most W wide, 32-bit column offsets;
//   * sweep: the rows of one color within one block form one run, cut into slices of 64,
//     so block b holds at most ceil(rows_b / 64) + C slices (C <= W colors: greedy colors
//     stay below a row's neighbour count plus one), each at most W_b - 1 entries wide (a
//     row's lower-color entries are off-diagonal ones).
struct PrecondLayout {
  size_t color = 0, own = 0, pa_dev = 0, pa_tmp = 0, pack = 0, plan = 0, sweep = 0;
  int64_t max_slices = 0, max_entries = 0;
  size_t total() const { return color + own + pa_dev + pa_tmp + pack + plan + sweep + kAlign; }
};
size_t sweep_plan_bytes(int64_t ns) { return 4 * align_up(8 * (size_t)(ns + 1)) + align_up(4 * (size_t)std::max<int64_t>(ns, 1)); }
size_t sweep_bytes(int64_t ns, int64_t ne) {
  const size_t slots = (size_t)std::max<int64_t>(ns, 1) * kWave, e = (size_t)std::max<int64_t>(ne, 1);
  return align_up(4 * slots) + align_up(8 * slots) + align_up(8 * e) + align_up(4 * e) +
         align_up(8 * (size_t)(ns + 1)) + align_up(4 * (size_t)std::max<int64_t>(ns, 1));
}
PrecondLayout precond_layout(const tsg_csr_s* A) {
  const int64_t n = A->n, nnz = std::max<int64_t>(A->nnz, 1), nb = cdiv(n, 256);
  PrecondLayout L;
  L.color = 2 * align_up(4 * (size_t)n) + align_up(4 * (size_t)nb) + align_up(4);
  L.own = 6 * align_up(4 * (size_t)n + 4) + align_up(4 * (size_t)nnz) + align_up(8 * (size_t)nnz) +
          align_up(16 * (size_t)n);
  L.pa_dev = 4096;
  L.pa_tmp = create_tmp_bytes(n);
  int32_t W = 1;
  for (int32_t w : A->blk_maxw) W = std::max(W, w);
  const int64_t nsl = cdiv(n, kWave);
  const size_t T = (size_t)kWave * nsl * W;
  L.pack = align_up(8 * (size_t)(nsl + 1)) + align_up(8 * T) + align_up(4 * T) + align_up(4 * T) + kAlign;
  for (size_t b = 0; b < A->blk_maxw.size(); ++b) {
    const int64_t rows = std::min<int64_t>(kGsBlock, n - (int64_t)b * kGsBlock);
    const int64_t sl = cdiv(rows, kWave) + W;
    L.max_slices += sl;
    L.max_entries += sl * kWave * std::max<int64_t>(A->blk_maxw[b] - 1, 0);
  }
  L.plan = sweep_plan_bytes(L.max_slices);
  L.sweep = sweep_bytes(L.max_slices, L.max_entries);
  return L;
}

// The sweep layout of handle H: the rows of color c in block b are perm[run(b, c)] (rows of
// H, in increasing order; run(b, c) = [koff[b ncol + c], koff[b ncol + c + 1]) in the
// color-major list perm); colors: the color of every row of H (device); padcol: a row of
// color 0.  Slices of 64 per run, ordered by color then block; widths, entry offsets, then
// the fill, into plan / mem (caller device memory of at least sweep_plan_bytes(max_ns) /
// sweep_bytes(max_ns, max_ne) bytes; the counts are checked against those bounds).
tsg_status build_sweep_layout(tsg_csr_s* H, int ncol, int64_t nblk, const std::vector<int64_t>& run_len,
                              const int32_t* perm, const int32_t* colors, int32_t padcol, void* plan, void* mem,
                              int64_t max_ns, int64_t max_ne, hipStream_t s) {
  std::vector<int64_t> sl((size_t)ncol + 1, 0), ss, se, sc;
  int64_t p = 0;
  for (int c = 0; c < ncol; ++c) {
    for (int64_t b = 0; b < nblk; ++b) {
      const int64_t len = run_len[(size_t)(b * ncol + c)];
      for (int64_t q = 0; q < len; q += kWave) {
        ss.push_back(p + q);
        se.push_back(p + std::min<int64_t>(q + kWave, len));
        sc.push_back(c);
      }
      p += len;
    }
    sl[c + 1] = (int64_t)ss.size();
  }
  const int64_t ns = (int64_t)ss.size();
  if (ns > max_ns) return fail(TSG_ERR_UNSUPPORTED, "internal: %lld sweep slices above the bound %lld", (long long)ns, (long long)max_ns);
  Carve pc{static_cast<char*>(plan)};
  int64_t* dss = pc.take<int64_t>((size_t)ns + 1);
  int64_t* dse = pc.take<int64_t>((size_t)ns + 1);
  int64_t* dsc = pc.take<int64_t>((size_t)ns + 1);
  int64_t* deo = pc.take<int64_t>((size_t)ns + 1);
  int32_t* dwd = pc.take<int32_t>((size_t)std::max<int64_t>(ns, 1));
  std::vector<int32_t> wh((size_t)ns);
  hipError_t e = hipMemcpyAsync(dss, ss.data(), sizeof(int64_t) * ns, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(dse, se.data(), sizeof(int64_t) * ns, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(dsc, sc.data(), sizeof(int64_t) * ns, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(gs_analyze_kernel, dim3(cdiv(ns * kWave, 256)), dim3(256), 0, s, H->row_ptr, H->col, perm,
                       dss, dse, dsc, colors, ns, dwd);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpyAsync(wh.data(), dwd, sizeof(int32_t) * ns, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail(TSG_ERR_HIP, "sweep layout: %s", hipGetErrorString(e));
  std::vector<int64_t> eo((size_t)ns + 1, 0);
  for (int64_t k = 0; k < ns; ++k) eo[k + 1] = eo[k] + (int64_t)kWave * wh[k];
  const int64_t nent = eo[ns];
  if (nent > max_ne) return fail(TSG_ERR_UNSUPPORTED, "internal: %lld sweep entries above the bound %lld", (long long)nent, (long long)max_ne);
  // carved with the bounds' sizes (the same regions whatever the coloring)
  Carve mc{static_cast<char*>(mem)};
  int32_t* prow = mc.take<int32_t>((size_t)std::max<int64_t>(max_ns, 1) * kWave);
  double* diag = mc.take<double>((size_t)std::max<int64_t>(max_ns, 1) * kWave);
  double* gval = mc.take<double>((size_t)std::max<int64_t>(max_ne, 1));
  int32_t* gcol = mc.take<int32_t>((size_t)std::max<int64_t>(max_ne, 1));
  int64_t* geo = mc.take<int64_t>((size_t)max_ns + 1);
  int32_t* gwd = mc.take<int32_t>((size_t)std::max<int64_t>(max_ns, 1));
  e = hipMemcpyAsync(geo, eo.data(), sizeof(int64_t) * (ns + 1), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(deo, eo.data(), sizeof(int64_t) * (ns + 1), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(gwd, dwd, sizeof(int32_t) * ns, hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(gs_fill_kernel, dim3(cdiv(ns * kWave, 256)), dim3(256), 0, s, H->row_ptr, H->col, H->val, perm,
                       dss, dse, dsc, colors, deo, dwd, ns, padcol, prow, diag, gval, gcol);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail(TSG_ERR_HIP, "sweep layout fill: %s", hipGetErrorString(e));
  H->gs_prow = prow;
  H->gs_diag = diag;
  H->gs_val = gval;
  H->gs_col = gcol;
  H->gs_eoff = geo;
  H->gs_width = gwd;
  H->gs_sloff = sl;
  H->ncolors = ncol;
  return TSG_OK;
}

}  // namespace

size_t tsg_csr_precond_bytes(tsg_csr A) { return A ? precond_layout(A).total() : 0; }

tsg_status tsg_csr_precond(tsg_csr A, void* buf, size_t bytes, void* stream) {
  if (!A) return fail(TSG_ERR_INVALID_ARG, "NULL handle");
  if (A->pa) return TSG_OK;  // already set up
  if (!buf) return fail(TSG_ERR_INVALID_ARG, "NULL buffer");
  if (reinterpret_cast<uintptr_t>(buf) % kAlign != 0) return fail(TSG_ERR_WORKSPACE, "buffer must be 256-byte aligned");
  const PrecondLayout L = precond_layout(A);
  if (bytes < L.total()) return fail(TSG_ERR_WORKSPACE, "buffer %zu < required %zu", bytes, L.total());
  hipStream_t s = (hipStream_t)stream;
  const int64_t n = A->n, nnz = A->nnz;
  const int nb = (int)cdiv(n, 256);
  Carve bc{static_cast<char*>(buf)};
  char* r_color = bc.take<char>(L.color);
  char* r_own = bc.take<char>(L.own);
  char* r_padev = bc.take<char>(L.pa_dev);
  char* r_patmp = bc.take<char>(L.pa_tmp);
  char* r_pack = bc.take<char>(L.pack);
  char* r_plan = bc.take<char>(L.plan);
  char* r_sweep = bc.take<char>(L.sweep);
  // ---- coloring: Jones-Plassmann rounds (two color arrays, counts, total)
  Carve cv{r_color};
  int32_t* ca = cv.take<int32_t>((size_t)n);
  int32_t* cb = cv.take<int32_t>((size_t)n);
  int32_t* cnt = cv.take<int32_t>((size_t)nb);
  int32_t* total = cv.take<int32_t>(1);
  tsg_csr pa = nullptr;
  auto bail = [&](tsg_status st) {
    (void)hipStreamSynchronize(s);
    if (pa) (void)tsg_csr_destroy(pa);
    return st;
  };
  hipLaunchKernelGGL(jp_init_kernel, dim3(nb), dim3(256), 0, s, ca, n);
  int32_t *cold = ca, *cnew = cb;
  int32_t left = 1;
  for (int64_t round = 0; left > 0; ++round) {
    if (round > n) return bail(fail(TSG_ERR_UNSUPPORTED, "coloring did not finish in %lld rounds", (long long)n));
    hipLaunchKernelGGL(jp_round_kernel, dim3(nb), dim3(256), 0, s, A->row_ptr, A->col, n, cold, cnew, cnt);
    hipLaunchKernelGGL(jp_total_kernel, dim3(1), dim3(1024), 0, s, cnt, nb, total);
    if (hipGetLastError() != hipSuccess) return bail(fail(TSG_ERR_HIP, "coloring launch failed"));
    if (hipMemcpyAsync(&left, total, sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return bail(fail(TSG_ERR_HIP, "coloring round failed"));
    std::swap(cold, cnew);
  }
  // ---- the order of P A P^T: blocks of kGsBlock consecutive rows, within a block the
  // rows by color, within a color in index order (counting sort on the host).  A color's
  // rows are then one run per block: the SpMV's and the sweep's gathers stay within a
  // block and its neighbours (L2-resident, and column distances small enough for the
  // packed operator's 16-bit deltas on banded operators), while the rows of one color
  // still do not couple.  Also its inverse, the row pointers of P A P^T, and the sweep's
  // row list (color-major: per color its runs in block order).
  std::vector<int32_t> ch((size_t)n), ph((size_t)n), ih((size_t)n), rp((size_t)n + 1), rpp((size_t)n + 1);
  if (hipMemcpyAsync(ch.data(), cold, sizeof(int32_t) * n, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipMemcpyAsync(rp.data(), A->row_ptr, sizeof(int32_t) * (n + 1), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return bail(fail(TSG_ERR_HIP, "reading the colors failed"));
  int ncol = 0;
  for (int64_t i = 0; i < n; ++i) ncol = std::max(ncol, ch[i] + 1);
  const int64_t nblk = cdiv(n, kGsBlock);
  std::vector<int64_t> koff((size_t)(nblk * ncol) + 1, 0);
  for (int64_t i = 0; i < n; ++i) koff[(i / kGsBlock) * ncol + ch[i] + 1] += 1;
  std::vector<int64_t> run_len((size_t)(nblk * ncol));
  for (int64_t k = 0; k < nblk * ncol; ++k) run_len[k] = koff[k + 1];
  for (int64_t k = 0; k < nblk * ncol; ++k) koff[k + 1] += koff[k];
  {
    std::vector<int64_t> pos(koff.begin(), koff.end() - 1);
    for (int64_t i = 0; i < n; ++i) ph[pos[(i / kGsBlock) * ncol + ch[i]]++] = (int32_t)i;
  }
  rpp[0] = 0;
  for (int64_t q = 0; q < n; ++q) {
    ih[ph[q]] = (int32_t)q;
    rpp[q + 1] = rpp[q] + (rp[ph[q] + 1] - rp[ph[q]]);
  }
  std::vector<int32_t> rows_by_color((size_t)n);
  int32_t padcol = -1;
  {
    std::vector<int64_t> off((size_t)ncol + 1, 0);
    for (int64_t i = 0; i < n; ++i) off[ch[i] + 1] += 1;
    for (int c = 0; c < ncol; ++c) off[c + 1] += off[c];
    std::vector<int64_t> pos(off.begin(), off.end() - 1);
    for (int64_t q = 0; q < n; ++q) {
      const int c = ch[ph[q]];
      rows_by_color[pos[c]++] = (int32_t)q;
      if (c == 0 && padcol < 0) padcol = (int32_t)q;
    }
  }
  // ---- colors (index order), perm, inv, P A P^T (CSR), colors of its rows, the sweep's
  // row list, two scratch vectors
  Carve oc{r_own};
  int32_t* colors = oc.take<int32_t>((size_t)n);
  int32_t* perm = oc.take<int32_t>((size_t)n);
  int32_t* inv = oc.take<int32_t>((size_t)n);
  int32_t* row_ptr_p = oc.take<int32_t>((size_t)n + 1);
  int32_t* colors_p = oc.take<int32_t>((size_t)n);
  int32_t* rlist = oc.take<int32_t>((size_t)n);
  int32_t* col_p = oc.take<int32_t>((size_t)std::max<int64_t>(nnz, 1));
  double* val_p = oc.take<double>((size_t)std::max<int64_t>(nnz, 1));
  double* tmp = oc.take<double>(2 * (size_t)n);
  hipError_t e = hipMemcpyAsync(colors, cold, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(perm, ph.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(inv, ih.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(row_ptr_p, rpp.data(), sizeof(int32_t) * (n + 1), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(rlist, rows_by_color.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(permute_csr_kernel, dim3(nb), dim3(256), 0, s, A->row_ptr, A->col, A->val, perm, inv, n,
                       row_ptr_p, col_p, val_p);
    hipLaunchKernelGGL(gather_i32_kernel, dim3(nb), dim3(256), 0, s, colors, perm, colors_p, n);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return bail(fail(TSG_ERR_HIP, "building P A P^T: %s", hipGetErrorString(e)));
  // ---- its own handle (Gershgorin interval, packed copy for the SpMV) and sweep layout,
  // all in the buffer
  TRY_OR(create_impl(n, nnz, row_ptr_p, col_p, val_p, s, r_padev, r_patmp, &pa), bail);
  const size_t pk = tsg_csr_pack_bytes(pa);
  if (pk > L.pack) return bail(fail(TSG_ERR_UNSUPPORTED, "internal: packed copy %zu above the bound %zu", pk, L.pack));
  TRY_OR(tsg_csr_pack(pa, r_pack, pk, stream), bail);
  TRY_OR(build_sweep_layout(pa, ncol, nblk, run_len, rlist, colors_p, padcol, r_plan, r_sweep, L.max_slices,
                            L.max_entries, s),
         bail);
  HIP_TRY(hipStreamSynchronize(s));
  pa->colors = colors_p;
  A->pa = pa;
  A->colors = colors;
  A->perm = perm;
  A->gs_tmp = tmp;
  A->ncolors = ncol;
  return TSG_OK;
}

int32_t tsg_csr_ncolors(tsg_csr A) { return A ? A->ncolors : 0; }

tsg_status tsg_csr_colors(tsg_csr A, int32_t* colors, void* stream) {
  if (!A || !colors) return fail(TSG_ERR_INVALID_ARG, "NULL argument");
  if (!A->colors) return fail(TSG_ERR_INVALID_ARG, "no preconditioner set-up (tsg_csr_precond)");
  HIP_TRY(hipMemcpyAsync(colors, A->colors, sizeof(int32_t) * A->n, hipMemcpyDeviceToDevice, (hipStream_t)stream));
  return TSG_OK;
}

tsg_status tsg_precond_apply(tsg_csr A, const double* w, double* z, void* stream) {
  if (!A || !w || !z) return fail(TSG_ERR_INVALID_ARG, "NULL argument");
  if (!A->pa) return fail(TSG_ERR_INVALID_ARG, "no preconditioner set-up (tsg_csr_precond)");
  if (w == z) return fail(TSG_ERR_INVALID_ARG, "z must not alias w");
  hipStream_t s = (hipStream_t)stream;
  const int64_t n = A->n;
  double *wp = A->gs_tmp, *zp = A->gs_tmp + n;
  hipLaunchKernelGGL(gather_f64_kernel, dim3(cdiv(n, 256)), dim3(256), 0, s, w, A->perm, wp, n);
  for (int c = 0; c < A->pa->ncolors; ++c) {
    const GsArgs g = gs_color_args(A->pa, c, wp, zp, nullptr, -1);
    if (g.n > 0) hipLaunchKernelGGL(gs_color_kernel, dim3(cdiv(g.n, 4)), dim3(256), 0, s, g);
  }
  hipLaunchKernelGGL(scatter_f64_kernel, dim3(cdiv(n, 256)), dim3(256), 0, s, zp, A->perm, z, n);
  HIP_LAUNCH_CHECK();
  return TSG_OK;
}

tsg_status tsg_ritz_newton(const double* H, int64_t ldh, int32_t k, int32_t s, double lo, double hi, double* out,
                           void* stream) {
  if (!H || !out) return fail(TSG_ERR_INVALID_ARG, "NULL argument");
  if (k < 1 || k > kMaxCols - 1 || s < 1 || s > kMaxS || s > k || ldh < k)
    return fail(TSG_ERR_INVALID_ARG, "need 1 <= s <= k <= 63, s <= 16, ldh >= k (k=%d s=%d ldh=%lld)", k, s,
                (long long)ldh);
  hipStream_t st = (hipStream_t)stream;
  hipLaunchKernelGGL(ritz_newton_kernel, dim3(1), dim3(kWave), 0, st, H, ldh, k, s, lo, hi, out);
  HIP_LAUNCH_CHECK();
  double flag = 0.0;
  HIP_TRY(hipMemcpyAsync(&flag, out + 2 * (int64_t)k + 3 * (int64_t)s, sizeof(double), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  return flag == 0.0 ? TSG_OK : fail(TSG_BREAKDOWN, "QR iteration for the Ritz values did not converge");
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
  if (p->s_hat != 0 && p->s_hat != p->m) {
    if (p->ortho != TSG_ORTHO_TWO_STAGE)
      return fail(TSG_ERR_INVALID_ARG, "s_hat=%d is a two-stage parameter", p->s_hat);
    if (p->s_hat < p->s || p->s_hat > p->m || p->s_hat % p->s != 0 || p->m % p->s_hat != 0)
      return fail(TSG_ERR_INVALID_ARG, "need s | s_hat | m (s=%d, s_hat=%d, m=%d)", p->s, p->s_hat, p->m);
  }
  if (p->basis < 0 || p->basis > 3) return fail(TSG_ERR_INVALID_ARG, "bad basis %d", p->basis);
  if (p->basis == TSG_BASIS_NEWTON && !p->newton_shifts)
    return fail(TSG_ERR_INVALID_ARG, "newton basis needs newton_shifts");
  if (p->precision < 0 || p->precision > 1) return fail(TSG_ERR_INVALID_ARG, "bad precision");
  if (!(p->tol >= 0.0)) return fail(TSG_ERR_INVALID_ARG, "bad tol");
  if (p->max_iters < 0) return fail(TSG_ERR_INVALID_ARG, "bad max_iters");
  if (p->timing < 0) return fail(TSG_ERR_INVALID_ARG, "bad timing %d", p->timing);
  if (p->precond < 0 || p->precond > 1) return fail(TSG_ERR_INVALID_ARG, "bad precond %d", p->precond);
  if (p->precond == TSG_PRECOND_MCGS && p->precision != TSG_PREC_FP64)
    return fail(TSG_ERR_INVALID_ARG, "the multicolor Gauss-Seidel preconditioner runs in FP64 only");
  if (p->flags & ~TSG_FLAG_EAGER) return fail(TSG_ERR_INVALID_ARG, "unknown flags 0x%x", p->flags);
  return TSG_OK;
}

// One request's device bytes: reduction buffers and state, basis, FP32 values (mixed form).
static size_t request_bytes(int64_t n, int64_t nnz, const tsg_solve_params* p) {
  size_t cb = common_bytes(n);
  size_t elem = p->precision == TSG_PREC_FP32_IR ? 4 : 8;
  size_t basis = align_up((size_t)basis_ld(n) * (p->m + 1) * elem);
  size_t v32 = p->precision == TSG_PREC_FP32_IR ? align_up((size_t)std::max<int64_t>(nnz, 1) * 4) : 0;
  size_t pre = p->precond == TSG_PRECOND_MCGS ? 4 * align_up((size_t)n * 8) : 0;
  return cb + basis + v32 + pre;
}

size_t tsg_solve_workspace_bytes(int64_t n, int64_t nnz, const tsg_solve_params* p) {
  if (n < 1 || nnz < 0 || !p || validate_params(n, p) != TSG_OK) return 0;
  return request_bytes(n, nnz, p) + kProgramBytesPerRequest + kAlign;
}

namespace {

// Basis parameters from the Gershgorin interval (Sec. VI uses the monomial basis).
// The basis interval: Gershgorin's of A, or [0, 2] for A M^{-1} (right preconditioning).
void basis_interval(const tsg_csr_s* A, const tsg_solve_params* p, double* lo, double* hi) {
  if (p->precond == TSG_PRECOND_MCGS) {
    *lo = 0.0;
    *hi = 2.0;
  } else {
    *lo = A->lo;
    *hi = A->hi;
  }
}

void basis_params(const tsg_csr_s* A, const tsg_solve_params* p, int sstep, double* theta, double* sigma) {
  double lo, hi;
  basis_interval(A, p, &lo, &hi);
  for (int i = 0; i < sstep; ++i) {
    if (p->ortho == TSG_ORTHO_CGS2) {
      theta[i] = 0.0;
      sigma[i] = 1.0;
    } else if (p->basis == TSG_BASIS_MONOMIAL) {
      theta[i] = 0.0;
      sigma[i] = std::max(std::fabs(lo), std::fabs(hi));
    } else if (p->basis == TSG_BASIS_SHIFTED || p->basis == TSG_BASIS_LEJA) {
      theta[i] = 0.5 * (lo + hi);
      sigma[i] = 0.5 * (hi - lo);
    } else {
      theta[i] = p->newton_shifts[i];
      sigma[i] = 0.5 * (hi - lo);
    }
    if (!(sigma[i] > 0.0)) sigma[i] = 1.0;
  }
}

int step_size(const tsg_solve_params* p) { return p->ortho == TSG_ORTHO_CGS2 ? 1 : p->s; }

// Two-stage stage 1 holds the shifted Cholesky QR remedy for s >= 8 and in the mixed
// form: there a numerically full-rank panel can be beyond the explicit second pass;
// smaller FP64 steps with a scaled basis stay far from that limit.
bool shifted_pass(const tsg_solve_params* p) {
  return p->ortho == TSG_ORTHO_TWO_STAGE && (p->s >= 8 || p->precision == TSG_PREC_FP32_IR);
}

// Carve one request's buffers from its workspace region: reduction buffers and state,
// the basis, and (mixed form) the FP32 copy of the values.
void carve_request(char* base, const tsg_csr_s* A, const tsg_solve_params* p, ReqCtx& q) {
  Carve cv{base};
  q.c = carve_common(cv, A->n);
  q.ld = basis_ld(A->n);
  q.n = A->n;
  q.leja = p->basis == TSG_BASIS_LEJA && p->ortho != TSG_ORTHO_CGS2;
  const bool f32 = p->precision == TSG_PREC_FP32_IR;
  if (A->packed) {
    q.fmt = A->sell_fmt;
    q.nnz = A->sell_total;
    q.n_index = A->nslices + 1;
    q.row_ptr = reinterpret_cast<const int32_t*>(A->soff);
    q.col = A->scol;
    q.val = A->v64;
  } else {
    q.fmt = FMT_CSR;
    q.nnz = A->nnz;
    q.n_index = A->n + 1;
    q.row_ptr = A->row_ptr;
    q.col = A->col;
    q.val = A->val;
  }
  if (f32) {
    q.V = cv.take<float>((size_t)q.ld * (p->m + 1));
    float* v32 = cv.take<float>((size_t)std::max<int64_t>(A->nnz, 1));  // CSR form's FP32 copy
    q.valT = A->packed ? (const void*)A->v32 : (const void*)v32;
  } else {
    q.V = cv.take<double>((size_t)q.ld * (p->m + 1));
    q.valT = q.val;
  }
  if (p->precond == TSG_PRECOND_MCGS) {
    q.A = A;
    q.colors = A->colors;  // NULL until tsg_csr_precond: rejected by the entry points
    q.zp = cv.take<double>((size_t)A->n);
    q.tp = cv.take<double>((size_t)A->n);
    q.bp = cv.take<double>((size_t)A->n);
    q.xp = cv.take<double>((size_t)A->n);
  }
}


// Enqueue a request's set-up: device parameters, FP32 values (mixed form), ||b||.
tsg_status init_request(const tsg_csr_s* A, const tsg_solve_params* p, ReqCtx& q, hipStream_t s) {
  const int sstep = step_size(p);
  const bool f32 = p->precision == TSG_PREC_FP32_IR;
  basis_params(A, p, sstep, q.theta, q.sigma);
  SmallState* hs = new (std::nothrow) SmallState();
  if (!hs) return fail(TSG_ERR_INVALID_ARG, "out of host memory");
  std::memset(hs, 0, sizeof(SmallState));
  hs->h.stop_panel = 1 << 30;
  hs->m = p->m;
  hs->s = sstep;
  hs->ortho = p->ortho;
  hs->prec = p->precision;
  hs->max_iters = p->max_iters;
  hs->tol = p->tol;
  hs->pivot_tol = f32 ? kPivotTolF32 : kPivotTolF64;
  hs->pip_tol = f32 ? kPivotTolF32 : kPipTolF64;
  for (int i = 0; i < sstep; ++i) {
    hs->theta[i] = q.theta[i];
    hs->sigma[i] = q.sigma[i];
  }
  basis_interval(A, p, &hs->glo, &hs->ghi);
  hs->ritz_pending = q.leja ? 1 : 0;
  // pageable source: the copy is staged before the call returns
  hipError_t e = hipMemcpyAsync(q.c.st, hs, offsetof(SmallState, Hh), hipMemcpyHostToDevice, s);
  delete hs;
  HIP_TRY(e);
  if (f32 && A->nnz > 0 && !A->packed) {
    hipLaunchKernelGGL(to_f32_kernel, dim3(cdiv(A->nnz, kRowBlock)), dim3(kRowBlock), 0, s, A->val,
                       (float*)q.valT, A->nnz);
  }
  const int nbr = (int)cdiv(q.n, kRowBlock);
  hipLaunchKernelGGL(norm_kernel, dim3(nbr), dim3(kRowBlock), 0, s, q.b, q.n, q.c.part1);
  hipLaunchKernelGGL(norm_tail_kernel, dim3(1), dim3(kTailThreads), 0, s, q.c.st, (const double*)q.c.part1, nbr);
  HIP_LAUNCH_CHECK();
  return TSG_OK;
}

void fill_info(tsg_solve_info* info, const StateHead& h, tsg_status st) {
  std::memset(info, 0, sizeof(*info));
  info->iters = h.iters;
  info->cycles = h.cycles;
  info->relres = h.relres;
  info->relres_est = h.est;
  info->status = st;
  info->truncated_cycles = h.truncated;
  info->pip_fallbacks = h.fallbacks;
  info->newton_from_cycle = h.newton_from;
  info->shifted_passes = h.shifted;
}

tsg_status head_status(const StateHead& h) {
  return h.status == 0 ? TSG_OK : (h.status == 1 ? TSG_NOT_CONVERGED : TSG_BREAKDOWN);
}

tsg_status run_solve(tsg_csr A, const tsg_solve_params* p, ReqCtx& q, char* dprog, hipStream_t s,
                     tsg_solve_info* info) {
  const int m = p->m;
  const int ortho = p->ortho;
  const int sstep = step_size(p);
  const bool f32 = p->precision == TSG_PREC_FP32_IR;
  Timer timer;
  const bool timing = p->timing != 0;
  const int64_t stride = p->timing > 1 ? p->timing : 1;  // time every stride-th cycle

  TRY(init_request(A, p, q, s));
  double bnorm = 0.0;
  HIP_TRY(hipMemcpyAsync(&bnorm, &q.c.st->bnorm, sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (bnorm == 0.0) {  // b = 0: x = 0 is the solution
    hipLaunchKernelGGL(zero_f64_kernel, dim3(cdiv(q.n, kRowBlock)), dim3(kRowBlock), 0, s, q.x, q.n);
    HIP_TRY(hipStreamSynchronize(s));
    if (info) {
      std::memset(info, 0, sizeof(*info));
      info->status = TSG_OK;
    }
    return TSG_OK;
  }

  // the launches of one restart cycle (identical in every cycle: what changes --
  // convergence, truncation, the fallback flag, the counters -- lives in the device state).
  // Two-stage: also a fast program without stage 1's gated fallback passes, run while no
  // cycle needed them; a cycle whose PIP pivot test fails there is run again in full (it
  // touched neither x nor the counters) and the full program runs from then on.
  Program P;
  P.f32 = f32;
  P.nreq = 1;
  Builder B{P, {&q}, 0};
  B.shifted = shifted_pass(p);
  TRY(build_cycle(B, m, sstep, ortho, p->s_hat));
  Program PF;
  PF.f32 = f32;
  PF.nreq = 1;
  const bool have_fast = ortho == TSG_ORTHO_TWO_STAGE;
  if (have_fast) {
    Builder BF{PF, {&q}, 0};
    BF.shifted = B.shifted;
    BF.fast = 1;
    TRY(build_cycle(BF, m, sstep, ortho, p->s_hat));
  }
  const size_t off_fast = align_up(P.blob.size());
  if (off_fast + PF.blob.size() > kProgramBytesPerRequest)
    return fail(TSG_ERR_UNSUPPORTED, "internal: launch image too large");
  HIP_TRY(hipMemcpyAsync(dprog, P.blob.data(), P.blob.size(), hipMemcpyHostToDevice, s));
  if (have_fast) HIP_TRY(hipMemcpyAsync(dprog + off_fast, PF.blob.data(), PF.blob.size(), hipMemcpyHostToDevice, s));
  char* dprog_fast = dprog + off_fast;

  StateHead* head = nullptr;
  HIP_TRY(hipHostMalloc((void**)&head, sizeof(StateHead), hipHostMallocDefault));
  hipEvent_t t0 = nullptr, t1 = nullptr;
  if (timing) {
    HIP_TRY(hipEventCreate(&t0));
    HIP_TRY(hipEventCreate(&t1));
    HIP_TRY(hipEventRecord(t0, s));
  }

  // graph mode: capture each program's cycle on a private stream, replay it on s.  A timed
  // cycle is launched directly (HIP events around each launch; same kernels and arguments).
  const bool use_graph = (p->flags & TSG_FLAG_EAGER) == 0;
  hipStream_t cs = nullptr;
  hipGraph_t graph[2] = {nullptr, nullptr};
  hipGraphExec_t exec[2] = {nullptr, nullptr};
  tsg_status result = TSG_OK;
  hipError_t e = hipSuccess;
  if (use_graph) {
    hipError_t ge = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    for (int g = 0; g < (have_fast ? 2 : 1) && ge == hipSuccess && result == TSG_OK; ++g) {
      ge = hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed);
      if (ge == hipSuccess) {
        tsg_status cst = g == 0 ? exec_program(P, dprog, cs, nullptr) : exec_program(PF, dprog_fast, cs, nullptr);
        ge = hipStreamEndCapture(cs, &graph[g]);
        if (cst != TSG_OK) result = cst;
      }
      if (ge == hipSuccess && result == TSG_OK) ge = hipGraphInstantiate(&exec[g], graph[g], nullptr, nullptr, 0);
    }
    if (ge != hipSuccess && result == TSG_OK)
      result = fail(TSG_ERR_HIP, "capture of a restart cycle failed: %s", hipGetErrorString(ge));
  }
  bool full = !have_fast;
  int64_t redone = 0;
  int64_t timed_cycles = 0;
  for (int64_t cyc = 0; result == TSG_OK; ++cyc) {
    timer.on = timing && cyc % stride == 0;
    for (int attempt = 0; attempt < 2; ++attempt) {
      const int g = full ? 0 : 1;
      if (use_graph && !timer.on) {
        e = hipGraphLaunch(exec[g], s);
        if (e != hipSuccess) {
          result = fail(TSG_ERR_HIP, "hipGraphLaunch: %s", hipGetErrorString(e));
          break;
        }
      } else {
        result = g == 0 ? exec_program(P, dprog, s, &timer) : exec_program(PF, dprog_fast, s, &timer);
        if (result != TSG_OK) break;
      }
      e = hipMemcpyAsync(head, &q.c.st->h, sizeof(StateHead), hipMemcpyDeviceToHost, s);
      if (e == hipSuccess) e = hipStreamSynchronize(s);
      if (e != hipSuccess) {
        result = fail(TSG_ERR_HIP, "cycle sync failed: %s", hipGetErrorString(e));
        break;
      }
      if (!head->redo) break;
      full = true;  // the cycle needs the fallback passes: run it again in full, and from now on
      redone += 1;
    }
    if (result != TSG_OK) break;
    timed_cycles += timer.on ? 1 : 0;
    if (timer.err != hipSuccess) {
      result = fail(TSG_ERR_HIP, "timing event: %s", hipGetErrorString(timer.err));
      break;
    }
    timer.harvest();
    if (head->done) break;
  }
  for (int g = 0; g < 2; ++g) {
    if (exec[g]) (void)hipGraphExecDestroy(exec[g]);
    if (graph[g]) (void)hipGraphDestroy(graph[g]);
  }
  if (cs) (void)hipStreamDestroy(cs);
  double ms_total = 0.0;
  if (timing && result == TSG_OK) {
    (void)hipEventRecord(t1, s);
    (void)hipEventSynchronize(t1);
    float tot = 0.f;
    (void)hipEventElapsedTime(&tot, t0, t1);
    ms_total = tot;
  }
  if (t0) (void)hipEventDestroy(t0);
  if (t1) (void)hipEventDestroy(t1);
  StateHead h = *head;
  (void)hipHostFree(head);
  if (result != TSG_OK) return result;
  tsg_status st = head_status(h);
  if (info) {
    fill_info(info, h, st);
    info->redone_cycles = redone;
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
  ReqCtx q;
  char* dprog = (char*)workspace + request_bytes(A->n, A->nnz, p);
  if (p->precond != TSG_PRECOND_MCGS) {
    q.b = b;
    q.x = x;
    carve_request((char*)workspace, A, p, q);
    return run_solve(A, p, q, dprog, (hipStream_t)stream, info);
  }
  // right preconditioning: the solve runs on the color-ordered system P A P^T with P b and
  // P x; x = P^T x_p afterwards (norms and the residual are permutation-invariant)
  if (!A->pa) return fail(TSG_ERR_INVALID_ARG, "precond = MCGS needs tsg_csr_precond on the operator first");
  hipStream_t s = (hipStream_t)stream;
  carve_request((char*)workspace, A->pa, p, q);
  const int nb = (int)cdiv(A->n, 256);
  hipLaunchKernelGGL(gather_f64_kernel, dim3(nb), dim3(256), 0, s, b, A->perm, q.bp, A->n);
  hipLaunchKernelGGL(gather_f64_kernel, dim3(nb), dim3(256), 0, s, (const double*)x, A->perm, q.xp, A->n);
  HIP_LAUNCH_CHECK();
  q.b = q.bp;
  q.x = q.xp;
  const tsg_status st = run_solve(A->pa, p, q, dprog, s, info);
  if (st < 0) return st;  // errors leave x untouched
  hipLaunchKernelGGL(scatter_f64_kernel, dim3(nb), dim3(256), 0, s, (const double*)q.xp, A->perm, x, A->n);
  HIP_LAUNCH_CHECK();
  HIP_TRY(hipStreamSynchronize(s));
  return st;
}

size_t tsg_orthogonalize_workspace_bytes(int64_t n, int32_t k, int32_t s) {
  if (n < 1 || k < 1 || k > kMaxCols || s < 1 || s > kMaxS) return 0;
  size_t cb = common_bytes(n);
  if (cb == (size_t)-1) return 0;
  return cb + kProgramBytesPerRequest + kAlign;
}

namespace {

// Q = Qhat Rinv in place, Rinv = the upper-triangular inverse in sm->Wk (ld kLd).
tsg_status launch_apply_rinv(double* X, int64_t ldx, int64_t n, int k, const SmallState* sm, hipStream_t st) {
  const double* Rinv = sm->Wk;
  const int64_t rpb = rinv_rows_per_block(n);
  const dim3 grid((unsigned)cdiv(n, rpb)), block(kRinvThreads);
  const bool o32 = rinv_off32(ldx);
#define TSG_RINV(NCT)                                                                                 \
  do {                                                                                                \
    if (o32) hipLaunchKernelGGL((apply_rinv_kernel<NCT, true>), grid, block, 0, st, X, ldx, n, k, Rinv, rpb, sm); \
    else hipLaunchKernelGGL((apply_rinv_kernel<NCT, false>), grid, block, 0, st, X, ldx, n, k, Rinv, rpb, sm);    \
  } while (0)
  switch ((k + 15) / 16) {
    case 1: TSG_RINV(1); break;
    case 2: TSG_RINV(2); break;
    case 3: TSG_RINV(3); break;
    default: TSG_RINV(4); break;
  }
#undef TSG_RINV
  HIP_LAUNCH_CHECK();
  return TSG_OK;
}

// Argument checks shared by the stand-alone orthogonalization entry points (host only).
tsg_status orthogonalize_check(int64_t n, int32_t k, const double* X, int64_t ldx, const double* R, int32_t ldr,
                               int32_t s, int32_t s_hat, int32_t algo) {
  if (!X || !R) return fail(TSG_ERR_INVALID_ARG, "NULL argument");
  if (n < 1 || k < 1 || k > kMaxCols || k > n)
    return fail(TSG_ERR_INVALID_ARG, "need 1 <= k <= min(n, 64): n=%lld k=%d", (long long)n, k);
  if (ldx < n || ldr < k) return fail(TSG_ERR_INVALID_ARG, "leading dimension too small");
  if (s < 1 || s > kMaxS) return fail(TSG_ERR_INVALID_ARG, "s=%d outside [1, 16]", s);
  if (algo != TSG_ORTHO_TWO_STAGE && algo != TSG_ORTHO_BCGS_PIP2 && algo != TSG_ORTHO_BCGS2_CHOLQR2)
    return fail(TSG_ERR_INVALID_ARG, "bad algo %d", algo);
  if (s_hat != 0 && s_hat < k - 1) {
    if (algo != TSG_ORTHO_TWO_STAGE) return fail(TSG_ERR_INVALID_ARG, "s_hat=%d is a two-stage parameter", s_hat);
    if (s_hat < s || s_hat % s != 0)
      return fail(TSG_ERR_INVALID_ARG, "s_hat=%d must be a multiple of s=%d (or 0, or >= k-1)", s_hat, s);
  }
  return TSG_OK;
}

// The stand-alone orthogonalization on a checked workspace `ws` of at least
// tsg_orthogonalize_workspace_bytes(n, k, s) bytes (256-byte aligned): every buffer of the
// call (small state, reduction partials, launch image) is carved from it, and everything
// read before it is written is initialized here.
// The launch program of a stand-alone orthogonalization (Sec. V, Fig. 5; Fig. 4b; Fig. 2b)
// of the n x k block of request q; n_main: the phases before the optional orthogonality check.
tsg_status build_ortho_program(Program& P, size_t& n_main, ReqCtx& q, int32_t k, int32_t s, int32_t s_hat,
                               int32_t algo, bool orth_err) {
  const bool two = algo == TSG_ORTHO_TWO_STAGE;
  P.nreq = 1;
  Builder B{P, {&q}, 1};
  // column 1 alone
  TRY(B.step(gram_step(0, 0, 1, 0, TAIL_SA_NORM, -1, 0)));
  // two-stage with panels: G2(0,0) comes with the first panel's reduction when column 0 and
  // the first panel fit one lean reduction
  const bool g00 = two && (k == 1 || 1 + std::min(s, k - 1) > kMaxGramNz);
  TRY(B.step(upd_step(g00 ? PK_FUSED : PK_UPDATE, 0, 0, 1, PF_HAS_T | PF_STORE | (g00 ? PF_GRAM_W : 0),
                      g00 ? TAIL_NORM0 : TAIL_NONE, -1, 0)));
  const bool lean2 = 2 * s <= kMaxGramNz;
  // big panels of the two-stage scheme (Sec. V, Fig. 5): the first holds column 0 and s_hat
  // columns, every later one s_hat columns (the last may be short); s_hat = 0 or >= k - 1:
  // one big panel, whose stage 2 is the CholQR of all k columns below
  const bool big = two && s_hat > 0 && s_hat < k - 1;
  int b0 = 0, b1 = big ? 1 + s_hat : k;
  int panel = 0;
  for (int c0 = 1; c0 < k; c0 += s, ++panel) {
    const int sw = std::min(s, k - c0);
    const bool last = c0 + sw >= k;
    const bool ends_big = big && c0 + sw == b1;
    // previous columns reduced along: column 0 for the first panel, none for the first panel
    // of a later big panel (the panel before formed its own block column), else the previous
    // panel (panels before the last have width s)
    const int nprev = !two ? 0 : (c0 == 1 ? (g00 ? 0 : 1) : ((big && c0 == b0) || !lean2 ? 0 : s));
    // the panel index gates each stage 1 sequence on its own fallback flag
    TRY(panel_sequence(B, algo, c0, sw, nprev, last || ends_big || !lean2, big ? panel : 0, 0));
    if (ends_big) {
      // stage 2 of the big panel: BCGS-PIP against the final columns before it, the R factor
      // updated, and Y(:, b0:b1) <- Y(:, :b1) Bs in 16-column chunks (explicit Q)
      TRY(B.big_stage2(b0, b1, big ? panel : 0));
      b0 = b1;
      b1 = std::min(b0 + s_hat, k);
    }
  }
  n_main = P.phases.size();
  if (orth_err) {  // the Gram of the result, 16 columns at a time, into st->Wk
    for (int c0 = 0; c0 < k; c0 += kMaxS) {
      const int sw = std::min(kMaxS, k - c0);
      TRY(B.step(gram_step(c0, c0, sw, 0, TAIL_GRAM_OUT, 0, 0, 0)));
    }
  }
  return TSG_OK;
}

// Programs of recent stand-alone orthogonalizations (per host thread): a call with the same
// shapes, scheme and pointers -- the block and the workspace the program's launch tables
// point into -- reuses the host image instead of building it again; the image is still
// copied to the workspace on every call.
struct OrthoKey {
  int64_t n, ldx;
  int32_t k, s, s_hat, algo;
  const void* X;
  const void* ws;
  bool err;
  bool operator==(const OrthoKey& o) const {
    return n == o.n && ldx == o.ldx && k == o.k && s == o.s && s_hat == o.s_hat && algo == o.algo && X == o.X &&
           ws == o.ws && err == o.err;
  }
};
struct OrthoProgram {
  OrthoKey key{};
  Program P;
  size_t n_main = 0;
};
constexpr size_t kOrthoPrograms = 4;
thread_local std::vector<OrthoProgram> t_ortho_programs;

tsg_status orthogonalize_ws(int64_t n, int32_t k, double* X, int64_t ldx, double* R, int32_t ldr, int32_t s,
                            int32_t s_hat, int32_t algo, char* ws, hipStream_t st, double* orth_err) {
  Carve cv{ws};
  Common c = carve_common(cv, n);
  char* dprog = cv.take<char>(kProgramBytesPerRequest);
  const bool two = algo == TSG_ORTHO_TWO_STAGE;

  // the state's head and parameters (the same for every call: formed once per host thread)
  thread_local std::vector<char> init_image;
  if (init_image.empty()) {
    SmallState* hs = new (std::nothrow) SmallState();
    if (!hs) return fail(TSG_ERR_INVALID_ARG, "out of host memory");
    std::memset(hs, 0, sizeof(SmallState));
    hs->h.stop_panel = 1 << 30;
    hs->pivot_tol = 0.0;  // stand-alone: fail only when a Gram is not positive definite
    hs->pip_tol = 0.0;
    hs->fail_col = -1;
    init_image.assign(reinterpret_cast<const char*>(hs), reinterpret_cast<const char*>(hs) + offsetof(SmallState, Hh));
    delete hs;
  }
  HIP_TRY(hipMemcpyAsync(c.st, init_image.data(), init_image.size(), hipMemcpyHostToDevice, st));
  hipLaunchKernelGGL(zero_f64_kernel, dim3(cdiv(kLd * kLd, 256)), dim3(256), 0, st, c.st->Hh,
                     (int64_t)kLd * kLd);
  hipLaunchKernelGGL(zero_f64_kernel, dim3(cdiv(kLd * kLd, 256)), dim3(256), 0, st, c.st->G2,
                     (int64_t)kLd * kLd);
  HIP_LAUNCH_CHECK();
  ReqCtx q;
  q.V = X;
  q.ld = ldx;
  q.n = n;
  q.c = c;
  const bool big = two && s_hat > 0 && s_hat < k - 1;
  // the launch program: reused from an earlier call with the same shapes, scheme and pointers
  const OrthoKey key{n, ldx, k, s, s_hat, algo, X, ws, orth_err != nullptr};
  const OrthoProgram* op = nullptr;
  for (const OrthoProgram& ent : t_ortho_programs)
    if (ent.key == key) op = &ent;
  if (!op) {
    OrthoProgram built;
    built.key = key;
    TRY(build_ortho_program(built.P, built.n_main, q, k, s, s_hat, algo, orth_err != nullptr));
    if (t_ortho_programs.size() >= kOrthoPrograms) t_ortho_programs.erase(t_ortho_programs.begin());
    t_ortho_programs.push_back(std::move(built));
    op = &t_ortho_programs.back();
  }
  const Program& P = op->P;
  const size_t n_main = op->n_main;
  if (P.blob.size() > kProgramBytesPerRequest) return fail(TSG_ERR_UNSUPPORTED, "internal: launch image too large");
  HIP_TRY(hipMemcpyAsync(dprog, P.blob.data(), P.blob.size(), hipMemcpyHostToDevice, st));
  TRY(exec_program(P, dprog, st, nullptr, 0, n_main));
  if (big) {  // every big panel's Q is final: the R factor is the assembly in st->Hh
    hipLaunchKernelGGL(copy_r_kernel, dim3(1), dim3(256), 0, st, c.st, 0, k, R, ldr);
  } else if (two) {
    // stage 2: one CholQR over all k columns, then Q = Qhat R2^{-1}
    hipLaunchKernelGGL(sa_stage2_kernel, dim3(1), dim3(256), 0, st, c.st, k);
    HIP_LAUNCH_CHECK();
    // returns at entry after a breakdown (the caller gets TSG_BREAKDOWN)
    TRY(launch_apply_rinv(X, ldx, n, k, c.st, st));
    hipLaunchKernelGGL(copy_r_kernel, dim3(1), dim3(256), 0, st, c.st, 1, k, R, ldr);
  } else {
    hipLaunchKernelGGL(copy_r_kernel, dim3(1), dim3(256), 0, st, c.st, 0, k, R, ldr);
  }
  HIP_LAUNCH_CHECK();
  if (orth_err) {
    TRY(exec_program(P, dprog, st, nullptr, n_main));
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

}  // namespace

tsg_status tsg_orthogonalize(int64_t n, int32_t k, double* X, int64_t ldx, double* R, int32_t ldr,
                             int32_t s, int32_t s_hat, int32_t algo, void* workspace, size_t ws_bytes,
                             void* stream, double* orth_err) {
  if (!workspace) return fail(TSG_ERR_INVALID_ARG, "NULL argument");
  TRY(orthogonalize_check(n, k, X, ldx, R, ldr, s, s_hat, algo));
  if (reinterpret_cast<uintptr_t>(workspace) % kAlign != 0)
    return fail(TSG_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  size_t need = tsg_orthogonalize_workspace_bytes(n, k, s);
  if (need == 0) return fail(TSG_ERR_INVALID_ARG, "problem too large for the reduction buffers");
  if (ws_bytes < need) return fail(TSG_ERR_WORKSPACE, "workspace %zu < required %zu", ws_bytes, need);
  return orthogonalize_ws(n, k, X, ldx, R, ldr, s, s_hat, algo, (char*)workspace, (hipStream_t)stream, orth_err);
}

// ------------------------------------------------------------------ one stage-1 panel
size_t tsg_block_pip_workspace_bytes(int64_t n, int32_t k, int32_t s) {
  if (k < 0 || s < 1 || s > kMaxS || k + s > kMaxCols) return 0;
  return tsg_orthogonalize_workspace_bytes(n, k + s, s);
}

tsg_status tsg_block_pip(int64_t n, int32_t k, int32_t s, double* V, int64_t ldv, double pip_tol, double pivot_tol,
                         int32_t chain, double* P, int32_t ldp, double* R, int32_t ldr, int32_t* out, void* workspace,
                         size_t ws_bytes, void* stream) {
  if (!V || !R || !workspace || (k > 0 && !P)) return fail(TSG_ERR_INVALID_ARG, "NULL argument");
  if (k < 0 || s < 1 || s > kMaxS || k + s > kMaxCols || k + s > n)
    return fail(TSG_ERR_INVALID_ARG, "need 0 <= k, 1 <= s <= 16, k + s <= min(n, 64): n=%lld k=%d s=%d",
                (long long)n, k, s);
  if (ldv < n || ldr < s || (k > 0 && ldp < k)) return fail(TSG_ERR_INVALID_ARG, "leading dimension too small");
  if (chain < 0 || chain > 2) return fail(TSG_ERR_INVALID_ARG, "chain=%d outside [0, 2]", chain);
  if (!(pip_tol >= 0.0 && pip_tol < 1.0) || !(pivot_tol >= 0.0 && pivot_tol < 1.0))
    return fail(TSG_ERR_INVALID_ARG, "pivot thresholds must lie in [0, 1)");
  if (chain >= 1 && !(pivot_tol > 0.0))
    return fail(TSG_ERR_INVALID_ARG, "the explicit and shifted passes need pivot_tol > 0");
  if (reinterpret_cast<uintptr_t>(workspace) % kAlign != 0)
    return fail(TSG_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  const size_t need = tsg_block_pip_workspace_bytes(n, k, s);
  if (need == 0) return fail(TSG_ERR_INVALID_ARG, "problem too large for the reduction buffers");
  if (ws_bytes < need) return fail(TSG_ERR_WORKSPACE, "workspace %zu < required %zu", ws_bytes, need);
  hipStream_t st = (hipStream_t)stream;
  Carve cv{(char*)workspace};
  Common c = carve_common(cv, n);
  char* dprog = cv.take<char>(kProgramBytesPerRequest);
  SmallState* hs = new (std::nothrow) SmallState();
  if (!hs) return fail(TSG_ERR_INVALID_ARG, "out of host memory");
  std::memset(hs, 0, sizeof(SmallState));
  hs->h.stop_panel = 1 << 30;
  hs->pivot_tol = pivot_tol;
  hs->pip_tol = pip_tol;
  hs->fail_col = -1;
  hipError_t e = hipMemcpyAsync(c.st, hs, offsetof(SmallState, Hh), hipMemcpyHostToDevice, st);
  delete hs;
  HIP_TRY(e);
  hipLaunchKernelGGL(zero_f64_kernel, dim3(cdiv(kLd * kLd, 256)), dim3(256), 0, st, c.st->Hh, (int64_t)kLd * kLd);
  HIP_LAUNCH_CHECK();
  ReqCtx q;
  q.V = V;
  q.ld = ldv;
  q.n = n;
  q.c = c;
  Program Pg;
  Pg.nreq = 1;
  // chain 0: PIP alone (a failed pivot is a breakdown); 1: + the explicit pass, gated on
  // the PIP pivot test; 2: + the shifted Cholesky QR pass, gated on the explicit pass's test
  Builder B{Pg, {&q}, chain > 0 ? 2 : 1};
  B.shifted = chain >= 2 ? 1 : 0;
  for (int pass = 0; pass <= chain; ++pass) {
    const int gate = pass + 1;
    TRY(B.step(gram_step(k, k, s, 0, pass == 0 ? TAIL_PIP : (pass == 1 ? TAIL_PIP_FB : TAIL_PIP_FB2), 0, 0, gate)));
    Step u = upd_step(PK_UPDATE, k, k, s, PF_HAS_P | PF_HAS_T | PF_STORE, TAIL_NONE, 0, 0);
    u.gate = gate;
    TRY(B.step(u));
  }
  if (Pg.blob.size() > kProgramBytesPerRequest) return fail(TSG_ERR_UNSUPPORTED, "internal: launch image too large");
  HIP_TRY(hipMemcpyAsync(dprog, Pg.blob.data(), Pg.blob.size(), hipMemcpyHostToDevice, st));
  TRY(exec_program(Pg, dprog, st, nullptr));
  hipLaunchKernelGGL(copy_panel_kernel, dim3(1), dim3(256), 0, st, (const SmallState*)c.st, k, s, P, ldp, R, ldr);
  HIP_LAUNCH_CHECK();
  StateHead h{};
  int32_t fcol = -1;
  HIP_TRY(hipMemcpyAsync(&h, &c.st->h, sizeof(StateHead), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(&fcol, &c.st->fail_col, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (out) {
    out[0] = h.fallbacks + h.shifted;
    out[1] = h.status == 2 ? fcol : -1;
  }
  if (h.status == 2) return fail(TSG_BREAKDOWN, "pivot %d of the panel failed after %d fallback pass(es)", fcol,
                                 h.fallbacks + h.shifted);
  return TSG_OK;
}

// ------------------------------------------------------------------ no-allocation entry
// tsg_orthogonalize_noalloc runs tsg_orthogonalize with its workspace in `scratch`, a
// file-scope device array of kNoAllocScratchBytes that every GPU the library runs on holds
// for the life of the process.  In host code the array's name only stands in for the
// symbol: its device address on the current device comes from hipGetSymbolAddress, taken
// once per device (with that device current) on the first call there, and only that
// address is ever passed to kernels or copies.
namespace {

constexpr size_t kNoAllocScratchBytes = size_t(12) << 20;
// the workspace of tsg_orthogonalize is the same ~9.3 MB for every n up to this many rows
// (the reduction partials outgrow their fixed size beyond it)
constexpr int64_t kNoAllocMaxRows = (int64_t)kMaxReduceBlocks * kMaxCols * kMaxNz * kRowBlock;
static __device__ __align__(256) char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_addr[kMaxDevices] = {};

tsg_status scratch_address(void** out) {
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(TSG_ERR_UNSUPPORTED, "device index %d out of range", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_addr[dev]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(TSG_ERR_HIP, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
    g_scratch_addr[dev] = p;
  }
  *out = g_scratch_addr[dev];
  return TSG_OK;
}

}  // namespace

size_t tsg_orthogonalize_noalloc_max_bytes(void) { return kNoAllocScratchBytes; }

tsg_status tsg_orthogonalize_noalloc(int64_t n, int32_t k, double* X, int64_t ldx, double* R, int32_t ldr,
                                     int32_t s, int32_t s_hat, int32_t algo, void* stream, double* orth_err) {
  TRY(orthogonalize_check(n, k, X, ldx, R, ldr, s, s_hat, algo));
  const size_t need = tsg_orthogonalize_workspace_bytes(n, k, s);
  if (n > kNoAllocMaxRows || need == 0 || need > kNoAllocScratchBytes)
    return fail(TSG_ERR_INVALID_ARG,
                "n=%lld k=%d s=%d needs %zu scratch bytes; the no-allocation entry point holds %zu "
                "(n <= %lld rows)",
                (long long)n, k, s, need, kNoAllocScratchBytes, (long long)kNoAllocMaxRows);
  void* ws = nullptr;
  TRY(scratch_address(&ws));
  return orthogonalize_ws(n, k, X, ldx, R, ldr, s, s_hat, algo, static_cast<char*>(ws), (hipStream_t)stream, orth_err);
}

// =================================================================== solve server
// Continuous batching of many solves that share the solver parameters.  Requests queue
// on the host; at every restart-cycle boundary the server admits queued requests in
// arrival order while their buffers fit its arena (and a slot is free), then runs ONE
// restart cycle of every active request: each phase of the cycle is one batched launch
// over all active requests, so small and large solves share every kernel.  Finished
// requests (converged, out of iterations, or broken down) leave at the cycle boundary and
// free their memory for the queue.  A request computes exactly what tsg_solve computes for
// it: its launches see their own block indices and buffers whatever else is batched.

namespace {

__global__ void gather_heads_kernel(SmallState* const* sts, StateHead* out, int nreq) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < nreq) out[r] = sts[r]->h;
}

// First-fit allocator of arena offsets (host bookkeeping only).
struct Arena {
  std::vector<std::pair<size_t, size_t>> free_;  // (offset, size), sorted by offset
  void init(size_t off, size_t bytes) { free_.assign(1, {off, bytes}); }
  bool alloc(size_t bytes, size_t* off) {
    bytes = align_up(bytes);
    for (size_t i = 0; i < free_.size(); ++i) {
      if (free_[i].second >= bytes) {
        *off = free_[i].first;
        free_[i].first += bytes;
        free_[i].second -= bytes;
        if (free_[i].second == 0) free_.erase(free_.begin() + i);
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = align_up(bytes);
    auto it = std::lower_bound(free_.begin(), free_.end(), std::make_pair(off, (size_t)0));
    it = free_.insert(it, {off, bytes});
    // merge with the next and the previous block
    if (it + 1 != free_.end() && it->first + it->second == (it + 1)->first) {
      it->second += (it + 1)->second;
      free_.erase(it + 1);
    }
    if (it != free_.begin() && (it - 1)->first + (it - 1)->second == it->first) {
      (it - 1)->second += it->second;
      free_.erase(it);
    }
  }
};

struct ServeReq {
  int64_t tag;
  tsg_csr A;
  ReqCtx q;
  size_t off = 0, bytes = 0;
};

}  // namespace

struct tsg_server_s {
  tsg_solve_params p;
  char* arena;
  size_t arena_bytes;
  int max_active;
  hipStream_t s;
  char* dimage;              // launch image of the current batch
  size_t image_bytes;
  StateHead* dheads;         // gathered heads (device)
  StateHead* hheads;         // pinned copy
  Arena mem;
  std::vector<ServeReq*> queue;   // FIFO
  std::vector<ServeReq*> active;
  std::vector<std::pair<int64_t, tsg_solve_info>> done;
  Program prog;
  size_t sts_off = 0;        // offset of the SmallState* table in the image
  bool dirty = true;         // membership changed: rebuild the launch image
};

size_t tsg_server_request_bytes(int64_t n, int64_t nnz, const tsg_solve_params* p) {
  if (n < 1 || nnz < 0 || !p || validate_params(n, p) != TSG_OK) return 0;
  return align_up(request_bytes(n, nnz, p));
}

tsg_status tsg_server_create(const tsg_solve_params* p, void* arena, size_t arena_bytes, int32_t max_active,
                             void* stream, tsg_server* out) {
  if (!p || !arena || !out) return fail(TSG_ERR_INVALID_ARG, "NULL argument");
  TRY(validate_params(1 << 30, p));
  if (max_active < 1 || max_active > 4096) return fail(TSG_ERR_INVALID_ARG, "max_active=%d outside [1, 4096]", max_active);
  if (p->timing != 0) return fail(TSG_ERR_UNSUPPORTED, "per-kernel timing is not available in the server");
  if (p->precond != TSG_PRECOND_NONE) return fail(TSG_ERR_UNSUPPORTED, "the server runs unpreconditioned solves");
  if (reinterpret_cast<uintptr_t>(arena) % kAlign != 0) return fail(TSG_ERR_WORKSPACE, "arena must be 256-byte aligned");
  const size_t image = align_up((size_t)max_active * kProgramBytesPerRequest);
  const size_t heads = align_up((size_t)max_active * sizeof(StateHead));
  if (arena_bytes < image + heads + (1 << 20))
    return fail(TSG_ERR_WORKSPACE, "arena %zu too small for %d slots", arena_bytes, max_active);
  tsg_server_s* S = new (std::nothrow) tsg_server_s();
  if (!S) return fail(TSG_ERR_INVALID_ARG, "out of host memory");
  S->p = *p;
  S->p.newton_shifts = nullptr;
  if (p->basis == TSG_BASIS_NEWTON) {
    delete S;
    return fail(TSG_ERR_UNSUPPORTED, "the server takes monomial or shifted bases");
  }
  S->arena = (char*)arena;
  S->arena_bytes = arena_bytes;
  S->max_active = max_active;
  S->s = (hipStream_t)stream;
  S->dimage = S->arena;
  S->image_bytes = image;
  S->dheads = reinterpret_cast<StateHead*>(S->arena + image);
  S->mem.init(image + heads, arena_bytes - image - heads);
  if (hipHostMalloc((void**)&S->hheads, heads, hipHostMallocDefault) != hipSuccess) {
    delete S;
    return fail(TSG_ERR_HIP, "hipHostMalloc of the status buffer failed");
  }
  *out = S;
  return TSG_OK;
}

tsg_status tsg_server_destroy(tsg_server S) {
  if (!S) return TSG_OK;
  (void)hipStreamSynchronize(S->s);
  (void)hipHostFree(S->hheads);
  for (auto* r : S->queue) delete r;
  for (auto* r : S->active) delete r;
  delete S;
  return TSG_OK;
}

tsg_status tsg_server_submit(tsg_server S, tsg_csr A, const double* b, double* x, int64_t tag) {
  if (!S || !A || !b || !x) return fail(TSG_ERR_INVALID_ARG, "NULL argument");
  TRY(validate_params(A->n, &S->p));
  const size_t bytes = align_up(request_bytes(A->n, A->nnz, &S->p));
  if (bytes > S->arena_bytes - S->image_bytes)
    return fail(TSG_ERR_INVALID_ARG, "request of %zu bytes can never fit the arena", bytes);
  ServeReq* r = new (std::nothrow) ServeReq();
  if (!r) return fail(TSG_ERR_INVALID_ARG, "out of host memory");
  r->tag = tag;
  r->A = A;
  r->bytes = bytes;
  r->q.b = b;
  r->q.x = x;
  S->queue.push_back(r);
  return TSG_OK;
}

namespace {

void retire(tsg_server S, ServeReq* r, const StateHead& h) {
  tsg_solve_info info;
  fill_info(&info, h, head_status(h));
  S->done.push_back({r->tag, info});
  S->mem.release(r->off, r->bytes);
  delete r;
}

}  // namespace

tsg_status tsg_server_step(tsg_server S, int32_t* n_active, int32_t* n_queued) {
  if (!S) return fail(TSG_ERR_INVALID_ARG, "NULL server");
  hipStream_t s = S->s;
  // ---- admission at the cycle boundary: arrival order, while memory and slots allow
  std::vector<ServeReq*> joining;
  size_t qi = 0;
  while (qi < S->queue.size() && (int)(S->active.size() + joining.size()) < S->max_active) {
    ServeReq* r = S->queue[qi];
    size_t off = 0;
    if (!S->mem.alloc(r->bytes, &off)) break;  // head of the line waits for memory
    r->off = off;
    carve_request(S->arena + off, r->A, &S->p, r->q);
    tsg_status st = init_request(r->A, &S->p, r->q, s);
    if (st != TSG_OK) {
      // nobody joins at this boundary: the requests stay queued and free their arena blocks
      S->mem.release(off, r->bytes);
      for (ServeReq* j : joining) S->mem.release(j->off, j->bytes);
      (void)hipStreamSynchronize(s);
      return st;
    }
    joining.push_back(r);
    ++qi;
  }
  S->queue.erase(S->queue.begin(), S->queue.begin() + qi);
  if (!joining.empty()) {
    // b = 0 solves finish at once (x = 0); read every new ||b|| with one synchronization
    std::vector<double> bn(joining.size());
    for (size_t i = 0; i < joining.size(); ++i)
      HIP_TRY(hipMemcpyAsync(&bn[i], &joining[i]->q.c.st->bnorm, sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    for (size_t i = 0; i < joining.size(); ++i) {
      ServeReq* r = joining[i];
      if (bn[i] == 0.0) {
        hipLaunchKernelGGL(zero_f64_kernel, dim3(cdiv(r->q.n, kRowBlock)), dim3(kRowBlock), 0, s, r->q.x, r->q.n);
        HIP_LAUNCH_CHECK();
        StateHead h{};
        h.done = 1;
        retire(S, r, h);
      } else {
        S->active.push_back(r);
        S->dirty = true;
      }
    }
  }
  if (!S->active.empty()) {
    // ---- the launch image of the current batch
    if (S->dirty) {
      S->prog = Program();
      S->prog.f32 = S->p.precision == TSG_PREC_FP32_IR;
      S->prog.nreq = (int)S->active.size();
      Builder B{S->prog, {}, 0};
      B.shifted = shifted_pass(&S->p);
      for (auto* r : S->active) B.R.push_back(&r->q);
      TRY(build_cycle(B, S->p.m, step_size(&S->p), S->p.ortho, S->p.s_hat));
      std::vector<SmallState*> sts;
      for (auto* r : S->active) sts.push_back(r->q.c.st);
      S->sts_off = S->prog.put(sts.data(), sizeof(SmallState*) * sts.size());
      if (S->prog.blob.size() > S->image_bytes) return fail(TSG_ERR_UNSUPPORTED, "internal: launch image too large");
      HIP_TRY(hipMemcpyAsync(S->dimage, S->prog.blob.data(), S->prog.blob.size(), hipMemcpyHostToDevice, s));
      S->dirty = false;
    }
    // ---- one restart cycle of every active request, then their status heads
    TRY(exec_program(S->prog, S->dimage, s, nullptr));
    const int na = (int)S->active.size();
    hipLaunchKernelGGL(gather_heads_kernel, dim3(cdiv(na, 256)), dim3(256), 0, s,
                       reinterpret_cast<SmallState* const*>(S->dimage + S->sts_off), S->dheads, na);
    HIP_LAUNCH_CHECK();
    HIP_TRY(hipMemcpyAsync(S->hheads, S->dheads, sizeof(StateHead) * na, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    std::vector<ServeReq*> keep;
    for (int i = 0; i < na; ++i) {
      if (S->hheads[i].done) {
        retire(S, S->active[i], S->hheads[i]);
        S->dirty = true;
      } else {
        keep.push_back(S->active[i]);
      }
    }
    S->active.swap(keep);
  }
  if (n_active) *n_active = (int32_t)S->active.size();
  if (n_queued) *n_queued = (int32_t)S->queue.size();
  return TSG_OK;
}

int32_t tsg_server_poll(tsg_server S, int64_t* tags, tsg_solve_info* infos, int32_t max) {
  if (!S || max <= 0) return 0;
  const int32_t k = (int32_t)std::min<size_t>((size_t)max, S->done.size());
  for (int32_t i = 0; i < k; ++i) {
    if (tags) tags[i] = S->done[i].first;
    if (infos) infos[i] = S->done[i].second;
  }
  S->done.erase(S->done.begin(), S->done.begin() + k);
  return k;
}
