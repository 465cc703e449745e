// ocsc.hip -- host runtime and C ABI of libocsc (see include/ocsc.h).
//
// One context owns the learner state of Algorithm 3 on one device and a HIP
// stream; every call validates its arguments on the host, then enqueues the
// kernels of kernels.hpp on that stream.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <type_traits>
#include <utility>
#include <vector>

#include "../../include/ocsc.h"
#include "bigplane.hpp"
#include "chol.hpp"
#include "diag.hpp"
#include "fold.hpp"
#include "group.hpp"
#include "kernels.hpp"

using namespace ocsc;

// Scratch of ocsc_objective_noalloc: part of the code object's static data,
// so that the call allocates nothing.  Each device that loads the library
// holds its own copy until the process ends.  Host code never passes the
// array's name to a kernel (on the host it is only a stand-in for the
// symbol); it uses the device address that ocsc_init looks up once per
// device with that device current.
static __device__ __align__(256) unsigned char scratch[OCSC_NOALLOC_SCRATCH_BYTES];

namespace {

thread_local std::string g_init_error;

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};

struct ProfEntry {
  int cls;
  hipEvent_t a, b;
};

}  // namespace

struct ocsc_ctx {
  // problem
  int K = 0, Mh = 0, Mw = 0, Ph = 0, Pw = 0, Wc = 0, Pf = 0, P = 0;
  double lam = 0, rho = 0, rho_d = 0;
  int Jz = 10, Jd = 10, maxB = 1, prec = OCSC_FP64;
  size_t sr = 8;   // bytes per real
  int nvb = 0;     // V-step column blocks
  int fpb = 1;     // frequencies solved side by side by one D-step workgroup
  int fs = 0;      // reals per frequency of C (K rows of pitch K+1, 16-byte multiple)
  int sweep_wgs = 0, slots_per_wg = 0, fold_wgs = 0;   // plain-sweep grid and run length; fold-sweep grid
  size_t sweep_smem = 0, plain_smem = 0, vapply_smem = 0;   // LDS of fold sweeps and of plain sweeps
  bool vstep_fused = false;   // one workgroup per filter (filters up to 16 x 16)
  bool big = false;           // two-pass plane transforms (a side above 128)
  bool keep_hist = false;     // OCSC_FLAG_KEEP_HISTORY (implied by OCSC_FLAG_CHOLESKY)
  bool chol = false;          // OCSC_FLAG_CHOLESKY: matrix-core history, C from an FP64 Cholesky
  bool dstream = false;       // K > 128 (Cholesky form): C_p streamed through LDS by k_dstep_stream
  int chol_chunk = 0;         // K > 128: frequencies per Schur-complement chunk
  void* Wchol = nullptr;      // K > 128: five 128 x 128 FP64 blocks per frequency of a chunk
  bool warm = false;          // OCSC_FLAG_WARM_START
  bool refine = false;        // OCSC_FLAG_REFINE: one refinement step after each D-step (precision form)
  ocsc_tuning tune{};         // launch shapes of the code update (ocsc_set_tuning / ocsc_autotune)
  // runtime
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  // device state (typed by prec)
  void *xh = nullptr, *Dh = nullptr, *gam = nullptr, *S = nullptr, *Zh = nullptr,
       *W = nullptr, *G = nullptr, *Cm = nullptr, *d = nullptr, *Th = nullptr, *rhs = nullptr,
       *V = nullptr, *apart = nullptr, *twH = nullptr, *twW = nullptr, *xh_obj = nullptr;
  double *obj_part = nullptr, *obj_out = nullptr;
  int obj_nr = 0, obj_nl = 0;
  // kept history and diagnostics: H (layout of C), codes when the caller keeps
  // none, per-sample partial sums of the pending codes, running sums, the
  // spectrum of given filters, exported filters, reduction partials, results
  void *Hm = nullptr, *Ubuf = nullptr, *Dv = nullptr, *Dexp = nullptr;
  void* Yb = nullptr;   // inverse column pass of the code spectra (two-pass grids)
  void* Zt = nullptr;   // last code spectra frequency-major [Pf][max_batch][K] (Cholesky form, max_batch > 1)
  double *pend = nullptr, *hacc = nullptr, *dpart = nullptr, *dres = nullptr;
  void* scratch = nullptr;   // device address of this device's static scratch (ocsc_objective_noalloc)
  int* brk = nullptr;        // Cholesky form: set by the factorisation when a pivot is not positive
  // host-side bookkeeping
  int64_t t = 0;
  int pending_B = 0;    // coded samples not yet accumulated
  int fold_B = 0;       // accumulated samples whose fold is still deferred
  unsigned sweep_count = 0;
  std::string err;
  // profiling
  unsigned prof_mask = 0;
  std::vector<ProfEntry> prof_live;
  std::vector<hipEvent_t> ev_pool;
  double prof_ms[OCSC_KC_COUNT] = {0};
  int64_t prof_n[OCSC_KC_COUNT] = {0};
};

namespace {

int fail(ocsc_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  else g_init_error = msg;
  return code;
}

#define HIPX(ctx, call)                                                                      \
  do {                                                                                       \
    hipError_t e_ = (call);                                                                  \
    if (e_ != hipSuccess)                                                                    \
      return fail(ctx, OCSC_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_));       \
  } while (0)

#define LAUNCHED(ctx)                                                                        \
  do {                                                                                       \
    hipError_t e_ = hipGetLastError();                                                       \
    if (e_ != hipSuccess)                                                                    \
      return fail(ctx, OCSC_E_HIP, std::string("kernel launch: ") + hipGetErrorString(e_));  \
  } while (0)

// A roctx range around each C-ABI call that enqueues or waits for work, so
// that a profiler trace (rocprofv3 --marker-trace) shows the host call above
// its kernels.  Without a profiler attached the calls cost a few nanoseconds.
struct ApiRange {
  explicit ApiRange(const char* name) { roctxRangePushA(name); }
  ~ApiRange() { roctxRangePop(); }
  ApiRange(const ApiRange&) = delete;
  ApiRange& operator=(const ApiRange&) = delete;
};
#define OCSC_RANGE() ApiRange api_range_(__func__)

bool pow2_in(int v, int lo, int hi) { return v >= lo && v <= hi && (v & (v - 1)) == 0; }

// ---------------------------------------------------------------- profiling
hipEvent_t ev_get(ocsc_ctx* c) {
  if (!c->ev_pool.empty()) {
    hipEvent_t e = c->ev_pool.back();
    c->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

int prof_collect(ocsc_ctx* c) {
  for (auto& pe : c->prof_live) {
    HIPX(c, hipEventSynchronize(pe.b));
    float ms = 0;
    HIPX(c, hipEventElapsedTime(&ms, pe.a, pe.b));
    c->prof_ms[pe.cls] += ms;
    c->prof_n[pe.cls] += 1;
    c->ev_pool.push_back(pe.a);
    c->ev_pool.push_back(pe.b);
  }
  c->prof_live.clear();
  return OCSC_OK;
}

struct ProfScope {
  ocsc_ctx* c;
  int cls;
  hipEvent_t a = nullptr;
  ProfScope(ocsc_ctx* c_, int cls_) : c(c_), cls(cls_) {
    if (c->prof_mask & (1u << cls)) {
      a = ev_get(c);
      if (a) (void)hipEventRecord(a, c->stream);
    }
  }
  ~ProfScope() {
    if (!a) return;
    hipEvent_t b = ev_get(c);
    if (!b) return;
    (void)hipEventRecord(b, c->stream);
    c->prof_live.push_back({cls, a, b});
    if (c->prof_live.size() >= 4096) prof_collect(c);
  }
};

// One timed kernel launch: the start and stop events travel with the launch
// (hipExtLaunchKernelGGL) and take the kernel's own start and end, so no
// event packets sit between the kernels of the stream.  Without timing the
// launch is a plain one.
struct LaunchTimer {
  ocsc_ctx* c;
  int cls;
  hipEvent_t a = nullptr, b = nullptr;
  LaunchTimer(ocsc_ctx* c_, int cls_) : c(c_), cls(cls_) {
    if (c->prof_mask & (1u << cls)) {
      a = ev_get(c);
      b = a ? ev_get(c) : nullptr;
      if (a && !b) {
        c->ev_pool.push_back(a);
        a = nullptr;
      }
    }
  }
  void launched() {
    if (!a) return;
    c->prof_live.push_back({cls, a, b});
    a = b = nullptr;
    if (c->prof_live.size() >= 4096) prof_collect(c);
  }
  ~LaunchTimer() {
    if (a) {
      c->ev_pool.push_back(a);
      c->ev_pool.push_back(b);
    }
  }
};
#define TIMED_LAUNCH(tm, kernel, grid, block, smem, stream, ...)                                    \
  do {                                                                                             \
    if ((tm).a) hipExtLaunchKernelGGL(kernel, grid, block, smem, stream, (tm).a, (tm).b, 0, __VA_ARGS__); \
    else hipLaunchKernelGGL(kernel, grid, block, smem, stream, __VA_ARGS__);                       \
  } while (0)

// ---------------------------------------------------------------- dispatch
// 128 x 128 planes: 16 waves per workgroup, so that one CU has enough waves
// to overlap the LDS and global latencies of the transform passes.
constexpr int plane_threads(int ph, int pw) { return ph * pw >= 128 * 128 ? 1024 : 256; }
// plane-kernel workgroup sizes offered to the tuner: at least four reals per thread
constexpr bool plane_nt_ok(int ph, int pw, int nt) {
  return (nt == 256 || nt == 512 || nt == 1024) && nt * 4 <= ph * pw;
}

#define OCSC_SIZE_CASES(X) \
  X(32, 32) X(32, 64) X(32, 128) X(64, 32) X(64, 64) X(64, 128) X(128, 32) X(128, 64) X(128, 128)
// grids whose planes do not fit in LDS: two-pass transforms (bigplane.hpp)
#define OCSC_BIG_CASES(X) X(256, 256) X(256, 512) X(512, 256) X(512, 512)
// one-pass grids whose code-plane step may also run as the two-pass kernels
#define OCSC_TWO_PASS_SMALL(X) X(64, 64) X(128, 128)
bool two_pass_capable(int ph, int pw) { return (ph == 64 && pw == 64) || (ph == 128 && pw == 128); }

bool big_grid(int ph, int pw) { return ph > 128 || pw > 128; }

// Two-pass forward R2C of nplanes planes into spectra of stride Pf (row pass
// into dst, column pass in place).
template <typename T>
int launch_big_rfft2(ocsc_ctx* c, const T* src, int sh, int sw, long sstride, cx<T>* dst, int nplanes) {
  const cx<T>* tH = (const cx<T>*)c->twH;
  const cx<T>* tW = (const cx<T>*)c->twW;
  const dim3 rows(c->Ph / BIG_RB, nplanes), cols((c->Wc + big_cb<T>() - 1) / big_cb<T>(), nplanes);
  switch (c->Ph * 1000 + c->Pw) {
#define X(A, B)                                                                                          \
  case A * 1000 + B:                                                                                     \
    hipLaunchKernelGGL((k_big_rows_fwd<T, A, B>), rows, dim3(256), 0, c->stream, src, sh, sw, sstride, dst, \
                       (long)c->Pf, tW);                                                                 \
    hipLaunchKernelGGL((k_big_cols<T, A, B, false>), cols, dim3(256), 0, c->stream, dst, dst, tH);       \
    break;
    OCSC_BIG_CASES(X)
#undef X
    default:
      return fail(c, OCSC_E_UNSUPPORTED, "no transform kernel for this grid");
  }
  LAUNCHED(c);
  return OCSC_OK;
}

template <typename T>
int launch_rfft2(ocsc_ctx* c, const T* src, int sh, int sw, long sstride, cx<T>* dst, long dstride,
                 int nplanes) {
  if (nplanes <= 0) return OCSC_OK;
  ProfScope ps(c, OCSC_KC_FFT);
  if (c->big) {
    if (dstride != c->Pf) return fail(c, OCSC_E_INVALID_ARG, "internal: spectrum stride");
    return launch_big_rfft2<T>(c, src, sh, sw, sstride, dst, nplanes);
  }
  const cx<T>* tH = (const cx<T>*)c->twH;
  const cx<T>* tW = (const cx<T>*)c->twW;
  switch (c->Ph * 1000 + c->Pw) {
#define X(A, B)                                                                                   \
  case A * 1000 + B:                                                                              \
    hipLaunchKernelGGL((k_rfft2<T, A, B, plane_threads(A, B)>), dim3(nplanes), dim3(plane_threads(A, B)), 0, \
                       c->stream, src, sh, sw, sstride, dst, dstride, tH, tW);                    \
    break;
    OCSC_SIZE_CASES(X)
#undef X
    default:
      return fail(c, OCSC_E_UNSUPPORTED, "no transform kernel for this grid");
  }
  LAUNCHED(c);
  return OCSC_OK;
}

template <typename T>
int launch_irfft2_crop(ocsc_ctx* c, const cx<T>* src, long sstride, T* dst, int oh, int ow, long dstride,
                       int nplanes) {
  ProfScope ps(c, OCSC_KC_FFT);
  const cx<T>* tH = (const cx<T>*)c->twH;
  const cx<T>* tW = (const cx<T>*)c->twW;
  if (c->big) {
    // column pass into the code workspace S (free between calls; nplanes <= K), then rows
    if (sstride != c->Pf || nplanes > c->maxB * c->K) return fail(c, OCSC_E_INVALID_ARG, "internal: spectrum stride");
    cx<T>* tmp = (cx<T>*)c->S;
    const dim3 rows((oh + BIG_RB - 1) / BIG_RB, nplanes), cols((c->Wc + big_cb<T>() - 1) / big_cb<T>(), nplanes);
    switch (c->Ph * 1000 + c->Pw) {
#define X(A, B)                                                                                           \
  case A * 1000 + B:                                                                                      \
    hipLaunchKernelGGL((k_big_cols<T, A, B, true>), cols, dim3(256), 0, c->stream, src, tmp, tH);         \
    hipLaunchKernelGGL((k_big_rows_inv_crop<T, A, B>), rows, dim3(256), 0, c->stream, (const cx<T>*)tmp,  \
                       (long)c->Pf, dst, oh, ow, dstride, tW);                                            \
    break;
      OCSC_BIG_CASES(X)
#undef X
      default:
        return fail(c, OCSC_E_UNSUPPORTED, "no transform kernel for this grid");
    }
    LAUNCHED(c);
    return OCSC_OK;
  }
  switch (c->Ph * 1000 + c->Pw) {
#define X(A, B)                                                                                         \
  case A * 1000 + B:                                                                                    \
    hipLaunchKernelGGL((k_irfft2_crop<T, A, B, plane_threads(A, B)>), dim3(nplanes), dim3(plane_threads(A, B)), 0, \
                       c->stream, src, sstride, dst, oh, ow, dstride, tH, tW);                          \
    break;
    OCSC_SIZE_CASES(X)
#undef X
    default:
      return fail(c, OCSC_E_UNSUPPORTED, "no transform kernel for this grid");
  }
  LAUNCHED(c);
  return OCSC_OK;
}

// Two-pass code-plane step of one grid in the context's launch shape (column
// block of col_bytes per spectrum row, row_block rows per row workgroup).
template <typename T, int A, int B, int CB, int RB>
void big_code_plane_shape(ocsc_ctx* c, const cx<T>* Zh, cx<T>* Yb, T* W, cx<T>* S, T* Uout, int nplanes, T kappa,
                          int first, int last) {
  const cx<T>* tH = (const cx<T>*)c->twH;
  const cx<T>* tW = (const cx<T>*)c->twW;
  constexpr int NTC = big_cols_nt<T, CB>();
  const dim3 rows(A / RB, nplanes), cols((c->Wc + CB - 1) / CB, nplanes);
  hipLaunchKernelGGL((k_big_cols<T, A, B, true, CB>), cols, dim3(NTC), 0, c->stream, Zh, Yb, tH);
  hipLaunchKernelGGL((k_big_code_rows<T, A, B, RB>), rows, dim3(256), 0, c->stream, (const cx<T>*)Yb, W, S, Uout,
                     tW, kappa, first, last);
  if (!last) hipLaunchKernelGGL((k_big_cols<T, A, B, false, CB>), cols, dim3(NTC), 0, c->stream, (const cx<T>*)S, S, tH);
}

template <typename T, int A, int B>
bool big_code_plane(ocsc_ctx* c, const cx<T>* Zh, cx<T>* Yb, T* W, cx<T>* S, T* Uout, int nplanes, T kappa,
                    int first, int last) {
  const int cbytes = c->tune.col_bytes, rb = c->tune.row_block;
#define X(CBY, RB)                                                                                        \
  if constexpr ((long)A * CBY <= 131072) {                                                                \
    if (cbytes == CBY && rb == RB) {                                                                      \
      big_code_plane_shape<T, A, B, CBY / (int)sizeof(cx<T>), RB>(c, Zh, Yb, W, S, Uout, nplanes, kappa,  \
                                                                  first, last);                           \
      return true;                                                                                        \
    }                                                                                                     \
  }
  X(128, 4) X(128, 8) X(128, 16) X(256, 4) X(256, 8) X(256, 16) X(512, 4) X(512, 8) X(512, 16)
#undef X
  return false;
}

template <typename T>
int launch_code_plane(ocsc_ctx* c, int off, int nplanes, T* Uout, int first, int last) {
  // samples [off, off + nplanes / K) of the code workspace
  cx<T>* const Zh = (cx<T>*)c->Zh + (size_t)off * c->K * c->Pf;
  cx<T>* const S = (cx<T>*)c->S + (size_t)off * c->K * c->Pf;
  cx<T>* const Yb = c->tune.two_pass == 1 ? (cx<T>*)c->Yb + (size_t)off * c->K * c->Pf : nullptr;
  T* const W = (T*)c->W + (size_t)off * c->K * c->P;
  ProfScope ps(c, OCSC_KC_CODEPLANE);
  const cx<T>* tH = (const cx<T>*)c->twH;
  const cx<T>* tW = (const cx<T>*)c->twW;
  const T kappa = (T)(c->lam / c->rho);
  if (c->tune.two_pass == 2) {
    // each plane split by row parity over two workgroups (the Z-step forms the spectrum)
    const int nt = c->tune.plane_threads;
    bool done = false;
    switch (c->Ph * 1000 + c->Pw) {
#define OCSC_SPLIT_NT(A, B, NT)                                                                          \
  if constexpr (plane_nt_ok(A, B, NT)) {                                                                 \
    if (nt == NT) {                                                                                      \
      hipLaunchKernelGGL((k_code_plane_split<T, A, B, NT>), dim3(split_rows((int)sizeof(T), A, B) * nplanes), \
                         dim3(NT), 0, c->stream,                                                         \
                         (const cx<T>*)Zh, W, S, Uout, tH, tW, kappa, first, last, nplanes);             \
      done = true;                                                                                       \
    }                                                                                                    \
  }
#define X(A, B)              \
  case A * 1000 + B:         \
    OCSC_SPLIT_NT(A, B, 256)  \
    OCSC_SPLIT_NT(A, B, 512)  \
    OCSC_SPLIT_NT(A, B, 1024) \
    break;
      OCSC_SIZE_CASES(X)
      OCSC_BIG_CASES(X)
#undef X
#undef OCSC_SPLIT_NT
      default:
        break;
    }
    if (!done) return fail(c, OCSC_E_UNSUPPORTED, "no split code-plane kernel for this grid and workgroup size");
    LAUNCHED(c);
    return OCSC_OK;
  }
  if (c->tune.two_pass) {
    // column inverse of Zh into Y, row pass (U-step, dual, rows of F(U - W)) into S, column pass on S
    bool done = false;
    switch (c->Ph * 1000 + c->Pw) {
#define X(A, B)                                              \
  case A * 1000 + B:                                         \
    done = big_code_plane<T, A, B>(c, Zh, Yb, W, S, Uout, nplanes, kappa, first, last); \
    break;
      OCSC_BIG_CASES(X)
      OCSC_TWO_PASS_SMALL(X)
#undef X
      default:
        break;
    }
    if (!done) return fail(c, OCSC_E_UNSUPPORTED, "no code-plane kernel for this grid and launch shape");
    LAUNCHED(c);
    return OCSC_OK;
  }
  const int nt = c->tune.plane_threads;
  bool done = false;
  switch (c->Ph * 1000 + c->Pw) {
#define OCSC_PLANE_NT(A, B, NT)                                                                          \
  if constexpr (plane_nt_ok(A, B, NT)) {                                                                 \
    if (nt == NT) {                                                                                      \
      hipLaunchKernelGGL((k_code_plane<T, A, B, NT>), dim3(nplanes), dim3(NT), 0, c->stream,             \
                         (const cx<T>*)Zh, W, S, Uout, tH, tW, kappa, first, last);                      \
      done = true;                                                                                       \
    }                                                                                                    \
  }
#define X(A, B)              \
  case A * 1000 + B:         \
    OCSC_PLANE_NT(A, B, 256)  \
    OCSC_PLANE_NT(A, B, 512)  \
    OCSC_PLANE_NT(A, B, 1024) \
    break;
    OCSC_SIZE_CASES(X)
#undef X
#undef OCSC_PLANE_NT
    default:
      break;
  }
  if (!done) return fail(c, OCSC_E_UNSUPPORTED, "no code-plane kernel for this grid and workgroup size");
  LAUNCHED(c);
  return OCSC_OK;
}

template <typename T, int KPT, int ZF, int SB>
void zstep_kernel(ocsc_ctx* c, int off, int B, int first, cx<T>* Zt) {
  const cx<T>* xh = (const cx<T>*)c->xh + (size_t)off * c->Pf;
  const cx<T>* S = (const cx<T>*)c->S + (size_t)off * c->K * c->Pf;
  cx<T>* Zh = (cx<T>*)c->Zh + (size_t)off * c->K * c->Pf;
  if (c->tune.two_pass == 2) {
    // S holds the column DFTs of the row residues of the split plane step
    const int F = split_rows(c->sr, c->Ph, c->Pw), zb = ZF / F;
    const dim3 grid((c->Pf / F + zb - 1) / zb, (B + SB - 1) / SB);
    hipLaunchKernelGGL((k_code_zstep<T, KPT, ZF, SB, true>), grid, dim3(16 * ZF), 0, c->stream,
                       (const cx<T>*)c->Dh, (const T*)c->gam, xh, S, Zh, c->K, c->Pf, B, first, Zt, c->maxB, off,
                       (const cx<T>*)c->twH, c->Wc, F);
    return;
  }
  const dim3 grid((c->Pf + ZF - 1) / ZF, (B + SB - 1) / SB);
  hipLaunchKernelGGL((k_code_zstep<T, KPT, ZF, SB, false>), grid, dim3(16 * ZF), 0, c->stream, (const cx<T>*)c->Dh,
                     (const T*)c->gam, xh, S, Zh, c->K, c->Pf, B, first, Zt, c->maxB, off, (const cx<T>*)nullptr,
                     c->Wc, 1);
}

template <typename T, int KPT>
bool zstep_shape(ocsc_ctx* c, int off, int B, int first, cx<T>* Zt) {
  const int zf = c->tune.zstep_freqs, sb = c->tune.zstep_samples;
#define X(ZF, SB) \
  if (zf == ZF && sb == SB) { zstep_kernel<T, KPT, ZF, SB>(c, off, B, first, Zt); return true; }
  X(16, 1) X(16, 2) X(16, 4) X(32, 1) X(32, 2) X(32, 4) X(64, 1) X(64, 2) X(64, 4)
#undef X
  return false;
}

template <typename T>
int launch_zstep(ocsc_ctx* c, int off, int B, int first, bool last) {
  ProfScope ps(c, OCSC_KC_ZSTEP);
  // the last iterate also goes frequency-major, for the matrix-core history
  // update and for the fold of several samples
  cx<T>* Zt = (last && c->Zt) ? (cx<T>*)c->Zt : nullptr;
  const int K = c->K;
  bool ok = false;
  if (K <= 16) ok = zstep_shape<T, 1>(c, off, B, first, Zt);
  else if (K <= 32) ok = zstep_shape<T, 2>(c, off, B, first, Zt);
  else if (K <= 64) ok = zstep_shape<T, 4>(c, off, B, first, Zt);
  else if (K <= 128) ok = zstep_shape<T, 8>(c, off, B, first, Zt);
  else if (K <= 256) ok = zstep_shape<T, 16>(c, off, B, first, Zt);
  else return fail(c, OCSC_E_UNSUPPORTED, "code Z-step supports K <= 256");
  if (!ok) return fail(c, OCSC_E_INVALID_ARG, "internal: Z-step shape");
  LAUNCHED(c);
  return OCSC_OK;
}

template <typename T>
int launch_gamma(ocsc_ctx* c) {
  ProfScope ps(c, OCSC_KC_OTHER);
  hipLaunchKernelGGL((k_gamma<T>), dim3((c->Pf + 63) / 64), dim3(256), 0, c->stream, (const cx<T>*)c->Dh,
                     (T*)c->gam, (T)c->rho, c->K, c->Pf);
  LAUNCHED(c);
  return OCSC_OK;
}

// Compile-time specialisations of the D-step sweep (real type, K, fpb); the
// generic kernels serve every other shape.
#define OCSC_SWEEP_SPECS(X) X(float, 100, 1) X(float, 16, 16) X(double, 16, 8)

// bytes of one D-step slot: C of fpb frequencies in the R-form
size_t sweep_slot_bytes(int K, int fpb, size_t sr) {
  const int vr = (int)(16 / sr);
  return (size_t)fpb * ((size_t)(K * (K + 1) + vr - 1) / vr * vr) * sr;
}

int sweep_nvm_for(int K, int fpb, size_t sr) {
#define X(T, KT, FPB) \
  if (sr == sizeof(T) && K == KT && fpb == FPB) return sweep_nvm<T, KT, FPB>();
  OCSC_SWEEP_SPECS(X)
#undef X
  return sweep_slot_bytes(K, fpb, sr) <= (size_t)256 * SWEEP_MAXV * 16 ? SWEEP_MAXV : SWEEP_MAXV_L;
}

// K rounded up to 16 for the matrix-core fold (FP32, K <= 128)
#define OCSC_FOLD_KP(X) X(16) X(32) X(48) X(64) X(80) X(96) X(112) X(128)

// One D-step sweep; nfold > 0 folds the kept spectra of nfold samples first.
template <typename T>
int launch_sweep(ocsc_ctx* c, int nfold, const void* rhs, void* rfold, void* dout, int cls) {
  LaunchTimer tm(c, cls);
  if constexpr (std::is_same<T, float>::value) {
    if (nfold >= 2 && !c->dstream) {
      // several pending samples (FP32): blocks of sixteen on the matrix cores,
      // then the first D-step as a plain sweep of the folded C
      const size_t lds = fold_mfma_lds(c->K, c->fs);
      bool done = false;
#define X(KP)                                                                                             \
  if (!done && (c->K + 15) / 16 * 16 == KP) {                                                             \
    TIMED_LAUNCH(tm, k_fold_mfma<KP>, dim3(c->Pf), dim3(FM_NT), lds, c->stream, (float*)c->Cm, c->fs, c->K, \
                 c->Pf, (float2*)c->G, (float2*)rfold, (const float2*)c->Zt, c->maxB, (const float2*)c->xh, \
                 nfold);                                                                                  \
    done = true;                                                                                          \
  }
      OCSC_FOLD_KP(X)
#undef X
      if (!done) return fail(c, OCSC_E_STATE, "internal: no fold kernel for this K");
      LAUNCHED(c);
      tm.launched();
      if (!dout) return OCSC_OK;
      return launch_sweep<T>(c, 0, rfold ? rfold : c->G, nullptr, dout, cls);
    }
  }
  // successive sweeps alternate direction (the tail of one sweep first in the
  // next; with the non-temporal loads of C this no longer changes the time,
  // and the direction changes no result)
  const int reverse = (int)(c->sweep_count & 1u);
  c->sweep_count++;
  if (c->dstream) {
    // K > 128 (Cholesky form, no fold): C_p streamed through LDS
    if (nfold || !dout) return fail(c, OCSC_E_STATE, "internal: no history fold in the K > 128 form");
    if constexpr (std::is_same<T, float>::value) {
      TIMED_LAUNCH(tm, k_dstep_stream, dim3(c->Pf), dim3(256), 0, c->stream, (const float*)c->Cm, c->fs, c->K,
                   c->Pf, (const float2*)rhs, (float2*)dout);
      LAUNCHED(c);
      tm.launched();
      return OCSC_OK;
    }
    return fail(c, OCSC_E_UNSUPPORTED, "the K > 128 form is FP32");
  }
  if (nfold == 0 && !dout) return fail(c, OCSC_E_STATE, "internal: a sweep with neither fold nor D-step");
  const size_t smem = nfold == 0 ? c->plain_smem : c->sweep_smem;
  const int mode = nfold == 0 ? 0 : (nfold == 1 ? 1 : 2);
#define OCSC_SWEEP_M(KT, FPB, M)                                                                              \
  TIMED_LAUNCH(tm, (k_dict_sweep<T, KT, FPB, M>), dim3(nfold ? c->fold_wgs : c->sweep_wgs), dim3(256), smem,   \
               c->stream,                                                                                     \
               (T*)c->Cm, (cx<T>*)c->G, (const cx<T>*)rhs, (const cx<T>*)c->Zh, (const cx<T>*)c->Zt, c->maxB,  \
               (const cx<T>*)c->xh, nfold, (cx<T>*)rfold, (cx<T>*)dout, c->K, c->Pf, c->fpb, c->fs,            \
               c->slots_per_wg, reverse)
#define OCSC_SWEEP(KT, FPB)                        \
  do {                                             \
    if (mode == 2) OCSC_SWEEP_M(KT, FPB, 2);       \
    else if (mode == 1) OCSC_SWEEP_M(KT, FPB, 1);  \
    else OCSC_SWEEP_M(KT, FPB, 0);                 \
  } while (0)
  bool done = false;
#define X(TT, KT, FPB)                                                          \
  if constexpr (std::is_same<T, TT>::value) {                                  \
    if (!done && c->K == KT && c->fpb == FPB) {                                \
      OCSC_SWEEP(KT, FPB);                                                     \
      done = true;                                                             \
    }                                                                          \
  }
  OCSC_SWEEP_SPECS(X)
#undef X
  if (!done) {
    if (sweep_nvm_for(c->K, c->fpb, sizeof(T)) == SWEEP_MAXV_L) OCSC_SWEEP(-1, 0);
    else OCSC_SWEEP(0, 0);
  }
#undef OCSC_SWEEP
#undef OCSC_SWEEP_M
  LAUNCHED(c);
  tm.launched();
  return OCSC_OK;
}

// LDS of the fused V-step for one plane size and real type (bytes)
template <typename T, int PH, int PW, int NQ>
constexpr size_t vstep_filter_lds() {
  using Gm = PlaneGeom<PH, PW>;
  return sizeof(cx<T>) * ((size_t)Gm::PF + (size_t)NQ * VF * Gm::WC + PH + PW) + sizeof(T) * (VF * VF + 16);
}
template <typename T> constexpr int vstep_nq() { return sizeof(T) == 4 ? 4 : 2; }

template <typename T>
bool vstep_fused_ok(int ph, int pw, int mh, int mw) {
  if (mh > VF || mw > VF) return false;
  size_t lds = 0;
  switch (ph * 1000 + pw) {
#define X(A, B) \
  case A * 1000 + B: lds = vstep_filter_lds<T, A, B, vstep_nq<T>()>(); break;
    OCSC_SIZE_CASES(X)
#undef X
    default: return false;
  }
  return lds <= 150 * 1024;
}

template <typename T>
int launch_vstep(ocsc_ctx* c, int first) {
  ProfScope ps(c, OCSC_KC_VSTEP);
  if (c->vstep_fused && sizeof(T) == 4) {
    // FP32: the pruned DFTs on the matrix cores
    switch (c->Ph * 1000 + c->Pw) {
#define X(A, B)                                                                                                \
  case A * 1000 + B:                                                                                           \
    hipLaunchKernelGGL((k_vstep_mfma<A, B>), dim3(c->K), dim3(1024), 0, c->stream, (const float2*)c->d,        \
                       (float2*)c->Th, (const float2*)c->G, (float2*)c->rhs, (float*)c->V,                     \
                       (const float2*)c->twH, (const float2*)c->twW, c->Mh, c->Mw, (float)c->rho_d, first);    \
    break;
      OCSC_SIZE_CASES(X)
#undef X
      default:
        return fail(c, OCSC_E_UNSUPPORTED, "no V-step kernel for this grid");
    }
    LAUNCHED(c);
    return OCSC_OK;
  }
  if (c->vstep_fused) {
    const cx<T>* tH = (const cx<T>*)c->twH;
    const cx<T>* tW = (const cx<T>*)c->twW;
    constexpr int NQ = vstep_nq<T>();
    switch (c->Ph * 1000 + c->Pw) {
#define X(A, B)                                                                                                 \
  case A * 1000 + B:                                                                                            \
    if constexpr (vstep_filter_lds<T, A, B, NQ>() <= 150 * 1024) {                                              \
      hipLaunchKernelGGL((k_vstep_filter<T, A, B, 1024, NQ>), dim3(c->K), dim3(1024), 0, c->stream,            \
                         (const cx<T>*)c->d, (cx<T>*)c->Th, (const cx<T>*)c->G, (cx<T>*)c->rhs, (T*)c->V, tH, tW, \
                         c->Mh, c->Mw, (T)c->rho_d, first);                                                     \
    }                                                                                                           \
    break;
      OCSC_SIZE_CASES(X)
#undef X
      default:
        return fail(c, OCSC_E_UNSUPPORTED, "no V-step kernel for this grid");
    }
    LAUNCHED(c);
    return OCSC_OK;
  }
  dim3 grid(c->nvb, c->K);
#define OCSC_VSTEP_COLS(MAXP)                                                                                    \
  hipLaunchKernelGGL((k_vstep_alpha<T, MAXP>), grid, dim3(256), 0, c->stream, (const cx<T>*)c->d,                \
                     (const cx<T>*)c->Th, (T*)c->apart, (const cx<T>*)c->twH, (const cx<T>*)c->twW, c->Ph,        \
                     c->Pw, c->Mh, c->Mw, first);                                                                \
  hipLaunchKernelGGL((k_vstep_apply<T, MAXP>), grid, dim3(256), c->vapply_smem, c->stream, (const cx<T>*)c->d,   \
                     (cx<T>*)c->Th, (const cx<T>*)c->G, (cx<T>*)c->rhs, (const T*)c->apart, (T*)c->V,             \
                     (const cx<T>*)c->twH, (const cx<T>*)c->twW, c->Ph, c->Pw, c->Mh, c->Mw, (T)c->rho_d, first)
  if (c->big) {
    OCSC_VSTEP_COLS(512);
  } else {
    OCSC_VSTEP_COLS(128);
  }
#undef OCSC_VSTEP_COLS
  LAUNCHED(c);
  return OCSC_OK;
}

// Apply a deferred history fold on its own (no D-step).
template <typename T>
int flush_fold(ocsc_ctx* c) {
  if (c->fold_B == 0) return OCSC_OK;
  int rc = launch_sweep<T>(c, c->fold_B, nullptr, c->warm ? c->rhs : nullptr, nullptr, OCSC_KC_HISTORY);
  if (rc) return rc;
  c->fold_B = 0;
  return OCSC_OK;
}

// The J_z ADMM iterations of samples [off, off + B) (spectra already in xh).
// With chunk_samples set, groups of that many samples run all their
// iterations before the next group starts, so that a group's code workspace
// (spectra, dual, column-pass output) can stay in the Infinity Cache between
// launches; the samples are independent, so the values are the same.
template <typename T>
int code_iterations(ocsc_ctx* c, int off, int B, T* Uout) {
  const int chunk = c->tune.chunk_samples > 0 ? c->tune.chunk_samples : B;
  for (int s0 = 0; s0 < B; s0 += chunk) {
    const int nb = B - s0 < chunk ? B - s0 : chunk;
    T* U = Uout ? Uout + (size_t)s0 * c->K * c->P : nullptr;
    for (int j = 0; j < c->Jz; ++j) {
      int rc = launch_zstep<T>(c, off + s0, nb, j == 0, j == c->Jz - 1);
      if (rc) return rc;
      rc = launch_code_plane<T>(c, off + s0, nb * c->K, U, j == 0, j == c->Jz - 1);
      if (rc) return rc;
    }
  }
  return OCSC_OK;
}

// ---------------------------------------------------------------- calls by type
// Code B samples into the pending slots [off, off + B) (off = 0: a new
// minibatch; off = pending_B: appended to the pending ones).
// Before the iterations: a deferred fold, then the sample spectra into slots [off, off + B).
template <typename T>
int code_prologue(ocsc_ctx* c, const void* x, int B, int off) {
  int rc = flush_fold<T>(c);
  if (rc) return rc;
  return launch_rfft2<T>(c, (const T*)x, c->Ph, c->Pw, c->P, (cx<T>*)c->xh + (size_t)off * c->Pf, c->Pf, B);
}

// Where the codes of slots [off, ...) go: the caller's buffer, else (history
// kept) the library's, else nowhere.
template <typename T>
T* code_out(ocsc_ctx* c, void* codes, int off) {
  return codes ? (T*)codes : (c->Ubuf ? (T*)c->Ubuf + (size_t)off * c->K * c->P : nullptr);
}

// After the iterations: per-sample partial sums for the kept history; the
// slots become pending.
template <typename T>
int code_epilogue(ocsc_ctx* c, const T* Uout, int B, int off) {
  if (c->keep_hist) {
    // per-sample partial sums of ||x_b||^2 (Parseval) and ||U_b||_1, added to
    // the running sums when the samples are accumulated
    ProfScope ps(c, OCSC_KC_OTHER);
    hipLaunchKernelGGL((k_wsq<T>), dim3(64, B), dim3(256), 0, c->stream,
                       (const cx<T>*)c->xh + (size_t)off * c->Pf, (const cx<T>*)nullptr, c->pend + (size_t)off * 64,
                       1, c->Pf, c->Pw);
    LAUNCHED(c);
    hipLaunchKernelGGL((k_abs_sum<T>), dim3(64, B), dim3(256), 0, c->stream, Uout,
                       c->pend + (size_t)(c->maxB + off) * 64, (long)c->K * c->P);
    LAUNCHED(c);
  }
  c->pending_B = off + B;
  return OCSC_OK;
}

// Code B samples into the pending slots [off, off + B) (off = 0: a new
// minibatch; off = pending_B: appended to the pending ones).
template <typename T>
int code_update_t(ocsc_ctx* c, const void* x, int B, void* codes, int off) {
  int rc = code_prologue<T>(c, x, B, off);
  if (rc) return rc;
  T* Uout = code_out<T>(c, codes, off);
  rc = code_iterations<T>(c, off, B, Uout);
  if (rc) return rc;
  return code_epilogue<T>(c, Uout, B, off);
}

// Batches on several contexts (slots from 0), their iterations in one
// cooperative launch of k_code_group on the first context's stream.
template <typename T>
int code_group_t(ocsc_ctx* const* cs, const void* const* xs, const int* Bs, void* const* codes, int n) {
  ocsc_ctx* c0 = cs[0];
  CodeGroupArgs<T> g{};
  g.n = n;
  g.Jz = c0->Jz;
  size_t smem = 16 * (CG_ZF + 1) * sizeof(cx<T>);
  int kmax = 0;
  T* U[CG_MAX] = {};
  long z = 0, pl = 0, r = 0, f = 0;
  for (int s = 0; s < n; ++s) {
    ocsc_ctx* c = cs[s];
    int rc = code_prologue<T>(c, xs[s], Bs[s], 0);
    if (rc) return rc;
    U[s] = code_out<T>(c, codes ? codes[s] : nullptr, 0);
    const int B = Bs[s], BK = B * c->K;
    g.ph[s] = c->Ph;
    g.pw[s] = c->Pw;
    g.K[s] = c->K;
    g.B[s] = B;
    g.Pf[s] = c->Pf;
    g.big[s] = c->big;
    g.ldt[s] = c->maxB;
    g.Dh[s] = (const cx<T>*)c->Dh;
    g.gam[s] = (const T*)c->gam;
    g.xh[s] = (const cx<T>*)c->xh;
    g.S[s] = (cx<T>*)c->S;
    g.Zh[s] = (cx<T>*)c->Zh;
    g.W[s] = (T*)c->W;
    g.Yb[s] = (cx<T>*)c->Yb;
    g.U[s] = U[s];
    g.Zt[s] = (cx<T>*)c->Zt;
    g.twH[s] = (const cx<T>*)c->twH;
    g.twW[s] = (const cx<T>*)c->twW;
    g.kappa[s] = (T)(c->lam / c->rho);
    g.z0[s] = (int)z;
    g.p0[s] = (int)pl;
    g.r0[s] = (int)r;
    g.f0[s] = (int)f;
    z += (long)((c->Pf + CG_ZF - 1) / CG_ZF) * ((B + CG_ZS - 1) / CG_ZS);
    size_t need;
    if (c->big) {
      g.any_big = 1;
      pl += (long)cg_col_blocks<T>(c->Pw) * BK;
      r += (long)(c->Ph / BIG_RB) * BK;
      f += (long)cg_col_blocks<T>(c->Pw) * BK;
      const size_t cols = (size_t)c->Ph * (big_cb<T>() + 1), rows = (size_t)BIG_RB * c->Wc + c->Pw;
      need = (cols > rows ? cols : rows) * sizeof(cx<T>);
    } else {
      pl += BK;
      need = ((size_t)c->Ph * c->Wc + c->Ph + c->Pw) * sizeof(cx<T>);
    }
    if (need > smem) smem = need;
    if (c->K > kmax) kmax = c->K;
  }
  if (z > INT32_MAX || pl > INT32_MAX || r > INT32_MAX || f > INT32_MAX)
    return fail(c0, OCSC_E_INVALID_ARG, "too many work items for one launch");
  g.z0[n] = (int)z;
  g.p0[n] = (int)pl;
  g.r0[n] = (int)r;
  g.f0[n] = (int)f;
  const void* fn = kmax <= 16 ? (const void*)k_code_group<T, 1> : (const void*)k_code_group<T, 8>;
  HIPX(c0, hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem));
  int per_cu = 0, cus = 0;
  HIPX(c0, hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, CG_NT, smem));
  HIPX(c0, hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c0->device));
  if (per_cu < 1 || cus < 1) return fail(c0, OCSC_E_UNSUPPORTED, "the grouped code kernel does not fit a CU");
  {
    ProfScope ps(c0, OCSC_KC_CODEPLANE);
    void* args[] = {&g};
    HIPX(c0, hipLaunchCooperativeKernel(fn, dim3(per_cu * cus), dim3(CG_NT), args, (unsigned)smem, c0->stream));
  }
  for (int s = 0; s < n; ++s) {
    int rc = code_epilogue<T>(cs[s], U[s], Bs[s], 0);
    if (rc) return rc;
  }
  return OCSC_OK;
}

// Runs a call over several contexts on the first context's stream: that
// stream first waits for the earlier work of every member's stream, each
// member's stream is the first one's during the call, and afterwards every
// member's stream waits for the call's work.
struct StreamJoin {
  ocsc_ctx* const* cs;
  int n;
  hipStream_t ls;
  std::vector<hipStream_t> saved;
  std::vector<hipEvent_t> evs;
  StreamJoin(ocsc_ctx* const* cs_, int n_) : cs(cs_), n(n_), ls(cs_[0]->stream), saved(n_) {
    for (int s = 0; s < n; ++s) saved[s] = cs[s]->stream;
  }
  hipError_t order(hipStream_t from, hipStream_t to) {
    if (from == to) return hipSuccess;
    hipEvent_t e = nullptr;
    hipError_t err = hipEventCreateWithFlags(&e, hipEventDisableTiming);
    if (err != hipSuccess) return err;
    evs.push_back(e);
    err = hipEventRecord(e, from);
    return err == hipSuccess ? hipStreamWaitEvent(to, e, 0) : err;
  }
  hipError_t enter() {
    for (int s = 1; s < n; ++s) {
      hipError_t err = order(saved[s], ls);
      if (err != hipSuccess) return err;
    }
    for (int s = 0; s < n; ++s) cs[s]->stream = ls;
    return hipSuccess;
  }
  hipError_t leave() {
    for (int s = 0; s < n; ++s) cs[s]->stream = saved[s];
    for (int s = 1; s < n; ++s) {
      hipError_t err = order(ls, saved[s]);
      if (err != hipSuccess) return err;
    }
    return hipSuccess;
  }
  ~StreamJoin() {
    for (int s = 0; s < n; ++s) cs[s]->stream = saved[s];
    for (auto e : evs) (void)hipEventDestroy(e);
  }
};

// Precision form with OCSC_FLAG_REFINE: one step of iterative refinement of
// d = C rhs against the kept H (k_dstep_refine), in place.
template <typename T>
int launch_refine(ocsc_ctx* c, const void* rhs) {
  if (!c->refine) return OCSC_OK;
  if constexpr (std::is_same<T, float>::value) {
    ProfScope ps(c, OCSC_KC_OTHER);
    hipLaunchKernelGGL(k_dstep_refine, dim3(c->Pf), dim3(256), 0, c->stream, (const float*)c->Hm,
                       (const float*)c->Cm, c->fs, c->K, c->Pf, c->rho_d, (const float2*)rhs, (float2*)c->d);
    LAUNCHED(c);
    return OCSC_OK;
  }
  return fail(c, OCSC_E_UNSUPPORTED, "refinement is part of the FP32 precision form");
}

template <typename T>
int dict_update_t(ocsc_ctx* c) {
  for (int tau = 0; tau < c->Jd; ++tau) {
    int rc;
    if (tau == 0 && c->fold_B) {
      // fold fused with the first sweep; its right-hand side is G (cold start)
      // or the carried one (warm start)
      rc = launch_sweep<T>(c, c->fold_B, nullptr, c->warm ? c->rhs : nullptr, c->d, OCSC_KC_HISTORY);
      c->fold_B = 0;
    } else {
      const void* r = (tau == 0 && !c->warm) ? c->G : c->rhs;
      rc = launch_sweep<T>(c, 0, r, nullptr, c->d, OCSC_KC_DSTEP);
      if (!rc) rc = launch_refine<T>(c, r);
    }
    if (rc) return rc;
    rc = launch_vstep<T>(c, tau == 0 && !c->warm);
    if (rc) return rc;
  }
  std::swap(c->Dh, c->d);
  // 1 / (rho + ||a_p||^2) of the new dictionary for the next code update
  // (the same kernel as after ocsc_set_dictionary, so a restored learner
  // continues bit for bit)
  return launch_gamma<T>(c);
}

// One DictOCSC over several contexts (grids) sharing one dictionary: each
// context's D-step, the column-block alpha partials of every context, one
// consensus V-step (k_vstep_group_v, weights P_s), then each context's Theta
// and right-hand side from the common V.  Everything is enqueued on the first
// context's stream.
template <typename T>
int dict_update_group_t(ocsc_ctx* const* cs, int n) {
  GroupArgs<T> ga{};
  ga.n = n;
  for (int s = 0; s < n; ++s) {
    ga.apart[s] = (const T*)cs[s]->apart;
    ga.V[s] = (T*)cs[s]->V;
    ga.nvb[s] = cs[s]->nvb;
    ga.w[s] = (T)cs[s]->P;
  }
  const int K = cs[0]->K, MM = cs[0]->Mh * cs[0]->Mw;
  for (int tau = 0; tau < cs[0]->Jd; ++tau) {
    for (int s = 0; s < n; ++s) {
      ocsc_ctx* c = cs[s];
      int rc;
      if (tau == 0 && c->fold_B) {
        rc = launch_sweep<T>(c, c->fold_B, nullptr, nullptr, c->d, OCSC_KC_HISTORY);
        c->fold_B = 0;
      } else {
        rc = launch_sweep<T>(c, 0, tau == 0 ? c->G : c->rhs, nullptr, c->d, OCSC_KC_DSTEP);
        if (!rc) rc = launch_refine<T>(c, tau == 0 ? c->G : c->rhs);
      }
      if (rc) return rc;
    }
    ProfScope ps(cs[0], OCSC_KC_VSTEP);
    for (int s = 0; s < n; ++s) {
      ocsc_ctx* c = cs[s];
      const dim3 grid(c->nvb, K);
#define OCSC_GROUP_ALPHA(MAXP)                                                                                  \
  hipLaunchKernelGGL((k_vstep_alpha<T, MAXP>), grid, dim3(256), 0, c->stream, (const cx<T>*)c->d,               \
                     (const cx<T>*)c->Th, (T*)c->apart, (const cx<T>*)c->twH, (const cx<T>*)c->twW, c->Ph,       \
                     c->Pw, c->Mh, c->Mw, tau == 0)
      if (c->big) {
        OCSC_GROUP_ALPHA(512);
      } else {
        OCSC_GROUP_ALPHA(128);
      }
#undef OCSC_GROUP_ALPHA
      LAUNCHED(c);
    }
    hipLaunchKernelGGL((k_vstep_group_v<T>), dim3(K), dim3(256), MM * sizeof(T), cs[0]->stream, ga, MM);
    LAUNCHED(cs[0]);
    for (int s = 0; s < n; ++s) {
      ocsc_ctx* c = cs[s];
      const dim3 grid(c->nvb, K);
#define OCSC_GROUP_APPLY(MAXP)                                                                                  \
  hipLaunchKernelGGL((k_vstep_apply<T, MAXP>), grid, dim3(256), c->vapply_smem, c->stream, (const cx<T>*)c->d,  \
                     (cx<T>*)c->Th, (const cx<T>*)c->G, (cx<T>*)c->rhs, (const T*)nullptr, (T*)c->V,             \
                     (const cx<T>*)c->twH, (const cx<T>*)c->twW, c->Ph, c->Pw, c->Mh, c->Mw, (T)c->rho_d,        \
                     tau == 0)
      if (c->big) {
        OCSC_GROUP_APPLY(512);
      } else {
        OCSC_GROUP_APPLY(128);
      }
#undef OCSC_GROUP_APPLY
      LAUNCHED(c);
    }
  }
  for (int s = 0; s < n; ++s) {
    std::swap(cs[s]->Dh, cs[s]->d);
    int rc = launch_gamma<T>(cs[s]);
    if (rc) return rc;
  }
  return OCSC_OK;
}

// Cholesky form: report (once) a breakdown the factorisation flagged since the
// last check.  Called by the calls that wait, after their stream sync.
int check_breakdown(ocsc_ctx* c) {
  if (!c->brk) return OCSC_OK;
  int h = 0;
  HIPX(c, hipMemcpyAsync(&h, c->brk, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIPX(c, hipStreamSynchronize(c->stream));
  if (!h) return OCSC_OK;
  HIPX(c, hipMemsetAsync(c->brk, 0, sizeof(int), c->stream));
  HIPX(c, hipStreamSynchronize(c->stream));
  return fail(c, OCSC_E_NUMERIC,
              "Cholesky breakdown: H_p + rho_d I was not positive definite at some frequency "
              "(a non-finite history, or an indefinite H given to ocsc_set_state); C holds NaN there");
}

template <typename T>
int objective_t(ocsc_ctx* c, const void* x, const void* codes, int B, double* out, int terms) {
  int rc = launch_rfft2<T>(c, (const T*)x, c->Ph, c->Pw, c->P, (cx<T>*)c->xh_obj, c->Pf, B);
  if (rc) return rc;
  rc = launch_rfft2<T>(c, (const T*)codes, c->Ph, c->Pw, c->P, (cx<T>*)c->S, c->Pf, B * c->K);
  if (rc) return rc;
  {
    ProfScope ps(c, OCSC_KC_OTHER);
    hipLaunchKernelGGL((k_obj_resid<T>), dim3(c->obj_nr, B), dim3(256), 0, c->stream, (const cx<T>*)c->xh_obj,
                       (const cx<T>*)c->Dh, (const cx<T>*)c->S, c->obj_part, c->K, c->Pw, c->Pf);
    LAUNCHED(c);
    double* lpart = c->obj_part + (size_t)c->maxB * c->obj_nr;
    hipLaunchKernelGGL((k_abs_sum<T>), dim3(c->obj_nl, B), dim3(256), 0, c->stream, (const T*)codes, lpart,
                       (long)c->K * c->P);
    LAUNCHED(c);
    hipLaunchKernelGGL(k_obj_final, dim3(B), dim3(256), 0, c->stream, c->obj_part, c->obj_nr, lpart, c->obj_nl,
                       c->obj_out, 1.0 / c->P, c->lam, terms);
    LAUNCHED(c);
  }
  const int nout = terms ? 2 * B : B;
  HIPX(c, hipMemcpyAsync(out, c->obj_out, sizeof(double) * nout, hipMemcpyDeviceToHost, c->stream));
  HIPX(c, hipStreamSynchronize(c->stream));
  rc = check_breakdown(c);
  if (rc) return rc;
  for (int b = 0; b < nout; ++b)
    if (!std::isfinite(out[b])) return fail(c, OCSC_E_NUMERIC, "objective is not finite");
  return OCSC_OK;
}

// ocsc_objective_noalloc: the kernels of objective_t with every buffer they
// write (sample and code spectra, reduction partials) carved out of the static
// scratch, and the result left in caller-owned device memory.  The partition
// into workgroups is the one of objective_t, so the values are the same bit
// for bit.
size_t noalloc_objective_bytes(const ocsc_ctx* c, int B) {
  auto up = [](size_t n) { return (n + 255) / 256 * 256; };
  const size_t sc = 2 * c->sr;
  return up((size_t)B * c->Pf * sc) + up((size_t)B * c->K * c->Pf * sc) + up((size_t)B * c->obj_nr * 8) +
         up((size_t)B * c->obj_nl * 8);
}

template <typename T>
int objective_noalloc_t(ocsc_ctx* c, const void* x, const void* codes, int B, double* out) {
  char* p = (char*)c->scratch;
  auto take = [&](size_t n) {
    char* q = p;
    p += (n + 255) / 256 * 256;
    return q;
  };
  cx<T>* xh = (cx<T>*)take((size_t)B * c->Pf * sizeof(cx<T>));
  cx<T>* uh = (cx<T>*)take((size_t)B * c->K * c->Pf * sizeof(cx<T>));
  double* rpart = (double*)take((size_t)B * c->obj_nr * sizeof(double));
  double* lpart = (double*)take((size_t)B * c->obj_nl * sizeof(double));
  int rc = launch_rfft2<T>(c, (const T*)x, c->Ph, c->Pw, c->P, xh, c->Pf, B);
  if (rc) return rc;
  rc = launch_rfft2<T>(c, (const T*)codes, c->Ph, c->Pw, c->P, uh, c->Pf, B * c->K);
  if (rc) return rc;
  hipLaunchKernelGGL((k_obj_resid<T>), dim3(c->obj_nr, B), dim3(256), 0, c->stream, (const cx<T>*)xh,
                     (const cx<T>*)c->Dh, (const cx<T>*)uh, rpart, c->K, c->Pw, c->Pf);
  LAUNCHED(c);
  hipLaunchKernelGGL((k_abs_sum<T>), dim3(c->obj_nl, B), dim3(256), 0, c->stream, (const T*)codes, lpart,
                     (long)c->K * c->P);
  LAUNCHED(c);
  hipLaunchKernelGGL(k_obj_final, dim3(B), dim3(256), 0, c->stream, (const double*)rpart, c->obj_nr,
                     (const double*)lpart, c->obj_nl, out, 1.0 / c->P, c->lam, 0);
  LAUNCHED(c);
  return OCSC_OK;
}

// Kept history: H_p += sum_b conj(z_bp) z_bp^T and the running sums, at
// accumulation time (the fold of G and C may still be deferred).
size_t chol_lds(int K) {
  const size_t n = (size_t)(K + CHOL_B - 1) / CHOL_B * CHOL_B;   // padded to whole column blocks
  return (n * (n + 1) / 2 + 2 * CHOL_B * CHOL_B) * 16;
}
// two workgroups of 512 threads per CU when the factor takes at most half the LDS
bool chol_small(int K) { return chol_lds(K) <= 80 * 1024; }

// Precision form: H += conj(Z)^T Z and G += conj(Z)^T x on the matrix cores
// (BF16 split, FP32 accumulation), then C = (H + rho_d I)^-1 by an FP64
// Cholesky per frequency.
int chol_history(ocsc_ctx* c, int B) {
  ProfScope ps(c, OCSC_KC_HISTORY);
  const int KP = (c->K + 15) / 16 * 16;
  switch (KP) {
#define X(N)                                                                                                  \
  case N:                                                                                                     \
    hipLaunchKernelGGL((k_herk_bf16<N, 8, 1, 32>), dim3(c->Pf, 1), dim3(512), 0, c->stream, (const float2*)c->Zt, \
                       c->maxB, B, (const float2*)c->xh, c->Pf, (float*)c->Hm, c->fs, (float2*)c->G, c->K);     \
    break;
    X(16) X(32) X(48) X(64) X(80) X(96) X(112) X(128)
#undef X
#define X(N)                                                                                                  \
  case N:                                                                                                     \
    hipLaunchKernelGGL((k_herk_bf16<N, 16, 2, 64>), dim3(c->Pf, 2), dim3(1024), 0, c->stream, (const float2*)c->Zt, \
                       c->maxB, B, (const float2*)c->xh, c->Pf, (float*)c->Hm, c->fs, (float2*)c->G, c->K);     \
    break;
    X(144) X(160) X(176) X(192) X(208) X(224) X(240) X(256)
#undef X
    default:
      return fail(c, OCSC_E_UNSUPPORTED, "the Cholesky form needs K <= 256");
  }
  LAUNCHED(c);
  if (!c->dstream) {
    // K <= 128: the VALU kernel; two workgroups share a CU.  (The matrix-core
    // kernel, one workgroup per CU for its 122 KB of blocks at K = 100, took
    // 3.18 ms per launch against 2.56 ms: its serial diagonal-block steps are
    // not covered by a second workgroup.)
    if (chol_small(c->K))
      hipLaunchKernelGGL((k_chol_inv_t<false, 512>), dim3(c->Pf), dim3(512), chol_lds(c->K), c->stream,
                         (const float*)c->Hm, (float*)c->Cm, (const double2*)nullptr, (double2*)nullptr, c->K, c->fs,
                         c->rho_d, c->brk);
    else
      hipLaunchKernelGGL((k_chol_inv_t<false, CHOL_NT>), dim3(c->Pf), dim3(CHOL_NT), chol_lds(c->K), c->stream,
                         (const float*)c->Hm, (float*)c->Cm, (const double2*)nullptr, (double2*)nullptr, c->K, c->fs,
                         c->rho_d, c->brk);
    LAUNCHED(c);
    return OCSC_OK;
  }
  // K > 128: block inverses and a Schur complement, chunk by chunk of frequencies
  double2* W = (double2*)c->Wchol;
  for (int f0 = 0; f0 < c->Pf; f0 += c->chol_chunk) {
    const int nf = std::min(c->chol_chunk, c->Pf - f0);
    const size_t bs = (size_t)CB_N * CB_N;
    double2* s0 = W;
    double2* s1 = W + 1 * (size_t)nf * bs;
    double2* s2 = W + 2 * (size_t)nf * bs;
    double2* s3 = W + 3 * (size_t)nf * bs;
    double2* s4 = W + 4 * (size_t)nf * bs;
    const dim3 g(2, 2, nf), gl(3, 1, nf);   // gl: Hermitian results, lower tiles only
    hipLaunchKernelGGL(k_schur_unpack, dim3(3 * 16, nf), dim3(256), 0, c->stream, (const float*)c->Hm, c->fs, c->K,
                       c->rho_d, f0, nf, W);
    hipLaunchKernelGGL((k_chol_inv_mfma<true>), dim3(nf), dim3(CM_NT), cm_lds(CB_N), c->stream,
                       (const float*)nullptr, (float*)nullptr, (const double2*)s0, s1, CB_N, 0, 0.0, c->brk);   // P = A11^-1
    hipLaunchKernelGGL((k_zgemm128<false, false>), g, dim3(256), 0, c->stream, (const double2*)s2,
                       (const double2*)s1, (const double2*)nullptr, s4, 1.0, 0.0);                   // B = A21 P
    hipLaunchKernelGGL((k_zgemm128<false, true, true>), gl, dim3(256), 0, c->stream, (const double2*)s4,
                       (const double2*)s2, (const double2*)s3, s3, -1.0, 1.0);                       // S = A22 - B A21^H
    hipLaunchKernelGGL((k_chol_inv_mfma<true>), dim3(nf), dim3(CM_NT), cm_lds(CB_N), c->stream,
                       (const float*)nullptr, (float*)nullptr, (const double2*)s3, s0, CB_N, 0, 0.0, c->brk);   // Q = S^-1
    hipLaunchKernelGGL((k_zgemm128<false, false>), g, dim3(256), 0, c->stream, (const double2*)s0,
                       (const double2*)s4, (const double2*)nullptr, s2, -1.0, 0.0);                  // C21 = -Q B
    hipLaunchKernelGGL((k_zgemm128<true, false, true>), gl, dim3(256), 0, c->stream, (const double2*)s4,
                       (const double2*)s2, (const double2*)s1, s1, -1.0, 1.0);                       // C11 = P - B^H C21
    const int kt = (c->K + SU_T - 1) / SU_T;
    hipLaunchKernelGGL(k_schur_pack, dim3(kt * kt, nf), dim3(256), 0, c->stream, (const double2*)W, f0, nf, c->K,
                       c->fs, (float*)c->Cm);
    LAUNCHED(c);
  }
  return OCSC_OK;
}

template <typename T>
int keep_history_t(ocsc_ctx* c, int B) {
  ProfScope ps(c, OCSC_KC_OTHER);
  if (!c->chol) {
    hipLaunchKernelGGL((k_hist_herk<T>), dim3(c->Pf), dim3(256), sizeof(cx<T>) * 8 * c->K, c->stream, (T*)c->Hm,
                       (const cx<T>*)c->Zh, B, c->K, c->Pf, c->fs);
    LAUNCHED(c);
  }
  hipLaunchKernelGGL(k_hist_sums, dim3(1), dim3(256), 0, c->stream, c->pend, B * 64,
                     c->pend + (size_t)c->maxB * 64, B * 64, c->hacc, 1.0 / c->P);
  LAUNCHED(c);
  return OCSC_OK;
}

template <typename T>
int surrogate_t(ocsc_ctx* c, const void* D, double* out) {
  int rc = flush_fold<T>(c);   // G must include every accumulated sample
  if (rc) return rc;
  const cx<T>* dsp = (const cx<T>*)c->Dh;
  if (D) {
    rc = launch_rfft2<T>(c, (const T*)D, c->Mh, c->Mw, (long)c->Mh * c->Mw, (cx<T>*)c->Dv, c->Pf, c->K);
    if (rc) return rc;
    dsp = (const cx<T>*)c->Dv;
  }
  {
    ProfScope ps(c, OCSC_KC_OTHER);
    hipLaunchKernelGGL((k_surr_quad<T>), dim3(c->Pf), dim3(256), sizeof(double) * 2 * c->K, c->stream,
                       (const T*)c->Hm, (const cx<T>*)c->G, dsp, c->dpart, c->K, c->Pf, c->Pw, c->fs);
    LAUNCHED(c);
    hipLaunchKernelGGL(k_surr_final, dim3(1), dim3(256), 0, c->stream, c->dpart, c->Pf, c->hacc, c->dres,
                       1.0 / c->P, c->lam);
    LAUNCHED(c);
  }
  HIPX(c, hipMemcpyAsync(out, c->dres, sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPX(c, hipStreamSynchronize(c->stream));
  rc = check_breakdown(c);
  if (rc) return rc;
  if (!std::isfinite(out[0])) return fail(c, OCSC_E_NUMERIC, "surrogate is not finite");
  return OCSC_OK;
}

template <typename T>
int diagnostics_t(ocsc_ctx* c, double* out) {
  const long fsz = (long)c->Mh * c->Mw;
  int rc = launch_rfft2<T>(c, (const T*)c->V, c->Mh, c->Mw, fsz, (cx<T>*)c->Dv, c->Pf, c->K);
  if (rc) return rc;
  rc = launch_irfft2_crop<T>(c, (const cx<T>*)c->Dh, c->Pf, (T*)c->Dexp, c->Mh, c->Mw, fsz, c->K);
  if (rc) return rc;
  {
    ProfScope ps(c, OCSC_KC_OTHER);
    const double invP = 1.0 / c->P;
    hipLaunchKernelGGL((k_wsq<T>), dim3(DIAG_BLOCKS), dim3(256), 0, c->stream, (const cx<T>*)c->Dh,
                       (const cx<T>*)c->Dv, c->dpart, c->K, c->Pf, c->Pw);
    LAUNCHED(c);
    hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(256), 0, c->stream, c->dpart, DIAG_BLOCKS, c->dres, invP, 1);
    LAUNCHED(c);
    hipLaunchKernelGGL((k_wsq<T>), dim3(DIAG_BLOCKS), dim3(256), 0, c->stream, (const cx<T>*)c->Dh,
                       (const cx<T>*)nullptr, c->dpart, c->K, c->Pf, c->Pw);
    LAUNCHED(c);
    hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(256), 0, c->stream, c->dpart, DIAG_BLOCKS, c->dres + 1, invP, 1);
    LAUNCHED(c);
    hipLaunchKernelGGL((k_plane_norm<T>), dim3(c->K), dim3(256), 0, c->stream, (const T*)c->V, (int)fsz,
                       c->dres + 2);
    LAUNCHED(c);
    hipLaunchKernelGGL((k_plane_norm<T>), dim3(c->K), dim3(256), 0, c->stream, (const T*)c->Dexp, (int)fsz,
                       c->dres + 2 + c->K);
    LAUNCHED(c);
  }
  const size_t n = 2 + 2 * (size_t)c->K;
  HIPX(c, hipMemcpyAsync(out, c->dres, sizeof(double) * n, hipMemcpyDeviceToHost, c->stream));
  HIPX(c, hipStreamSynchronize(c->stream));
  rc = check_breakdown(c);
  if (rc) return rc;
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(out[i])) return fail(c, OCSC_E_NUMERIC, "diagnostics are not finite");
  return OCSC_OK;
}

template <typename T>
int init_state_t(ocsc_ctx* c) {
  hipLaunchKernelGGL((k_c_init<T>), dim3(2048), dim3(256), 0, c->stream, (T*)c->Cm, c->K, c->Pf, c->fs,
                     (T)(1.0 / c->rho_d));
  LAUNCHED(c);
  return launch_gamma<T>(c);
}

// Packed [Pf][K][K] reals <-> the internal per-frequency layout of C.
template <typename T>
int cinv_layout_t(ocsc_ctx* c, const void* src, void* dst, int to_internal) {
  hipLaunchKernelGGL((k_cinv_layout<T>), dim3(2048), dim3(256), 0, c->stream, (const T*)src, (T*)dst, c->K, c->Pf,
                     c->fs, to_internal);
  LAUNCHED(c);
  return OCSC_OK;
}

void free_all(ocsc_ctx* c) {
  void** bufs[] = {&c->xh, &c->Dh, &c->gam, &c->S,    &c->Zh,   &c->W,      &c->G,
                   &c->Cm, &c->d,  &c->Th,  &c->rhs,  &c->V,    &c->apart, &c->twH, &c->twW,
                   &c->xh_obj, &c->Hm, &c->Ubuf, &c->Dv, &c->Dexp, (void**)&c->pend, (void**)&c->hacc,
                   (void**)&c->dpart, (void**)&c->dres, &c->Yb, &c->Zt, &c->Wchol, (void**)&c->brk};
  for (void** b : bufs)
    if (*b) {
      (void)hipFree(*b);
      *b = nullptr;
    }
  if (c->obj_part) (void)hipFree(c->obj_part);
  if (c->obj_out) (void)hipFree(c->obj_out);
  c->obj_part = c->obj_out = nullptr;
  for (auto& pe : c->prof_live) {
    (void)hipEventDestroy(pe.a);
    (void)hipEventDestroy(pe.b);
  }
  c->prof_live.clear();
  for (auto e : c->ev_pool) (void)hipEventDestroy(e);
  c->ev_pool.clear();
}

int state_bytes(const ocsc_ctx* c, int which, size_t* out) {
  const size_t sc = 2 * c->sr;
  switch (which) {
    case OCSC_STATE_DICT_HAT:
    case OCSC_STATE_G:
    case OCSC_STATE_THETA: *out = (size_t)c->K * c->Pf * sc; return OCSC_OK;
    case OCSC_STATE_CINV: *out = (size_t)c->Pf * c->K * c->K * c->sr; return OCSC_OK;
    case OCSC_STATE_V: *out = (size_t)c->K * c->Mh * c->Mw * c->sr; return OCSC_OK;
    case OCSC_STATE_ZHAT: *out = (size_t)c->maxB * c->K * c->Pf * sc; return OCSC_OK;
    case OCSC_STATE_XHAT: *out = (size_t)c->maxB * c->Pf * sc; return OCSC_OK;
    case OCSC_STATE_H:
      if (!c->keep_hist) return OCSC_E_INVALID_ARG;
      *out = (size_t)c->Pf * c->K * c->K * c->sr;
      return OCSC_OK;
    case OCSC_STATE_SUMS:
      if (!c->keep_hist) return OCSC_E_INVALID_ARG;
      *out = 2 * sizeof(double);
      return OCSC_OK;
    case OCSC_STATE_RHS:
      if (!c->warm) return OCSC_E_INVALID_ARG;
      *out = (size_t)c->K * c->Pf * sc;
      return OCSC_OK;
    default: return OCSC_E_INVALID_ARG;
  }
}

void* state_ptr(ocsc_ctx* c, int which) {
  switch (which) {
    case OCSC_STATE_DICT_HAT: return c->Dh;
    case OCSC_STATE_G: return c->G;
    case OCSC_STATE_CINV: return c->Cm;
    case OCSC_STATE_V: return c->V;
    case OCSC_STATE_THETA: return c->Th;
    case OCSC_STATE_ZHAT: return c->Zh;
    case OCSC_STATE_XHAT: return c->xh;
    case OCSC_STATE_H: return c->Hm;
    case OCSC_STATE_SUMS: return c->hacc;
    case OCSC_STATE_RHS: return c->rhs;
    default: return nullptr;
  }
}

}  // namespace

// ===================================================================== C ABI
extern "C" {

void ocsc_default_opts(ocsc_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->struct_size = (int32_t)sizeof(ocsc_opts);
  o->iters_code = 10;
  o->iters_dict = 10;
  o->max_batch = 1;
  o->precision = OCSC_FP64;
  o->flags = 0;
  o->rho_dict = 0.0;
  o->stream = nullptr;
}

int ocsc_init(ocsc_ctx** out, int K, int filt_h, int filt_w, int pad_h, int pad_w, double lambda, double rho,
              const ocsc_opts* opts) {
  OCSC_RANGE();
  g_init_error.clear();
  if (!out) return fail(nullptr, OCSC_E_INVALID_ARG, "out is NULL");
  ocsc_opts o;
  ocsc_default_opts(&o);
  if (opts) {
    if (opts->struct_size != (int32_t)sizeof(ocsc_opts))
      return fail(nullptr, OCSC_E_INVALID_ARG, "opts->struct_size does not match this library");
    o = *opts;
  }
  if (K < 1) return fail(nullptr, OCSC_E_INVALID_ARG, "K must be >= 1");
  if (!pow2_in(pad_h, 32, 1024) || !pow2_in(pad_w, 32, 1024))
    return fail(nullptr, OCSC_E_INVALID_ARG, "pad_h and pad_w must be powers of two in [32, 1024]");
  if (filt_h < 1 || filt_w < 1 || filt_h > pad_h || filt_w > pad_w)
    return fail(nullptr, OCSC_E_INVALID_ARG, "need 1 <= filt <= pad");
  if (!(lambda >= 0.0) || !std::isfinite(lambda)) return fail(nullptr, OCSC_E_INVALID_ARG, "lambda must be >= 0");
  if (!(rho > 0.0) || !std::isfinite(rho)) return fail(nullptr, OCSC_E_INVALID_ARG, "rho must be > 0");
  if (o.iters_code < 1 || o.iters_dict < 1) return fail(nullptr, OCSC_E_INVALID_ARG, "iteration counts must be >= 1");
  if (o.max_batch < 1 || o.max_batch > 65535) return fail(nullptr, OCSC_E_INVALID_ARG, "max_batch must be in [1, 65535]");
  if (o.precision != OCSC_FP64 && o.precision != OCSC_FP32)
    return fail(nullptr, OCSC_E_INVALID_ARG, "unknown precision");
  if (o.flags & ~(OCSC_FLAG_OWN_STREAM | OCSC_FLAG_KEEP_HISTORY | OCSC_FLAG_WARM_START | OCSC_FLAG_CHOLESKY |
                  OCSC_FLAG_REFINE))
    return fail(nullptr, OCSC_E_INVALID_ARG, "unknown bits in opts->flags");
  if ((o.flags & OCSC_FLAG_REFINE) && !(o.flags & OCSC_FLAG_CHOLESKY))
    return fail(nullptr, OCSC_E_UNSUPPORTED, "OCSC_FLAG_REFINE needs OCSC_FLAG_CHOLESKY");
  if ((o.flags & OCSC_FLAG_CHOLESKY) &&
      (o.precision != OCSC_FP32 || K > 256 || (o.flags & OCSC_FLAG_WARM_START)))
    return fail(nullptr, OCSC_E_UNSUPPORTED, "the Cholesky form needs an FP32 context, K <= 256 and a cold start");
  // K > 128 runs only in the Cholesky form: its D-step streams C_p instead of holding it in LDS
  const bool dstream = (o.flags & OCSC_FLAG_CHOLESKY) && K > 128;
  if (!std::isfinite(o.rho_dict)) return fail(nullptr, OCSC_E_INVALID_ARG, "rho_dict must be finite");
  if (big_grid(pad_h, pad_w) && !((pad_h == 256 || pad_h == 512) && (pad_w == 256 || pad_w == 512)))
    return fail(nullptr, OCSC_E_UNSUPPORTED,
                "plane kernels exist for grids with both sides <= 128 or both sides in {256, 512}");
  if (big_grid(pad_h, pad_w) && (size_t)o.max_batch * K > 65535)
    return fail(nullptr, OCSC_E_UNSUPPORTED, "max_batch * K must be <= 65535 on grids above 128");
  const size_t sr = o.precision == OCSC_FP64 ? 8 : 4;
  // D-step sweep: C_p (K rows of pitch K+1) must fit in LDS; a slot of fpb
  // frequencies must fit the prefetch registers (256 threads x SWEEP_MAXV x 16 B,
  // or SWEEP_MAXV_L vectors for a single frequency)
  const int vr = (int)(16 / sr);
  const int fs = (K * (K + 1) + vr - 1) / vr * vr;
  int fpb = 1;
  while (fpb < 16 && 256 / (fpb * 2) >= K) fpb *= 2;
  auto sweep_bytes = [&](int f) { return sweep_lds_bytes(K, f, fs, (int)sr, sweep_nvm_for(K, f, sr)); };
  const size_t max_lds = 160 * 1024 - 1024;
  const size_t max_slot = (size_t)256 * SWEEP_MAXV * 16;
  if (!dstream && K > 128)
    return fail(nullptr, OCSC_E_UNSUPPORTED, "K > 128 needs the Cholesky form (FP32, K <= 256)");
  if (!dstream && (sweep_bytes(1) > max_lds || sweep_slot_bytes(K, 1, sr) > (size_t)256 * SWEEP_MAXV_L * 16 ||
                   sweep_plain_lds_bytes(K, 1, fs, (int)sr, sweep_nvm_for(K, 1, sr), 1) > max_lds))
    return fail(nullptr, OCSC_E_UNSUPPORTED,
                "K too large for the LDS-resident D-step of this precision (FP64: K <= 92; FP32: K <= 128)");
  while (fpb > 1 && (sweep_bytes(fpb) > 64 * 1024 || (size_t)fpb * fs * sr > max_slot)) fpb /= 2;

  ocsc_ctx* c = new (std::nothrow) ocsc_ctx();
  if (!c) return fail(nullptr, OCSC_E_OOM, "host allocation failed");
  c->K = K; c->Mh = filt_h; c->Mw = filt_w; c->Ph = pad_h; c->Pw = pad_w;
  c->Wc = pad_w / 2 + 1; c->Pf = pad_h * c->Wc; c->P = pad_h * pad_w;
  c->lam = lambda; c->rho = rho;
  c->rho_d = o.rho_dict > 0 ? o.rho_dict : rho * c->P;
  c->Jz = o.iters_code; c->Jd = o.iters_dict; c->maxB = o.max_batch; c->prec = o.precision;
  c->sr = sr;
  const int vb = sr == 8 ? vblock<double>() : vblock<float>();
  c->nvb = (c->Wc + vb - 1) / vb;
  c->fpb = fpb;
  c->fs = fs;
  c->sweep_smem = sweep_bytes(fpb);
  {
    // One round of workgroups over the chip.  A fold sweep deals its slots
    // out round by round to as many workgroups as fit at once.  A plain sweep
    // gives each workgroup a run of slots and holds the run's right-hand
    // sides in LDS; it runs at most two workgroups per CU with runs half as
    // long again (K=100: 490 workgroups of 17 slots took 57 us per sweep
    // against 64 us for 757 of 11), and the run length is capped by what
    // fits in LDS.
    const int nslots = (c->Pf + fpb - 1) / fpb;
    const int nvm = sweep_nvm_for(K, fpb, sr);
    const size_t plain0 = sweep_plain_lds_bytes(K, fpb, fs, (int)sr, nvm, 0);
    const size_t per_slot = (size_t)fpb * K * 2 * sr;
    const int occ_fold = std::max(1, std::min(8, (int)((160 * 1024) / (c->sweep_smem + 64))));   // + static LDS
    c->fold_wgs = std::min(nslots, 256 * occ_fold);
    int occ = (int)((160 * 1024) / (std::max(c->sweep_smem, plain0 + per_slot) + 64));
    occ = occ < 1 ? 1 : (occ > 2 ? 2 : occ);
    const size_t budget = (size_t)(160 * 1024) / occ - 64;
    int spw = (nslots + 256 * occ - 1) / (256 * occ);
    const int spw_max = (int)((budget - plain0) / per_slot);
    if (spw > spw_max) spw = spw_max;
    c->slots_per_wg = spw;
    c->sweep_wgs = (nslots + spw - 1) / spw;
    c->plain_smem = plain0 + (size_t)spw * per_slot;
  }
  c->vapply_smem = (((size_t)filt_h * filt_w * sr + 15) & ~(size_t)15) + (size_t)filt_h * vb * 2 * sr;
  c->big = big_grid(pad_h, pad_w);
  c->tune.plane_threads = c->big ? 256 : plane_threads(pad_h, pad_w);
  c->tune.zstep_freqs = 16;
  c->tune.zstep_samples = 1;
  c->tune.col_bytes = 128;
  c->tune.row_block = BIG_RB;
  c->tune.chunk_samples = 0;
  c->tune.two_pass = c->big ? 1 : 0;
  c->chol = (o.flags & OCSC_FLAG_CHOLESKY) != 0;
  c->dstream = dstream;
  c->chol_chunk = dstream ? std::min(c->Pf, 2048) : 0;
  c->keep_hist = (o.flags & OCSC_FLAG_KEEP_HISTORY) != 0 || c->chol;
  c->warm = (o.flags & OCSC_FLAG_WARM_START) != 0;
  c->refine = (o.flags & OCSC_FLAG_REFINE) != 0;
  c->vstep_fused = sr == 8 ? vstep_fused_ok<double>(pad_h, pad_w, filt_h, filt_w)
                           : vstep_fused_ok<float>(pad_h, pad_w, filt_h, filt_w);

  auto bail = [&](int code, const std::string& m) {
    g_init_error = m;
    free_all(c);
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
    return code;
  };
  hipError_t e = hipGetDevice(&c->device);
  if (e != hipSuccess) return bail(OCSC_E_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
  {
    // the static scratch's address on this device, looked up once per device
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (c->device < 0 || c->device >= kMaxDevices) return bail(OCSC_E_UNSUPPORTED, "device index above 63");
    if (!g_scratch_dev[c->device]) {
      void* addr = nullptr;
      e = hipGetSymbolAddress(&addr, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !addr)
        return bail(OCSC_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
      g_scratch_dev[c->device] = addr;
    }
    c->scratch = g_scratch_dev[c->device];
  }
  if (!(o.flags & OCSC_FLAG_OWN_STREAM)) {
    c->stream = (hipStream_t)o.stream;
  } else {
    e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
    if (e != hipSuccess) return bail(OCSC_E_HIP, std::string("hipStreamCreate: ") + hipGetErrorString(e));
    c->own_stream = true;
  }
  if (c->chol) {
    const int kb = c->dstream ? CB_N : K;   // the factorised block size
    const void* fn = c->dstream ? (const void*)k_chol_inv_mfma<true>
                                : (chol_small(K) ? (const void*)k_chol_inv_t<false, 512>
                                                 : (const void*)k_chol_inv_t<false, CHOL_NT>);
    e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)(c->dstream ? cm_lds(kb) : chol_lds(kb)));
    if (e != hipSuccess) return bail(OCSC_E_HIP, std::string("hipFuncSetAttribute: ") + hipGetErrorString(e));
  }
  if (!c->dstream && std::max(c->sweep_smem, c->plain_smem) > 64 * 1024) {
#define M3(T, KT, FPB) \
  (const void*)k_dict_sweep<T, KT, FPB, 0>, (const void*)k_dict_sweep<T, KT, FPB, 1>, (const void*)k_dict_sweep<T, KT, FPB, 2>
    const void* fns[] = {M3(double, 0, 0), M3(float, 0, 0), M3(double, -1, 0), M3(float, -1, 0)
#define X(T, KT, FPB) , M3(T, KT, FPB)
                         OCSC_SWEEP_SPECS(X)
#undef X
    };
#undef M3
    for (const void* fn : fns) {
      e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)std::max(c->sweep_smem, c->plain_smem));
      if (e != hipSuccess) return bail(OCSC_E_HIP, std::string("hipFuncSetAttribute: ") + hipGetErrorString(e));
    }
  }

  if (!c->dstream && sr == 4 && c->maxB > 1) {
    const void* fn = nullptr;
#define X(KP) \
    if ((K + 15) / 16 * 16 == KP) fn = (const void*)k_fold_mfma<KP>;
    OCSC_FOLD_KP(X)
#undef X
    if (fn) {
      e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)fold_mfma_lds(K, c->fs));
      if (e != hipSuccess) return bail(OCSC_E_HIP, std::string("hipFuncSetAttribute: ") + hipGetErrorString(e));
    }
  }

  const size_t sc = 2 * sr, K_ = K, Pf = c->Pf, B = c->maxB;
  c->obj_nr = (c->Pf + 255) / 256;
  c->obj_nl = 64;
  struct { void** p; size_t n; } allocs[] = {
      {&c->xh, B * Pf * sc},        {&c->Dh, K_ * Pf * sc},          {&c->gam, Pf * sr},
      {&c->S, B * K_ * Pf * sc},       {&c->Zh, B * K_ * Pf * sc},
      {&c->W, B * K_ * c->P * sr},  {&c->G, K_ * Pf * sc},           {&c->Cm, Pf * (size_t)c->fs * sr},
      {&c->d, K_ * Pf * sc},        {&c->Th, K_ * Pf * sc},          {&c->rhs, K_ * Pf * sc},
      {&c->V, K_ * filt_h * filt_w * sr},
      {&c->apart, K_ * c->nvb * filt_h * filt_w * sr},
      {&c->twH, (size_t)pad_h * sc}, {&c->twW, (size_t)pad_w * sc}, {&c->xh_obj, B * Pf * sc},
      {(void**)&c->obj_part, B * (size_t)(c->obj_nr + c->obj_nl) * sizeof(double)},
      {(void**)&c->obj_out, 2 * B * sizeof(double)},
      {&c->Dv, K_ * Pf * sc},       {&c->Dexp, K_ * filt_h * filt_w * sr},
      {(void**)&c->dpart, (size_t)std::max<int>(c->Pf, DIAG_BLOCKS) * sizeof(double)},
      {(void**)&c->dres, (2 + 2 * K_) * sizeof(double)},
      {(void**)&c->hacc, 2 * sizeof(double)},
      {&c->Hm, c->keep_hist ? Pf * (size_t)c->fs * sr : 0},
      {&c->Ubuf, c->keep_hist ? B * K_ * c->P * sr : 0},
      {(void**)&c->pend, c->keep_hist ? 2 * B * 64 * sizeof(double) : 0},
      {&c->Yb, c->big ? B * K_ * Pf * sc : 0},
      {&c->Zt, (c->chol || B > 1) ? Pf * B * K_ * sc : 0},
      {&c->Wchol, c->dstream ? (size_t)5 * c->chol_chunk * CB_N * CB_N * 16 : 0},
      {(void**)&c->brk, c->chol ? sizeof(int) : 0}};
  for (auto& a : allocs) {
    if (a.n == 0) continue;
    e = hipMalloc(a.p, a.n);
    if (e != hipSuccess) return bail(OCSC_E_OOM, std::string("hipMalloc: ") + hipGetErrorString(e));
    e = hipMemsetAsync(*a.p, 0, a.n, c->stream);
    if (e != hipSuccess) return bail(OCSC_E_HIP, std::string("hipMemsetAsync: ") + hipGetErrorString(e));
  }
  // twiddle tables e^{-2 pi i j / N}, computed in double
  {
    std::vector<double> h(2 * (size_t)std::max(pad_h, pad_w));
    auto upload = [&](void* dst, int N) -> hipError_t {
      for (int j = 0; j < N; ++j) {
        const double a = 2.0 * M_PI * (double)j / (double)N;
        h[2 * j] = std::cos(a);
        h[2 * j + 1] = -std::sin(a);
      }
      if (sr == 8) return hipMemcpy(dst, h.data(), (size_t)N * 16, hipMemcpyHostToDevice);
      std::vector<float> f(2 * (size_t)N);
      for (int j = 0; j < 2 * N; ++j) f[j] = (float)h[j];
      return hipMemcpy(dst, f.data(), (size_t)N * 8, hipMemcpyHostToDevice);
    };
    e = upload(c->twH, pad_h);
    if (e == hipSuccess) e = upload(c->twW, pad_w);
    if (e != hipSuccess) return bail(OCSC_E_HIP, std::string("twiddle upload: ") + hipGetErrorString(e));
  }
  int rc = sr == 8 ? init_state_t<double>(c) : init_state_t<float>(c);
  if (rc) return bail(rc, c->err);
  e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return bail(OCSC_E_HIP, std::string("init sync: ") + hipGetErrorString(e));
  *out = c;
  return OCSC_OK;
}

int ocsc_destroy(ocsc_ctx* c) {
  OCSC_RANGE();
  if (!c) return OCSC_OK;
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  free_all(c);
  if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
  delete c;
  return OCSC_OK;
}

int ocsc_set_dictionary(ocsc_ctx* c, const void* D) {
  OCSC_RANGE();
  if (!c) return OCSC_E_INVALID_ARG;
  if (!D) return fail(c, OCSC_E_INVALID_ARG, "D_dev is NULL");
  const long fs = (long)c->Mh * c->Mw;
  int rc = c->sr == 8
               ? launch_rfft2<double>(c, (const double*)D, c->Mh, c->Mw, fs, (cx<double>*)c->Dh, c->Pf, c->K)
               : launch_rfft2<float>(c, (const float*)D, c->Mh, c->Mw, fs, (cx<float>*)c->Dh, c->Pf, c->K);
  if (rc) return rc;
  return c->sr == 8 ? launch_gamma<double>(c) : launch_gamma<float>(c);
}

int ocsc_get_dictionary(ocsc_ctx* c, void* D) {
  OCSC_RANGE();
  if (!c) return OCSC_E_INVALID_ARG;
  if (!D) return fail(c, OCSC_E_INVALID_ARG, "D_dev_out is NULL");
  const long fs = (long)c->Mh * c->Mw;
  return c->sr == 8 ? launch_irfft2_crop<double>(c, (const cx<double>*)c->Dh, c->Pf, (double*)D, c->Mh, c->Mw, fs, c->K)
                    : launch_irfft2_crop<float>(c, (const cx<float>*)c->Dh, c->Pf, (float*)D, c->Mh, c->Mw, fs, c->K);
}

int ocsc_code_update(ocsc_ctx* c, const void* x, int B, void* codes) {
  OCSC_RANGE();
  if (!c) return OCSC_E_INVALID_ARG;
  if (!x) return fail(c, OCSC_E_INVALID_ARG, "x_dev is NULL");
  if (((uintptr_t)x | (uintptr_t)codes) & 15) return fail(c, OCSC_E_INVALID_ARG, "buffers must be 16-byte aligned");
  if (B < 1 || B > c->maxB) return fail(c, OCSC_E_INVALID_ARG, "B must be in [1, max_batch]");
  return c->sr == 8 ? code_update_t<double>(c, x, B, codes, 0) : code_update_t<float>(c, x, B, codes, 0);
}

int ocsc_code_update_group(ocsc_ctx* const* ctxs, const void* const* xs, const int* Bs, void* const* codes, int n) {
  OCSC_RANGE();
  if (!ctxs || !xs || !Bs || n < 1 || n > CG_MAX)
    return fail(nullptr, OCSC_E_INVALID_ARG, "need 1 <= n <= 8 contexts, samples and batch sizes");
  ocsc_ctx* c0 = ctxs[0];
  if (!c0) return fail(nullptr, OCSC_E_INVALID_ARG, "NULL context");
  for (int s = 0; s < n; ++s) {
    ocsc_ctx* c = ctxs[s];
    if (!c) return fail(c0, OCSC_E_INVALID_ARG, "NULL context");
    for (int r = 0; r < s; ++r)
      if (ctxs[r] == c) return fail(c0, OCSC_E_INVALID_ARG, "a context is listed twice");
    if (c->sr != c0->sr || c->Jz != c0->Jz || c->device != c0->device)
      return fail(c0, OCSC_E_INVALID_ARG, "contexts differ in precision, iters_code or device");
    if (!xs[s]) return fail(c0, OCSC_E_INVALID_ARG, "x_dev is NULL");
    void* cd = codes ? codes[s] : nullptr;
    if (((uintptr_t)xs[s] | (uintptr_t)cd) & 15) return fail(c0, OCSC_E_INVALID_ARG, "buffers must be 16-byte aligned");
    if (Bs[s] < 1 || Bs[s] > c->maxB) return fail(c0, OCSC_E_INVALID_ARG, "B must be in [1, max_batch]");
  }
  for (int s = 0; s < n; ++s)
    if (ctxs[s]->K > 128) return fail(c0, OCSC_E_UNSUPPORTED, "the grouped code launch supports K <= 128");
  int coop = 0;
  HIPX(c0, hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, c0->device));
  if (!coop) return fail(c0, OCSC_E_UNSUPPORTED, "the device has no cooperative launch");
  StreamJoin join(ctxs, n);
  hipError_t err = join.enter();
  if (err != hipSuccess) return fail(c0, OCSC_E_HIP, std::string("stream ordering: ") + hipGetErrorString(err));
  const int rc = c0->sr == 8 ? code_group_t<double>(ctxs, xs, Bs, codes, n) : code_group_t<float>(ctxs, xs, Bs, codes, n);
  err = join.leave();
  if (rc) return rc;
  if (err != hipSuccess) return fail(c0, OCSC_E_HIP, std::string("stream ordering: ") + hipGetErrorString(err));
  return OCSC_OK;
}

int ocsc_code_append(ocsc_ctx* c, const void* x, int B, void* codes) {
  OCSC_RANGE();
  if (!c) return OCSC_E_INVALID_ARG;
  if (!x) return fail(c, OCSC_E_INVALID_ARG, "x_dev is NULL");
  if (((uintptr_t)x | (uintptr_t)codes) & 15) return fail(c, OCSC_E_INVALID_ARG, "buffers must be 16-byte aligned");
  if (B < 1 || c->pending_B + B > c->maxB)
    return fail(c, OCSC_E_INVALID_ARG, "B must be >= 1 and the pending samples must fit max_batch");
  const int off = c->pending_B;
  return c->sr == 8 ? code_update_t<double>(c, x, B, codes, off) : code_update_t<float>(c, x, B, codes, off);
}

int ocsc_history_accumulate(ocsc_ctx* c) {
  OCSC_RANGE();
  if (!c) return OCSC_E_INVALID_ARG;
  if (c->pending_B == 0) return fail(c, OCSC_E_STATE, "no coded samples to accumulate");
  if (c->keep_hist) {
    int rc = c->sr == 8 ? keep_history_t<double>(c, c->pending_B) : keep_history_t<float>(c, c->pending_B);
    if (rc) return rc;
  }
  if (c->chol) {
    // G, H and C are updated now; there is no Sherman-Morrison fold to defer
    int rc = chol_history(c, c->pending_B);
    if (rc) return rc;
    c->fold_B = 0;
  } else {
    c->fold_B = c->pending_B;
  }
  c->t += c->pending_B;
  c->pending_B = 0;
  return OCSC_OK;
}

int ocsc_dict_update(ocsc_ctx* c) {
  OCSC_RANGE();
  if (!c) return OCSC_E_INVALID_ARG;
  if (c->t == 0) return fail(c, OCSC_E_STATE, "dict_update needs at least one accumulated sample");
  return c->sr == 8 ? dict_update_t<double>(c) : dict_update_t<float>(c);
}

int ocsc_dict_update_group(ocsc_ctx* const* ctxs, int n) {
  OCSC_RANGE();
  if (!ctxs || n < 1 || n > GROUP_MAX) return fail(nullptr, OCSC_E_INVALID_ARG, "need 1 <= n <= 8 contexts");
  ocsc_ctx* c0 = ctxs[0];
  if (!c0) return fail(nullptr, OCSC_E_INVALID_ARG, "NULL context");
  for (int s = 0; s < n; ++s) {
    ocsc_ctx* c = ctxs[s];
    if (!c) return fail(c0, OCSC_E_INVALID_ARG, "NULL context");
    for (int r = 0; r < s; ++r)
      if (ctxs[r] == c) return fail(c0, OCSC_E_INVALID_ARG, "a context is listed twice");
    if (c->K != c0->K || c->Mh != c0->Mh || c->Mw != c0->Mw || c->sr != c0->sr || c->Jd != c0->Jd ||
        c->device != c0->device)
      return fail(c0, OCSC_E_INVALID_ARG, "contexts differ in K, filter size, precision, iters_dict or device");
  }
  for (int s = 0; s < n; ++s) {
    if (ctxs[s]->warm) return fail(c0, OCSC_E_UNSUPPORTED, "the shared dictionary update starts cold");
    if (ctxs[s]->t == 0) return fail(c0, OCSC_E_STATE, "every context needs at least one accumulated sample");
  }
  // run on the first context's stream, after every member's earlier work
  StreamJoin join(ctxs, n);
  hipError_t err = join.enter();
  if (err != hipSuccess) return fail(c0, OCSC_E_HIP, std::string("stream ordering: ") + hipGetErrorString(err));
  for (int s = 0; s < n; ++s) ctxs[s]->pending_B = 0;
  const int rc = c0->sr == 8 ? dict_update_group_t<double>(ctxs, n) : dict_update_group_t<float>(ctxs, n);
  // later work on every member's stream waits for the update
  err = join.leave();
  if (rc) return rc;
  if (err != hipSuccess) return fail(c0, OCSC_E_HIP, std::string("stream ordering: ") + hipGetErrorString(err));
  return OCSC_OK;
}

int ocsc_objective(ocsc_ctx* c, const void* x, const void* codes, int B, double* out) {
  OCSC_RANGE();
  if (!c) return OCSC_E_INVALID_ARG;
  if (!x || !codes || !out) return fail(c, OCSC_E_INVALID_ARG, "NULL buffer");
  if (((uintptr_t)x | (uintptr_t)codes) & 15) return fail(c, OCSC_E_INVALID_ARG, "buffers must be 16-byte aligned");
  if (B < 1 || B > c->maxB) return fail(c, OCSC_E_INVALID_ARG, "B must be in [1, max_batch]");
  return c->sr == 8 ? objective_t<double>(c, x, codes, B, out, 0) : objective_t<float>(c, x, codes, B, out, 0);
}

int ocsc_objective_terms(ocsc_ctx* c, const void* x, const void* codes, int B, double* out) {
  OCSC_RANGE();
  if (!c) return OCSC_E_INVALID_ARG;
  if (!x || !codes || !out) return fail(c, OCSC_E_INVALID_ARG, "NULL buffer");
  if (((uintptr_t)x | (uintptr_t)codes) & 15) return fail(c, OCSC_E_INVALID_ARG, "buffers must be 16-byte aligned");
  if (B < 1 || B > c->maxB) return fail(c, OCSC_E_INVALID_ARG, "B must be in [1, max_batch]");
  return c->sr == 8 ? objective_t<double>(c, x, codes, B, out, 1) : objective_t<float>(c, x, codes, B, out, 1);
}

int ocsc_objective_noalloc(ocsc_ctx* c, const void* x, const void* codes, int B, double* out_dev) {
  OCSC_RANGE();
  if (!c) return OCSC_E_INVALID_ARG;
  if (!x || !codes || !out_dev) return fail(c, OCSC_E_INVALID_ARG, "NULL buffer");
  if (((uintptr_t)x | (uintptr_t)codes) & 15) return fail(c, OCSC_E_INVALID_ARG, "buffers must be 16-byte aligned");
  if ((uintptr_t)out_dev & 7) return fail(c, OCSC_E_INVALID_ARG, "out_dev must be 8-byte aligned");
  if (B < 1 || B > 65535) return fail(c, OCSC_E_INVALID_ARG, "B must be in [1, 65535]");
  if (noalloc_objective_bytes(c, B) > (size_t)OCSC_NOALLOC_SCRATCH_BYTES)
    return fail(c, OCSC_E_INVALID_ARG,
                "B (K + 1) spectra and the partial sums exceed the static scratch (OCSC_NOALLOC_SCRATCH_BYTES)");
  if (!c->scratch) return fail(c, OCSC_E_HIP, "no scratch address for this device");
  // no kernel timing here: timing events are created on demand
  const unsigned mask = c->prof_mask;
  c->prof_mask = 0;
  const int rc = c->sr == 8 ? objective_noalloc_t<double>(c, x, codes, B, out_dev)
                            : objective_noalloc_t<float>(c, x, codes, B, out_dev);
  c->prof_mask = mask;
  return rc;
}

int ocsc_surrogate(ocsc_ctx* c, const void* D, double* out) {
  OCSC_RANGE();
  if (!c) return OCSC_E_INVALID_ARG;
  if (!out) return fail(c, OCSC_E_INVALID_ARG, "out_host is NULL");
  if ((uintptr_t)D & 15) return fail(c, OCSC_E_INVALID_ARG, "buffers must be 16-byte aligned");
  if (!c->keep_hist) return fail(c, OCSC_E_STATE, "the surrogate needs a context created with OCSC_FLAG_KEEP_HISTORY");
  return c->sr == 8 ? surrogate_t<double>(c, D, out) : surrogate_t<float>(c, D, out);
}

int ocsc_diagnostics(ocsc_ctx* c, double* out) {
  OCSC_RANGE();
  if (!c) return OCSC_E_INVALID_ARG;
  if (!out) return fail(c, OCSC_E_INVALID_ARG, "out_host is NULL");
  return c->sr == 8 ? diagnostics_t<double>(c, out) : diagnostics_t<float>(c, out);
}

// ---------------------------------------------------------------- graphs
}  // extern "C"

namespace {

bool tuning_valid(const ocsc_ctx* c, const ocsc_tuning& t) {
  const bool pt = (c->big && t.two_pass != 2) ? t.plane_threads == 256 : plane_nt_ok(c->Ph, c->Pw, t.plane_threads);
  const bool zf = t.zstep_freqs == 16 || t.zstep_freqs == 32 || t.zstep_freqs == 64;
  const bool sb = t.zstep_samples == 1 || t.zstep_samples == 2 || t.zstep_samples == 4;
  const bool cb = (t.col_bytes == 128 || t.col_bytes == 256 || t.col_bytes == 512) &&
                  (long)c->Ph * t.col_bytes <= 131072;
  const bool rb = t.row_block == 4 || t.row_block == 8 || t.row_block == 16;
  const bool ch = t.chunk_samples == 0 || t.chunk_samples == 1 || t.chunk_samples == 2 || t.chunk_samples == 4 ||
                  t.chunk_samples == 8 || t.chunk_samples == 16;
  const bool tp = c->big ? (t.two_pass == 1 || t.two_pass == 2)
                         : (t.two_pass == 0 || t.two_pass == 2 || (t.two_pass == 1 && two_pass_capable(c->Ph, c->Pw)));
  return pt && zf && sb && cb && rb && ch && tp;
}

// The column-pass output of the two-pass code-plane step, allocated when a
// one-pass grid first selects that step.
int ensure_column_buffer(ocsc_ctx* c) {
  if (c->Yb) return OCSC_OK;
  const size_t bytes = (size_t)c->maxB * c->K * c->Pf * 2 * c->sr;
  hipError_t e = hipMalloc(&c->Yb, bytes);
  if (e != hipSuccess) {
    c->Yb = nullptr;
    (void)hipGetLastError();
    return fail(c, OCSC_E_OOM, std::string("column buffer: ") + hipGetErrorString(e));
  }
  return OCSC_OK;
}

struct EventPair {
  hipEvent_t a = nullptr, b = nullptr;
  ~EventPair() {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
  }
};

// Mean duration of `reps` launches after one untimed launch.
template <typename F>
int time_launches(ocsc_ctx* c, EventPair& ev, F&& launch, int reps, double* ms_out) {
  int rc = launch();
  if (rc) return rc;
  HIPX(c, hipEventRecord(ev.a, c->stream));
  for (int r = 0; r < reps; ++r) {
    rc = launch();
    if (rc) return rc;
  }
  HIPX(c, hipEventRecord(ev.b, c->stream));
  HIPX(c, hipEventSynchronize(ev.b));
  float ms = 0;
  HIPX(c, hipEventElapsedTime(&ms, ev.a, ev.b));
  *ms_out = ms / reps;
  return OCSC_OK;
}

// Try every launch shape of the Z-step and of the plane kernel on the code
// workspace (samples [0, B)) and keep the fastest of each.  The Z-step runs
// as a middle iteration (reads S) and the plane kernel as a middle iteration
// (reads and writes W, writes S); the values in the workspace are irrelevant
// to the timing.
template <typename T>
int autotune_t(ocsc_ctx* c, int B, double* best_ms) {
  int rc = flush_fold<T>(c);
  if (rc) return rc;
  EventPair ev;
  HIPX(c, hipEventCreate(&ev.a));
  HIPX(c, hipEventCreate(&ev.b));
  const unsigned mask = c->prof_mask;
  c->prof_mask = 0;
  const ocsc_tuning start = c->tune;
  ocsc_tuning best = start;
  double best_z = 1e30, best_p = 1e30;
  constexpr int REPS = 3;
  // Z-step tiles; tp = 2: the Z-step of the split plane step (it forms its
  // input from two half-height spectra)
  auto tune_zstep = [&](int tp, ocsc_tuning& into, double& ms_best) {
    for (int zf : {16, 32, 64}) {
      for (int sb : {1, 2, 4}) {
        c->tune = start;
        c->tune.two_pass = tp;
        c->tune.zstep_freqs = zf;
        c->tune.zstep_samples = sb;
        double ms = 0;
        rc = time_launches(c, ev, [&] { return launch_zstep<T>(c, 0, B, 0, false); }, REPS, &ms);
        if (rc) return;
        if (ms < ms_best) {
          ms_best = ms;
          into.zstep_freqs = zf;
          into.zstep_samples = sb;
        }
      }
    }
  };
  tune_zstep(c->big ? 1 : 0, best, best_z);
  c->tune = start;
  if (c->tune.two_pass == 2) c->tune.two_pass = c->big ? 1 : 0;
  // plane step: workgroup size of the one-pass kernel, or column block x row
  // block of the two-pass kernels (two-pass grids, and 64 x 64 / 128 x 128
  // grids as an alternative)
  if (two_pass_capable(c->Ph, c->Pw)) rc = ensure_column_buffer(c);
  for (int tp = 0; tp < 2 && !rc; ++tp) {
    for (int nt : {256, 512, 1024}) {
      for (int cby : {128, 256, 512}) {
        for (int rb : {4, 8, 16}) {
          if (rc) break;
          // a one-pass shape varies the workgroup size only, a two-pass one the blocks only
          if (tp == 0 && (cby != start.col_bytes || rb != start.row_block)) continue;
          if (tp == 1 && nt != 256) continue;
          c->tune.two_pass = tp;
          c->tune.plane_threads = nt;
          c->tune.col_bytes = cby;
          c->tune.row_block = rb;
          if (!tuning_valid(c, c->tune)) continue;
          double ms = 0;
          rc = time_launches(c, ev, [&] { return launch_code_plane<T>(c, 0, B * c->K, nullptr, 0, 0); }, REPS, &ms);
          if (rc) break;
          if (ms < best_p) {
            best_p = ms;
            best.two_pass = tp;
            best.plane_threads = nt;
            best.col_bytes = cby;
            best.row_block = rb;
          }
        }
      }
    }
  }
  // split planes, with the Z-step tile chosen for them: kept if the Z-step
  // and plane step together beat the unsplit pair
  if (!rc) {
    ocsc_tuning split = best;
    split.two_pass = 2;
    double sz = 1e30, sp = 1e30;
    tune_zstep(2, split, sz);
    for (int nt : {256, 512, 1024}) {
      if (rc) break;
      ocsc_tuning t = split;
      t.plane_threads = nt;
      if (!tuning_valid(c, t)) continue;
      c->tune = t;
      double ms = 0;
      rc = time_launches(c, ev, [&] { return launch_code_plane<T>(c, 0, B * c->K, nullptr, 0, 0); }, REPS, &ms);
      if (rc) break;
      if (ms < sp) {
        sp = ms;
        split.plane_threads = nt;
      }
    }
    if (!rc && sz + sp < best_z + best_p) {
      best = split;
      best_z = sz;
      best_p = sp;
    }
  }
  // sample groups: whole code updates (all iterations) with the chosen kernel shapes
  double best_c = 1e30;
  c->tune = best;
  for (int ch : {0, 1, 2, 4, 8, 16}) {
    if (rc) break;
    if (ch >= B) continue;
    c->tune.chunk_samples = ch;
    double ms = 0;
    rc = time_launches(c, ev, [&] { return code_iterations<T>(c, 0, B, (T*)nullptr); }, 2, &ms);
    if (rc) break;
    if (ms < best_c * 0.98 || ch == 0) {   // a group size must win by 2% over the whole batch
      best_c = ms;
      best.chunk_samples = ch;
    }
  }
  c->prof_mask = mask;
  c->tune = rc ? start : best;
  if (rc) return rc;
  *best_ms = best_z + best_p;
  return OCSC_OK;
}

}  // namespace

struct ocsc_graph {
  ocsc_ctx* c = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int B = 0;
};

extern "C" {

int ocsc_graph_create(ocsc_ctx* c, const void* x, int B, void* codes, ocsc_graph** out) {
  OCSC_RANGE();
  if (!c) return OCSC_E_INVALID_ARG;
  if (!x || !out) return fail(c, OCSC_E_INVALID_ARG, "NULL buffer");
  if (((uintptr_t)x | (uintptr_t)codes) & 15) return fail(c, OCSC_E_INVALID_ARG, "buffers must be 16-byte aligned");
  if (B < 1 || B > c->maxB) return fail(c, OCSC_E_INVALID_ARG, "B must be in [1, max_batch]");
  if (!c->stream) return fail(c, OCSC_E_UNSUPPORTED, "graph capture needs a context on a non-default stream");
  if (c->pending_B || c->fold_B) return fail(c, OCSC_E_STATE, "graph capture needs no pending codes and no deferred fold");
  ocsc_graph* gr = new (std::nothrow) ocsc_graph();
  if (!gr) return fail(c, OCSC_E_OOM, "host allocation failed");
  gr->c = c;
  gr->B = B;
  // Two steps: each dictionary update swaps the dictionary and D-step buffers,
  // so after two the buffers (and the sweep directions, J_d sweeps per step)
  // are where they started and the same graph can be replayed.
  const unsigned mask = c->prof_mask;
  const int64_t t0 = c->t;
  const unsigned sc0 = c->sweep_count;
  c->prof_mask = 0;
  hipError_t e = hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal);
  int rc = e == hipSuccess ? OCSC_OK : fail(c, OCSC_E_HIP, std::string("hipStreamBeginCapture: ") + hipGetErrorString(e));
  const size_t xs = (size_t)B * c->P * c->sr, us = (size_t)B * c->K * c->P * c->sr;
  for (int s = 0; s < 2 && rc == OCSC_OK; ++s) {
    rc = ocsc_code_update(c, (const char*)x + s * xs, B, codes ? (char*)codes + s * us : nullptr);
    if (rc == OCSC_OK) rc = ocsc_history_accumulate(c);
    if (rc == OCSC_OK) rc = ocsc_dict_update(c);
  }
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(c->stream, &g);
  if (rc == OCSC_OK && e != hipSuccess)
    rc = fail(c, OCSC_E_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
  c->prof_mask = mask;
  c->t = t0;   // nothing ran yet; each launch counts its 2B samples
  c->sweep_count = sc0;
  c->pending_B = c->fold_B = 0;
  if (rc == OCSC_OK) {
    gr->graph = g;
    e = hipGraphInstantiate(&gr->exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) rc = fail(c, OCSC_E_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
  } else if (g) {
    (void)hipGraphDestroy(g);
  }
  if (rc != OCSC_OK) {
    if (gr->graph) (void)hipGraphDestroy(gr->graph);
    delete gr;
    return rc;
  }
  *out = gr;
  return OCSC_OK;
}

int ocsc_graph_launch(ocsc_graph* gr) {
  OCSC_RANGE();
  if (!gr) return OCSC_E_INVALID_ARG;
  ocsc_ctx* c = gr->c;
  if (c->pending_B || c->fold_B) return fail(c, OCSC_E_STATE, "pending codes or a deferred fold");
  HIPX(c, hipGraphLaunch(gr->exec, c->stream));
  c->t += 2 * gr->B;
  return OCSC_OK;
}

int ocsc_graph_destroy(ocsc_graph* gr) {
  if (!gr) return OCSC_OK;
  if (gr->c && gr->c->stream) (void)hipStreamSynchronize(gr->c->stream);
  if (gr->exec) (void)hipGraphExecDestroy(gr->exec);
  if (gr->graph) (void)hipGraphDestroy(gr->graph);
  delete gr;
  return OCSC_OK;
}

// ---------------------------------------------------------------- launch shapes
int ocsc_get_tuning(const ocsc_ctx* c, ocsc_tuning* out) {
  if (!c || !out) return OCSC_E_INVALID_ARG;
  *out = c->tune;
  return OCSC_OK;
}

int ocsc_set_tuning(ocsc_ctx* c, const ocsc_tuning* t) {
  if (!c) return OCSC_E_INVALID_ARG;
  if (!t) return fail(c, OCSC_E_INVALID_ARG, "tuning is NULL");
  if (!tuning_valid(c, *t)) return fail(c, OCSC_E_INVALID_ARG, "unsupported launch shape");
  if (t->two_pass == 1) {
    const int rc = ensure_column_buffer(c);
    if (rc) return rc;
  }
  c->tune = *t;
  return OCSC_OK;
}

int ocsc_autotune(ocsc_ctx* c, int B, ocsc_tuning* out, double* best_ms) {
  OCSC_RANGE();
  if (!c) return OCSC_E_INVALID_ARG;
  if (B < 1 || B > c->maxB) return fail(c, OCSC_E_INVALID_ARG, "B must be in [1, max_batch]");
  if (c->pending_B) return fail(c, OCSC_E_STATE, "pending codes occupy the code workspace");
  if (c->stream) {
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    HIPX(c, hipStreamIsCapturing(c->stream, &st));
    if (st != hipStreamCaptureStatusNone) return fail(c, OCSC_E_STATE, "the context stream is being captured");
  }
  double ms = 0;
  const int rc = c->sr == 8 ? autotune_t<double>(c, B, &ms) : autotune_t<float>(c, B, &ms);
  if (rc) return rc;
  if (out) *out = c->tune;
  if (best_ms) *best_ms = ms;
  return OCSC_OK;
}

int ocsc_sync(ocsc_ctx* c) {
  OCSC_RANGE();
  if (!c) return OCSC_E_INVALID_ARG;
  HIPX(c, hipStreamSynchronize(c->stream));
  return check_breakdown(c);
}

const char* ocsc_last_error(const ocsc_ctx* c) { return c ? c->err.c_str() : g_init_error.c_str(); }

int ocsc_state_bytes(const ocsc_ctx* c, int which, int64_t* out) {
  if (!c || !out) return OCSC_E_INVALID_ARG;
  size_t n = 0;
  if (state_bytes(c, which, &n)) return OCSC_E_INVALID_ARG;
  *out = (int64_t)n;
  return OCSC_OK;
}

int ocsc_get_state(ocsc_ctx* c, int which, void* dst) {
  OCSC_RANGE();
  if (!c) return OCSC_E_INVALID_ARG;
  size_t n = 0;
  if (!dst || state_bytes(c, which, &n)) return fail(c, OCSC_E_INVALID_ARG, "bad state item or NULL dst");
  if (which == OCSC_STATE_CINV || which == OCSC_STATE_G || which == OCSC_STATE_RHS) {
    int rc = c->sr == 8 ? flush_fold<double>(c) : flush_fold<float>(c);
    if (rc) return rc;
  }
  if (which == OCSC_STATE_CINV || which == OCSC_STATE_H) {
    void* m = which == OCSC_STATE_H ? c->Hm : c->Cm;
    int rc = c->sr == 8 ? cinv_layout_t<double>(c, m, dst, 0) : cinv_layout_t<float>(c, m, dst, 0);
    if (rc) return rc;
  } else {
    HIPX(c, hipMemcpyAsync(dst, state_ptr(c, which), n, hipMemcpyDeviceToDevice, c->stream));
  }
  HIPX(c, hipStreamSynchronize(c->stream));
  return OCSC_OK;
}

int ocsc_set_state(ocsc_ctx* c, int which, const void* src) {
  OCSC_RANGE();
  if (!c) return OCSC_E_INVALID_ARG;
  size_t n = 0;
  if (!src || state_bytes(c, which, &n) || which == OCSC_STATE_ZHAT || which == OCSC_STATE_XHAT)
    return fail(c, OCSC_E_INVALID_ARG, "bad state item or NULL src");
  // a deferred fold is applied before the item is replaced
  int rf = c->sr == 8 ? flush_fold<double>(c) : flush_fold<float>(c);
  if (rf) return rf;
  c->pending_B = 0;
  if (which == OCSC_STATE_CINV || which == OCSC_STATE_H) {
    void* m = which == OCSC_STATE_H ? c->Hm : c->Cm;
    int rc = c->sr == 8 ? cinv_layout_t<double>(c, src, m, 1) : cinv_layout_t<float>(c, src, m, 1);
    if (rc) return rc;
  } else {
    HIPX(c, hipMemcpyAsync(state_ptr(c, which), src, n, hipMemcpyDeviceToDevice, c->stream));
  }
  if (which == OCSC_STATE_DICT_HAT) {
    int rc = c->sr == 8 ? launch_gamma<double>(c) : launch_gamma<float>(c);
    if (rc) return rc;
  }
  HIPX(c, hipStreamSynchronize(c->stream));
  return OCSC_OK;
}

int ocsc_get_count(const ocsc_ctx* c, int64_t* t) {
  if (!c || !t) return OCSC_E_INVALID_ARG;
  *t = c->t;
  return OCSC_OK;
}

int ocsc_set_count(ocsc_ctx* c, int64_t t) {
  if (!c || t < 0) return OCSC_E_INVALID_ARG;
  c->t = t;
  return OCSC_OK;
}

int ocsc_profile_enable(ocsc_ctx* c, unsigned mask) {
  if (!c) return OCSC_E_INVALID_ARG;
  int rc = prof_collect(c);
  if (rc) return rc;
  c->prof_mask = mask & ((1u << OCSC_KC_COUNT) - 1);
  for (int i = 0; i < OCSC_KC_COUNT; ++i) {
    c->prof_ms[i] = 0;
    c->prof_n[i] = 0;
  }
  return OCSC_OK;
}

int ocsc_profile_read(ocsc_ctx* c, int cls, double* ms, int64_t* n) {
  if (!c || cls < 0 || cls >= OCSC_KC_COUNT || !ms || !n) return OCSC_E_INVALID_ARG;
  int rc = prof_collect(c);
  if (rc) return rc;
  *ms = c->prof_ms[cls];
  *n = c->prof_n[cls];
  return OCSC_OK;
}

}  // extern "C"
