// dstep.hpp -- history fold and D-step sweep (eqs. B_update, C_update and
// sub_d_sol) over the per-frequency inverse matrices C_p, and their layout.
//
// C_p = (H_p + rho_d I)^-1 lives in HBM as T[Pf][fs]: K rows of pitch K + 1
// reals, R-form R[i][j] = Re C_ij (j >= i), R[j][i] = Im C_ij (j > i).
#pragma once
#include "common.hpp"

namespace ocsc {

// ---------------------------------------------------------------------------
// Per-frequency Hermitian algebra on C held in LDS.
//
// C_p is stored (in HBM and in LDS alike) as K rows of pitch ld = K + 1 reals:
// R[i][j] = Re C_ij for j >= i and R[j][i] = Im C_ij for j > i (the Hermitian
// matrix in K*K reals; the pad column is unused).  Frequency p occupies fs
// reals (fs = K*ld rounded up to 16 bytes), so a block of consecutive
// frequencies is one contiguous run that stages into LDS by 16-byte copies.
// ---------------------------------------------------------------------------

// Sum of v over the tpg threads of one group (tpg a power of two; groups are
// aligned sub-waves or whole waves).  scratch: one T per wave of the block.
// Every thread of the group gets the total.  Contains a block-wide barrier.
template <typename T>
__device__ __forceinline__ T group_sum(T v, int tpg, T* scratch) {
  const int w = tpg < 64 ? tpg : 64;
  for (int off = w >> 1; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  if (tpg <= 64) return v;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) scratch[wave] = v;
  __syncthreads();
  const int nw = tpg >> 6, w0 = (wave / nw) * nw;
  T s = 0;
  for (int i = 0; i < nw; ++i) s += scratch[w0 + i];
  __syncthreads();
  return s;
}

// y = C x by the lt-th of the tpg threads serving one frequency.  Thread
// (i, h) sums row i over the h-th of ns column chunks; at column j it reads
// p = R[i][j] and q = R[j][i] and forms C_ij = (p, q) above the diagonal and
// (q, -p) below it.  Partial sums pass through part[ns][K].
template <typename T>
__device__ __forceinline__ void herm_matvec(const T* __restrict__ R, int K, int ld, const cx<T>* x, cx<T>* y,
                                            cx<T>* part, int lt, int tpg, int ns) {
  const int chunk = (K + ns - 1) / ns;
  for (int task = lt; task < K * ns; task += tpg) {
    const int h = task / K, i = task - h * K;
    const int j0 = h * chunk, j1 = min(K, j0 + chunk);
    const T* rowp = R + i * ld;
    const T* colp = R + i;
    T yr = 0, yi = 0;
#pragma unroll 4
    for (int j = j0; j < j1; ++j) {
      const T p = rowp[j], q = colp[j * ld];
      const cx<T> xv = x[j];
      const bool up = j > i;
      const T a = up ? p : q;
      const T b = up ? q : -p;
      yr += a * xv.x - b * xv.y;
      yi += a * xv.y + b * xv.x;
    }
    if (i >= j0 && i < j1) {   // the loop took Im C_ii = -R[i][i]; it is zero
      const T dg = rowp[i];
      const cx<T> xv = x[i];
      yr -= dg * xv.y;
      yi += dg * xv.x;
    }
    part[h * K + i] = mk<T>(yr, yi);
  }
  __syncthreads();
  for (int i = lt; i < K; i += tpg) {
    cx<T> s = part[i];
    for (int h = 1; h < ns; ++h) s = cadd<T>(s, part[h * K + i]);
    y[i] = s;
  }
  __syncthreads();
}

// y1 = C x1 and y2 = C x2 in one pass over C (same thread layout as
// herm_matvec); part holds 2 * ns * K partial sums.
template <typename T>
__device__ __forceinline__ void herm_matvec2(const T* __restrict__ R, int K, int ld, const cx<T>* x1,
                                             const cx<T>* x2, cx<T>* y1, cx<T>* y2, cx<T>* part, int lt,
                                             int tpg, int ns) {
  const int chunk = (K + ns - 1) / ns;
  cx<T>* part2 = part + ns * K;
  for (int task = lt; task < K * ns; task += tpg) {
    const int h = task / K, i = task - h * K;
    const int j0 = h * chunk, j1 = min(K, j0 + chunk);
    const T* rowp = R + i * ld;
    const T* colp = R + i;
    T ar = 0, ai = 0, br = 0, bi = 0;
#pragma unroll 4
    for (int j = j0; j < j1; ++j) {
      const T p = rowp[j], q = colp[j * ld];
      const cx<T> u = x1[j], v = x2[j];
      const bool up = j > i;
      const T a = up ? p : q;
      const T b = up ? q : -p;
      ar += a * u.x - b * u.y;
      ai += a * u.y + b * u.x;
      br += a * v.x - b * v.y;
      bi += a * v.y + b * v.x;
    }
    if (i >= j0 && i < j1) {
      const T dg = rowp[i];
      const cx<T> u = x1[i], v = x2[i];
      ar -= dg * u.y;
      ai += dg * u.x;
      br -= dg * v.y;
      bi += dg * v.x;
    }
    part[h * K + i] = mk<T>(ar, ai);
    part2[h * K + i] = mk<T>(br, bi);
  }
  __syncthreads();
  for (int i = lt; i < K; i += tpg) {
    cx<T> s1 = part[i], s2 = part2[i];
    for (int h = 1; h < ns; ++h) {
      s1 = cadd<T>(s1, part[h * K + i]);
      s2 = cadd<T>(s2, part2[h * K + i]);
    }
    y1[i] = s1;
    y2[i] = s2;
  }
  __syncthreads();
}

// C <- C - beta v v^H on the stored reals: R[i][j] (j >= i) loses
// beta Re(v_i conj v_j); R[i][j] (j < i, holding Im C_ji) loses beta Im(v_j conj v_i).
template <typename T>
__device__ __forceinline__ void herm_rank1(T* __restrict__ R, int K, int ld, const cx<T>* v, T beta, int lt,
                                           int tpg, int ns) {
  const int chunk = (K + ns - 1) / ns;
  for (int task = lt; task < K * ns; task += tpg) {
    const int h = task / K, i = task - h * K;
    const int j0 = h * chunk, j1 = min(K, j0 + chunk);
    const cx<T> vi = v[i];
    T* rowp = R + i * ld;
    for (int j = j0; j < j1; ++j) {
      const cx<T> vj = v[j];
      rowp[j] -= beta * (j >= i ? (vi.x * vj.x + vi.y * vj.y) : (vj.y * vi.x - vj.x * vi.y));
    }
  }
  __syncthreads();
}

// Compile-time variants for a fixed K and group width TPG: the row pitch and
// column chunk are constants, the column loop is unrolled, and every LDS
// access is a base register plus an immediate offset.
template <int KT, int TPG>
struct HGeo {
  static constexpr int LD = KT + 1;
  static constexpr int RP = TPG >= 64 ? (KT + 63) / 64 * 64 : KT;   // row slots of a column chunk
  static constexpr int NS0 = TPG / RP;
  static constexpr int NS = NS0 < 1 ? 1 : (NS0 > 4 ? 4 : NS0);        // column chunks
  static constexpr int CH = (KT + NS - 1) / NS;                       // columns per chunk
  static constexpr int TASKS = RP * NS;
};

template <typename T, int KT, int TPG, int NX>
__device__ __forceinline__ void herm_matvec_ct(const T* __restrict__ R, const cx<T>* const (&x)[NX],
                                               cx<T>* const (&y)[NX], cx<T>* part, int lt) {
  using H = HGeo<KT, TPG>;
  for (int task = lt; task < H::TASKS; task += TPG) {
    const int h = task / H::RP, i = task % H::RP;
    if (i < KT) {
      const int j0 = h * H::CH;
      const T* rowp = R + i * H::LD + j0;   // R[i][j0 + jj]
      const T* colp = R + j0 * H::LD + i;   // R[j0 + jj][i]
      T ar[NX], ai[NX];
#pragma unroll
      for (int n = 0; n < NX; ++n) ar[n] = ai[n] = 0;
#pragma unroll
      for (int jj = 0; jj < H::CH; ++jj) {
        if (H::CH * H::NS != KT && j0 + jj >= KT) break;
        const T p = rowp[jj], q = colp[jj * H::LD];
        const bool up = j0 + jj > i;
        const T a = up ? p : q;
        const T b = up ? q : -p;
#pragma unroll
        for (int n = 0; n < NX; ++n) {
          const cx<T> xv = x[n][j0 + jj];
          ar[n] += a * xv.x - b * xv.y;
          ai[n] += a * xv.y + b * xv.x;
        }
      }
      if (i >= j0 && i < j0 + H::CH) {   // the loop took Im C_ii = -R[i][i]; it is zero
        const T dg = R[i * H::LD + i];
#pragma unroll
        for (int n = 0; n < NX; ++n) {
          const cx<T> xv = x[n][i];
          ar[n] -= dg * xv.y;
          ai[n] += dg * xv.x;
        }
      }
#pragma unroll
      for (int n = 0; n < NX; ++n) part[(n * H::NS + h) * KT + i] = mk<T>(ar[n], ai[n]);
    }
  }
  __syncthreads();
  for (int i = lt; i < KT; i += TPG) {
#pragma unroll
    for (int n = 0; n < NX; ++n) {
      cx<T> sum = part[(n * H::NS) * KT + i];
#pragma unroll
      for (int h = 1; h < H::NS; ++h) sum = cadd<T>(sum, part[(n * H::NS + h) * KT + i]);
      y[n][i] = sum;
    }
  }
  __syncthreads();
}

template <typename T, int KT, int TPG>
__device__ __forceinline__ void herm_rank1_ct(T* __restrict__ R, const cx<T>* v, T beta, int lt) {
  using H = HGeo<KT, TPG>;
  for (int task = lt; task < H::TASKS; task += TPG) {
    const int h = task / H::RP, i = task % H::RP;
    if (i < KT) {
      const int j0 = h * H::CH;
      const cx<T> vi = v[i];
      T* rowp = R + i * H::LD + j0;
#pragma unroll
      for (int jj = 0; jj < H::CH; ++jj) {
        if (H::CH * H::NS != KT && j0 + jj >= KT) break;
        const cx<T> vj = v[j0 + jj];
        const T re = vi.x * vj.x + vi.y * vj.y, im = vj.y * vi.x - vj.x * vi.y;
        rowp[jj] -= beta * (j0 + jj >= i ? re : im);
      }
    }
  }
  __syncthreads();
}

// N sums over the tpg threads of one group at once (as group_sum; scratch:
// N values per wave of the block).  Contains block-wide barriers when tpg > 64.
template <typename T, int N>
__device__ __forceinline__ void group_sum_vec(T (&v)[N], int tpg, T* scratch) {
  const int w = tpg < 64 ? tpg : 64;
#pragma unroll
  for (int n = 0; n < N; ++n)
    for (int off = w >> 1; off > 0; off >>= 1) v[n] += __shfl_xor(v[n], off, 64);
  if (tpg <= 64) return;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0)
#pragma unroll
    for (int n = 0; n < N; ++n) scratch[wave * N + n] = v[n];
  __syncthreads();
  const int nw = tpg >> 6, w0 = (wave / nw) * nw;
#pragma unroll
  for (int n = 0; n < N; ++n) {
    T s = 0;
    for (int i = 0; i < nw; ++i) s += scratch[(w0 + i) * N + n];
    v[n] = s;
  }
  __syncthreads();
}

// Y_n = C X_n for NB vectors in one pass over C (thread layout of
// herm_matvec); X, Y: [NB][K]; part: [NB][ns][K].
template <typename T, int NB>
__device__ __forceinline__ void herm_matvec_n(const T* __restrict__ R, int K, int ld, const cx<T>* X, cx<T>* Y,
                                              cx<T>* part, int lt, int tpg, int ns) {
  const int chunk = (K + ns - 1) / ns;
  for (int task = lt; task < K * ns; task += tpg) {
    const int h = task / K, i = task - h * K;
    const int j0 = h * chunk, j1 = min(K, j0 + chunk);
    const T* rowp = R + i * ld;
    const T* colp = R + i;
    T yr[NB], yi[NB];
#pragma unroll
    for (int n = 0; n < NB; ++n) yr[n] = yi[n] = 0;
#pragma unroll 2
    for (int j = j0; j < j1; ++j) {
      const T p = rowp[j], q = colp[j * ld];
      const bool up = j > i;
      const T a = up ? p : q;
      const T b = up ? q : -p;
#pragma unroll
      for (int n = 0; n < NB; ++n) {
        const cx<T> xv = X[n * K + j];
        yr[n] += a * xv.x - b * xv.y;
        yi[n] += a * xv.y + b * xv.x;
      }
    }
    if (i >= j0 && i < j1) {   // the loop took Im C_ii = -R[i][i]; it is zero
      const T dg = rowp[i];
#pragma unroll
      for (int n = 0; n < NB; ++n) {
        const cx<T> xv = X[n * K + i];
        yr[n] -= dg * xv.y;
        yi[n] += dg * xv.x;
      }
    }
#pragma unroll
    for (int n = 0; n < NB; ++n) part[(n * ns + h) * K + i] = mk<T>(yr[n], yi[n]);
  }
  __syncthreads();
  for (int i = lt; i < K; i += tpg) {
#pragma unroll
    for (int n = 0; n < NB; ++n) {
      cx<T> s = part[(n * ns) * K + i];
      for (int h = 1; h < ns; ++h) s = cadd<T>(s, part[(n * ns + h) * K + i]);
      Y[n * K + i] = s;
    }
  }
  __syncthreads();
}

// C <- C - sum_n beta_n v_n v_n^H on the stored reals (as herm_rank1); V: [NB][K].
template <typename T, int NB>
__device__ __forceinline__ void herm_rank_n(T* __restrict__ R, int K, int ld, const cx<T>* V, const T (&beta)[NB],
                                            int lt, int tpg, int ns) {
  const int chunk = (K + ns - 1) / ns;
  for (int task = lt; task < K * ns; task += tpg) {
    const int h = task / K, i = task - h * K;
    const int j0 = h * chunk, j1 = min(K, j0 + chunk);
    cx<T> vi[NB];
#pragma unroll
    for (int n = 0; n < NB; ++n) vi[n] = V[n * K + i];
    T* rowp = R + i * ld;
    for (int j = j0; j < j1; ++j) {
      T dlt = 0;
#pragma unroll
      for (int n = 0; n < NB; ++n) {
        const cx<T> vj = V[n * K + j];
        dlt += beta[n] * (j >= i ? (vi[n].x * vj.x + vi[n].y * vj.y) : (vj.y * vi[n].x - vj.x * vi[n].y));
      }
      rowp[j] -= dlt;
    }
  }
  __syncthreads();
}

// 16-byte vectors of one slot (fpb consecutive frequencies) held by one
// thread: at most SWEEP_MAXV in the generic kernel (KT = 0), at most
// SWEEP_MAXV_L in the generic kernel for large slots (KT = -1; one frequency of
// up to 69,632 bytes: FP32 K <= 131, FP64 K <= 92).
constexpr int SWEEP_MAXV = 12;
constexpr int SWEEP_MAXV_L = 17;

// 16-byte vectors of one slot per thread: exact for the compile-time
// specialisations (KT > 0), the bound of the generic kernels otherwise.
template <typename T, int KT, int FPB>
__host__ __device__ constexpr int sweep_nvm() {
  if constexpr (KT > 0) {
    constexpr int VR = 16 / (int)sizeof(T);
    constexpr int fs = (KT * (KT + 1) + VR - 1) / VR * VR;
    return (FPB * fs * (int)sizeof(T) / 16 + 255) / 256;
  } else if constexpr (KT < 0) {
    return SWEEP_MAXV_L;
  } else {
    return SWEEP_MAXV;
  }
}

// LDS of one D-step workgroup:
//   [C of fpb frequencies, padded to nvm * 256 16-byte vectors]
//   [per frequency group: x (max(K, group width)), y, C u, C G (K each), partial sums (8K)] complex.
// The padding and the wide x take the stores of lanes past the slot or past K,
// so staging needs no guard.
__host__ __device__ inline size_t sweep_r_bytes(int fpb, int fs, int sr, int nvm) {
  const size_t a = (size_t)fpb * fs * sr, b = (size_t)nvm * 256 * 16;
  return a > b ? a : b;
}
__host__ __device__ inline int sweep_group_vecs(int K, int fpb) {
  const int tpg = 256 / fpb;
  return (K > tpg ? K : tpg) + 11 * K;
}
__host__ __device__ inline size_t sweep_lds_bytes(int K, int fpb, int fs, int sr, int nvm) {
  return sweep_r_bytes(fpb, fs, sr, nvm) + (size_t)fpb * sweep_group_vecs(K, fpb) * 2 * sr;
}
// A plain sweep (no fold) instead holds [C][run of right-hand sides: spw*fpb*K][partial sums: 4K per group].
__host__ __device__ inline size_t sweep_plain_lds_bytes(int K, int fpb, int fs, int sr, int nvm, int spw) {
  return sweep_r_bytes(fpb, fs, sr, nvm) + ((size_t)spw * fpb * K + (size_t)fpb * 4 * K) * 2 * sr;
}

// The prefetch is straight-line code: every lane loads (indices past the slot
// are clamped to its last vector) and every lane stores (past the slot into
// the padding).  Guarded loads and stores would leave the compiler unable to
// prove that the previous slot's loads into the same registers have landed,
// and it would then wait for all of them before each new load.
// C is read once per sweep, so its loads (and the fold's write-back, see
// slot_writeback) carry the non-temporal hint: its lines are the first to
// leave the caches, and the small vectors of the step (right-hand sides, d,
// which the V-step reads next) stay there.
template <int NV_MAX>
__device__ __forceinline__ void slot_fetch(v4f (&reg)[NV_MAX], const v4f* __restrict__ src, int nvec, int tid) {
#pragma unroll
  for (int v = 0; v < NV_MAX; ++v) reg[v] = __builtin_nontemporal_load(&src[min(tid + v * 256, nvec - 1)]);
}

// the updated C of a slot back to HBM (nv 16-byte vectors)
__device__ __forceinline__ void slot_writeback(v4f* __restrict__ dst, const v4f* src, int nv, int tid) {
  for (int e = tid; e < nv; e += 256) __builtin_nontemporal_store(src[e], &dst[e]);
}

template <int NV_MAX>
__device__ __forceinline__ void slot_stage(const v4f (&reg)[NV_MAX], v4f* dst, int tid) {
#pragma unroll
  for (int v = 0; v < NV_MAX; ++v) dst[tid + v * 256] = reg[v];
}

// A plain sweep keeps the right-hand sides of a workgroup's whole run of
// frequencies [f0, f0 + nrun) in LDS as rb[i][k] (i = p - f0), loaded once at
// the start; each d_p overwrites its right-hand side and the run is stored
// once at the end.  Per filter row the run is one contiguous stretch of
// [K][Pf], so HBM sees whole cache lines instead of one 8-byte value per
// frequency.  All loads of a batch are issued before the first LDS store.
constexpr int RUN_BATCH = 8;

template <typename T>
__device__ __forceinline__ void run_load(cx<T>* rb, const cx<T>* __restrict__ src, int f0, int nrun, int K,
                                         int Pf, int tid) {
  const int n = K * nrun;
  for (int c0 = 0; c0 < n; c0 += RUN_BATCH * 256) {
    cx<T> r[RUN_BATCH];
#pragma unroll
    for (int j = 0; j < RUN_BATCH; ++j) {
      const int e = min(c0 + tid + j * 256, n - 1);
      const int k = e / nrun, i = e - k * nrun;
      r[j] = src[(size_t)k * Pf + f0 + i];
    }
#pragma unroll
    for (int j = 0; j < RUN_BATCH; ++j) {
      const int e = c0 + tid + j * 256;
      if (e < n) {
        const int k = e / nrun, i = e - k * nrun;
        rb[i * K + k] = r[j];
      }
    }
  }
}

template <typename T>
__device__ __forceinline__ void run_store(const cx<T>* rb, cx<T>* __restrict__ dst, int f0, int nrun, int K,
                                          int Pf, int tid) {
  const int n = K * nrun;
  for (int e = tid; e < n; e += 256) {
    const int k = e / nrun, i = e - k * nrun;
    dst[(size_t)k * Pf + f0 + i] = rb[i * K + k];
  }
}

// ---------------------------------------------------------------------------
// D-step sweep over all frequencies (eq. sub_d_sol, column form):
//   d_p = C_p rhs_p.
// A workgroup walks a run of slots (fpb frequencies each; the fpb groups of
// 256/fpb threads work side by side); while one slot is being solved the next
// slot's C is already in flight into registers.  The runs of workgroups that
// share an XCD are adjacent in frequency.
//
// nfold > 0: before the D-step the kept spectra of nfold samples are folded
// into the history in sample order (eqs. B_update and C_update):
//   u = conj(z_p);  G_p += u x_p;  v = C_p u;  C_p <- C_p - v v^H / (1 + u^H v),
// with z_p read from Zh ([B][K][Pf], one sample) or, for several samples, from
// the frequency-major copy Zt ([Pf][ldt][K], each sample's K values
// contiguous), fetched a few samples ahead;
// the updated C_p is written back and the right-hand side is the updated G_p
// (the first DictOCSC iterate, from V = Theta = 0).  With rfold (warm start)
// the right-hand side is instead the carried G + rho_d (F(V) - Theta), which
// the fold advances by the same increments as G and writes back.
// dout == nullptr: fold only.
// MODE: 0 plain sweep (nfold = 0), 1 one-sample fold, 2 multi-sample fold;
// each is its own kernel instance, so that no form carries the registers or
// the slot order of another.
// ---------------------------------------------------------------------------
template <typename T, int KT, int FPB, int MODE>
__global__ __launch_bounds__(256, 3) void k_dict_sweep(T* __restrict__ Cm, cx<T>* __restrict__ G,
                                                    const cx<T>* __restrict__ rhs,
                                                    const cx<T>* __restrict__ Zh,
                                                    const cx<T>* __restrict__ Zt, int ldt,
                                                    const cx<T>* __restrict__ xh, int nfold,
                                                    cx<T>* __restrict__ rfold,
                                                    cx<T>* __restrict__ dout,
                                                    int K_, int Pf, int fpb_, int fs_, int slots_per_wg,
                                                    int reverse) {
  // KT > 0: K and fpb fixed at compile time (the arguments then equal them);
  // KT = 0, -1: generic, slots of up to SWEEP_MAXV, SWEEP_MAXV_L vectors per thread
  constexpr bool CT = KT > 0;
  constexpr bool MF = MODE == 2;
  constexpr bool plain = MODE == 0;
  constexpr int VR = 16 / (int)sizeof(T);
  const int K = CT ? KT : K_;
  const int fpb = CT ? FPB : fpb_;
  const int fs = CT ? (KT * (KT + 1) + VR - 1) / VR * VR : fs_;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int ld = K + 1;
  const int tpg = 256 / fpb;
  const int tid = threadIdx.x;
  const int g = tid / tpg, lt = tid % tpg;
  int ns = tpg / K;
  ns = ns < 1 ? 1 : (ns > 4 ? 4 : ns);
  // 16-byte vectors per thread for one slot (compile-time for a fixed K)
  constexpr int NVM = sweep_nvm<T, KT, FPB>();
  T* Rall = reinterpret_cast<T*>(smem_raw);
  cx<T>* vecs = reinterpret_cast<cx<T>*>(smem_raw + sweep_r_bytes(fpb, fs, (int)sizeof(T), NVM));
  const int XV = K > tpg ? K : tpg;
  cx<T>* xv = vecs + (size_t)g * sweep_group_vecs(K, fpb);   // rhs / u (XV entries)
  cx<T>* yv = xv + XV;                             // result / updated G
  cx<T>* vv = yv + K;                              // C u
  cx<T>* gv = vv + K;                              // C G
  cx<T>* part = gv + K;                            // [8][K]
  __shared__ T wsum[4];
  T* R = Rall + (size_t)g * fs;

  const int nslots = (Pf + fpb - 1) / fpb;
  const int nwg = gridDim.x;
  const int run = xcd_block(blockIdx.x, nwg);
  const int nvec = (int)((size_t)fpb * fs * sizeof(T) / 16);
  // A plain sweep walks a contiguous run of slots (its right-hand sides come
  // in as whole lines, see run_load).  A fold sweep takes its slots round by
  // round instead, slot s * nwg + run in round s: the workgroups of one XCD
  // then hold neighbouring frequencies at the same time and share the cache
  // lines of the per-frequency spectra, G and d that a fold reads and writes.
  const int s_begin = plain ? run * slots_per_wg : 0;
  const int s_end = plain ? min(nslots, s_begin + slots_per_wg) : (run < nslots ? (nslots - 1 - run) / nwg + 1 : 0);
  v4f reg[NVM];

  auto slot_of = [&](int s) {
    const int i = plain ? s : s * nwg + run;
    return reverse ? nslots - 1 - i : i;
  };
  auto slot_vecs = [&](int sl) {
    return min(nvec, (int)(((size_t)min(fpb, Pf - sl * fpb) * fs * sizeof(T)) / 16));
  };
  // plain sweep: the run's right-hand sides in LDS (see run_load)
  const int f0 = (reverse ? nslots - s_end : s_begin) * fpb;
  const int nrun = min(Pf, (reverse ? nslots - s_begin : s_end) * fpb) - f0;
  cx<T>* rb = vecs;
  cx<T>* rpart = vecs + (size_t)slots_per_wg * fpb * K + (size_t)g * 4 * K;
  if (s_begin < s_end) {
    const int sl = slot_of(s_begin);
    slot_fetch<NVM>(reg, reinterpret_cast<const v4f*>(Cm + (size_t)sl * fpb * fs), slot_vecs(sl), tid);
    if (plain) run_load<T>(rb, rhs, f0, nrun, K, Pf, tid);
  }
  for (int s = s_begin; s < s_end; ++s) {
    const int sl = slot_of(s);
    const int p = sl * fpb + g;
    const bool ok = p < Pf;
    const int nv = slot_vecs(sl);
    __syncthreads();   // previous slot finished with LDS
    slot_stage<NVM>(reg, reinterpret_cast<v4f*>(Rall), tid);
    __syncthreads();
    if (s + 1 < s_end) {   // next slot's C is in flight during this slot
      const int sn = slot_of(s + 1);
      slot_fetch<NVM>(reg, reinterpret_cast<const v4f*>(Cm + (size_t)sn * fpb * fs), slot_vecs(sn), tid);
    }
    if (!MF && plain) {
      // d_p replaces its right-hand side in the run buffer (p - f0 < slots_per_wg * fpb)
      cx<T>* xr = rb + (size_t)(p - f0) * K;
      if constexpr (CT) {
        const cx<T>* const xs[1] = {xr};
        cx<T>* const ys[1] = {xr};
        herm_matvec_ct<T, KT, 256 / FPB, 1>(R, xs, ys, rpart, lt);
      } else {
        herm_matvec<T>(R, K, ld, xr, xr, rpart, lt, tpg, ns);
      }
    } else if (!MF) {
      // one sample: v = C u and g = C G_new in one pass; d = g - beta v (v^H G_new)
      if (ok && lt < K) {
        const cx<T> u = cconj<T>(Zh[(size_t)lt * Pf + p]);
        const cx<T> du = cmul<T>(u, xh[p]);
        const cx<T> gn = cadd<T>(G[(size_t)lt * Pf + p], du);
        G[(size_t)lt * Pf + p] = gn;
        xv[lt] = u;
        if (rfold) {
          const cx<T> rn = cadd<T>(rfold[(size_t)lt * Pf + p], du);
          rfold[(size_t)lt * Pf + p] = rn;
          yv[lt] = rn;
        } else {
          yv[lt] = gn;
        }
      }
      __syncthreads();
      if constexpr (CT) {
        const cx<T>* const xs[2] = {xv, yv};
        cx<T>* const ys[2] = {vv, gv};
        herm_matvec_ct<T, KT, 256 / FPB, 2>(R, xs, ys, part, lt);
      } else {
        herm_matvec2<T>(R, K, ld, xv, yv, vv, gv, part, lt, tpg, ns);
      }
      T su = 0, tr = 0, ti = 0;
      if (lt < K) {
        const cx<T> u = xv[lt], v = vv[lt], gn = yv[lt];
        su = u.x * v.x + u.y * v.y;                  // Re(conj(u) v)
        tr = v.x * gn.x + v.y * gn.y;                // conj(v) G
        ti = v.x * gn.y - v.y * gn.x;
      }
      su = group_sum<T>(su, tpg, wsum);
      tr = group_sum<T>(tr, tpg, wsum);
      ti = group_sum<T>(ti, tpg, wsum);
      const T beta = (T)1 / ((T)1 + su);
      if (dout && lt < K) {
        const cx<T> v = vv[lt];
        const cx<T> tv = mk<T>(beta * tr, beta * ti);
        yv[lt] = csub<T>(gv[lt], cmul<T>(v, tv));
      }
      if constexpr (CT) herm_rank1_ct<T, KT, 256 / FPB>(R, vv, beta, lt);
      else herm_rank1<T>(R, K, ld, vv, beta, lt, tpg, ns);
      slot_writeback(reinterpret_cast<v4f*>(Cm + (size_t)sl * fpb * fs), reinterpret_cast<const v4f*>(Rall), nv, tid);
    } else if constexpr (MF) {
      // several samples, folded in sample order in blocks of FB (the
      // recursion of eq. C_update applied FB times per pass over C).  With
      // u_q = conj(z_q) and Y_q = C u_q for the block (one pass), M_jk = u_j^H Y_k:
      //   v_j = C_(j-1) u_j = sum_k T_kj Y_k,
      //   T_.j = e_j - sum_(i<j) beta_i (v_i^H u_j) T_.i,   v_i^H u_j = sum_k conj(T_ki) conj(M_jk),
      //   beta_j = 1 / (1 + Re u_j^H v_j) = 1 / (1 + Re sum_k T_kj M_jk),
      // then C <- C - sum_j beta_j v_j v_j^H in one pass.  The block's z and x
      // come from the frequency-major copy (each sample's K values contiguous)
      // and the next block's are fetched during this one; G_p stays in a
      // register (the same sums in the same order as one sample at a time).
      constexpr int FB = 3;
      __shared__ T wsv[4 * 2 * FB * FB];
      cx<T>* U = xv;                   // [FB][K]: u, then v
      cx<T>* Y = xv + FB * K;          // [FB][K]
      cx<T>* P = xv + 2 * FB * K;      // [FB][2][K] (the group's area holds >= 12 K)
      const int ns2 = ns < 2 ? ns : 2;
      cx<T> dsum = mk<T>(0, 0), gacc = mk<T>(0, 0);
      cx<T> zq[FB], xq[FB];
      const cx<T>* zt = Zt + (size_t)p * ldt * K;
#pragma unroll
      for (int q = 0; q < FB; ++q) zq[q] = xq[q] = mk<T>(0, 0);
      if (ok && lt < K) {
        gacc = G[(size_t)lt * Pf + p];
#pragma unroll
        for (int q = 0; q < FB; ++q) {
          if (q < nfold) {
            zq[q] = zt[(size_t)q * K + lt];
            xq[q] = xh[(size_t)q * Pf + p];
          }
        }
      }
      for (int b0 = 0; b0 < nfold; b0 += FB) {
        if (lt < K) {
#pragma unroll
          for (int q = 0; q < FB; ++q) {
            cx<T> u = mk<T>(0, 0);
            if (ok && b0 + q < nfold) {
              u = cconj<T>(zq[q]);
              const cx<T> du = cmul<T>(u, xq[q]);
              gacc = cadd<T>(gacc, du);
              dsum = cadd<T>(dsum, du);
            }
            U[q * K + lt] = u;
          }
          if (ok) {
#pragma unroll
            for (int q = 0; q < FB; ++q) {
              const int bn = b0 + FB + q;
              if (bn < nfold) {
                zq[q] = zt[(size_t)bn * K + lt];
                xq[q] = xh[(size_t)bn * Pf + p];
              }
            }
          }
        }
        __syncthreads();
        herm_matvec_n<T, FB>(R, K, ld, U, Y, P, lt, tpg, ns2);
        T m[2 * FB * FB];
#pragma unroll
        for (int j = 0; j < FB; ++j) {
#pragma unroll
          for (int k = 0; k < FB; ++k) {
            T sr = 0, si = 0;
            if (lt < K) {
              const cx<T> uj = U[j * K + lt], yk = Y[k * K + lt];
              sr = uj.x * yk.x + uj.y * yk.y;   // conj(u_j) y_k
              si = uj.x * yk.y - uj.y * yk.x;
            }
            m[2 * (j * FB + k)] = sr;
            m[2 * (j * FB + k) + 1] = si;
          }
        }
        group_sum_vec<T, 2 * FB * FB>(m, tpg, wsv);
        cx<T> tc[FB][FB];   // tc[k][j] = T_kj
        T beta[FB];
#pragma unroll
        for (int j = 0; j < FB; ++j) {
#pragma unroll
          for (int k = 0; k < FB; ++k) tc[k][j] = mk<T>(k == j ? (T)1 : (T)0, 0);
#pragma unroll
          for (int i = 0; i < j; ++i) {
            T cr = 0, ci = 0;   // v_i^H u_j
#pragma unroll
            for (int k = 0; k < FB; ++k) {
              const T mr = m[2 * (j * FB + k)], mi = m[2 * (j * FB + k) + 1];
              const cx<T> t = tc[k][i];   // conj(t) conj(M_jk) = conj(t M_jk)
              cr += t.x * mr - t.y * mi;
              ci -= t.x * mi + t.y * mr;
            }
            const T fr = beta[i] * cr, fi = beta[i] * ci;
#pragma unroll
            for (int k = 0; k < FB; ++k) {
              const cx<T> t = tc[k][i];
              tc[k][j] = mk<T>(tc[k][j].x - (fr * t.x - fi * t.y), tc[k][j].y - (fr * t.y + fi * t.x));
            }
          }
          T sj = 0;   // Re u_j^H v_j
#pragma unroll
          for (int k = 0; k < FB; ++k) {
            const T mr = m[2 * (j * FB + k)], mi = m[2 * (j * FB + k) + 1];
            sj += tc[k][j].x * mr - tc[k][j].y * mi;
          }
          beta[j] = (T)1 / ((T)1 + sj);
        }
        __syncthreads();   // U (read for M) is overwritten by v below
        if (lt < K) {
#pragma unroll
          for (int j = 0; j < FB; ++j) {
            cx<T> v = mk<T>(0, 0);
#pragma unroll
            for (int k = 0; k < FB; ++k) {
              const cx<T> y = Y[k * K + lt], t = tc[k][j];
              v = mk<T>(v.x + t.x * y.x - t.y * y.y, v.y + t.x * y.y + t.y * y.x);
            }
            U[j * K + lt] = v;
          }
        }
        __syncthreads();
        herm_rank_n<T, FB>(R, K, ld, U, beta, lt, tpg, ns);
      }
      if (ok && lt < K) G[(size_t)lt * Pf + p] = gacc;
      slot_writeback(reinterpret_cast<v4f*>(Cm + (size_t)sl * fpb * fs), reinterpret_cast<const v4f*>(Rall), nv, tid);
      if (rfold && ok && lt < K) {
        const cx<T> rn = cadd<T>(rfold[(size_t)lt * Pf + p], dsum);
        rfold[(size_t)lt * Pf + p] = rn;
        if (dout) xv[lt] = rn;
      } else if (dout && ok && lt < K) {
        xv[lt] = gacc;
      }
      __syncthreads();
      if (dout) herm_matvec<T>(R, K, ld, xv, yv, part, lt, tpg, ns);
    }
    if (!dout || plain) continue;
    __syncthreads();
    if (ok && lt < K) dout[(size_t)lt * Pf + p] = yv[lt];
  }
  if (plain && s_begin < s_end) run_store<T>(rb, dout, f0, nrun, K, Pf, tid);   // the last matvec ended with a barrier
}

// Packed [Pf][K][K] <-> the per-frequency layout of pitch ld = K + 1 and stride fs.
template <typename T>
__global__ void k_cinv_layout(const T* __restrict__ src, T* __restrict__ dst, int K, int Pf, int fs, int to_internal) {
  const size_t kk = (size_t)K * K;
  const size_t n = kk * Pf;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
    const size_t p = e / kk, r = e % kk;
    const size_t i = r / K, j = r % K;
    const size_t in = p * fs + i * (K + 1) + j;
    if (to_internal) dst[in] = src[e];
    else dst[e] = src[in];
  }
}

// C_p = I / rho_d for every frequency, in the per-frequency layout (pitch K + 1, stride fs).
template <typename T>
__global__ void k_c_init(T* __restrict__ Cm, int K, int Pf, int fs, T inv_rho_d) {
  const size_t n = (size_t)fs * Pf;
  const int ld = K + 1;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
    const int r = (int)(e % fs);
    const int i = r / ld, j = r % ld;
    Cm[e] = (i < K && i == j) ? inv_rho_d : (T)0;
  }
}

}  // namespace ocsc
