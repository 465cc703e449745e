// kernels.hpp -- gfx950 kernels of the OCSC hot path (templated on the real type).
//
// Layouts in HBM (Pf = PH * (PW/2+1) stored frequencies, P = PH * PW):
//   spectra     cx[plane][Pf]          plane = b*K + k (codes) or k (dictionary)
//   real planes T[plane][PH][PW]
//   inverse C   T[Pf][K][K]            R-form: R[i][j] = Re C_ij (j >= i),
//                                              R[j][i] = Im C_ij (j > i)
#pragma once
#include "fft_lds.hpp"

namespace ocsc {

// blockIdx -> work-block index: consecutive work blocks go to the same XCD
// (blocks are dispatched round-robin over the 8 XCDs), so neighbouring
// frequencies share one L2.  A bijection on [0, nb).
__device__ __forceinline__ int xcd_block(int b, int nb) {
  const int q = nb >> 3;
  if (b >= (q << 3)) return b;
  return (b & 7) * q + (b >> 3);
}

template <int PH, int PW, typename T>
__device__ __forceinline__ void load_tables(cx<T>* sH, cx<T>* sW, const cx<T>* twH, const cx<T>* twW,
                                            int tid, int nt) {
  for (int i = tid; i < PH; i += nt) sH[i] = twH[i];
  for (int i = tid; i < PW; i += nt) sW[i] = twW[i];
}

typedef float v4f __attribute__((ext_vector_type(4)));

// Global <-> LDS traffic of one PH x PW plane in 16-byte vectors.  Every
// thread issues all of its loads before it stores any of them, so the plane's
// HBM latency is paid once, not once per loop trip.
template <typename T, int PH, int PW, int NT>
struct PlaneIO {
  using G = PlaneGeom<PH, PW>;
  static constexpr int VR = 16 / (int)sizeof(T);   // reals per vector
  static constexpr int NSV = G::PF * 2 / VR;       // vectors per half spectrum
  static constexpr int NRV = G::P / VR;            // vectors per real plane
  static constexpr int CS = (NSV + NT - 1) / NT;
  static constexpr int CR = (NRV + NT - 1) / NT;
  // LDS slot (complex index) of the first pixel pair of real vector e
  static __device__ __forceinline__ int slot(int e) {
    const int i = e * VR;
    return (i / PW) * G::LDW + ((i % PW) >> 1);
  }
  static __device__ __forceinline__ void spec_in(cx<T>* buf, const cx<T>* src, int tid) {
    const v4f* s = reinterpret_cast<const v4f*>(src);
    v4f* d = reinterpret_cast<v4f*>(buf);
    v4f r[CS];
#pragma unroll
    for (int q = 0; q < CS; ++q) {
      const int e = tid + q * NT;
      if (NSV % NT == 0 || e < NSV) r[q] = s[e];
    }
#pragma unroll
    for (int q = 0; q < CS; ++q) {
      const int e = tid + q * NT;
      if (NSV % NT == 0 || e < NSV) d[e] = r[q];
    }
  }
  static __device__ __forceinline__ void spec_out(cx<T>* dst, const cx<T>* buf, int tid) {
    const v4f* s = reinterpret_cast<const v4f*>(buf);
    v4f* d = reinterpret_cast<v4f*>(dst);
#pragma unroll
    for (int q = 0; q < CS; ++q) {
      const int e = tid + q * NT;
      if (NSV % NT == 0 || e < NSV) d[e] = s[e];
    }
  }
  // real plane (row pitch PW) -> packed pixel pairs in LDS
  static __device__ __forceinline__ void real_in(cx<T>* buf, const T* src, int tid) {
    const v4f* s = reinterpret_cast<const v4f*>(src);
    v4f r[CR];
#pragma unroll
    for (int q = 0; q < CR; ++q) {
      const int e = tid + q * NT;
      if (NRV % NT == 0 || e < NRV) r[q] = s[e];
    }
#pragma unroll
    for (int q = 0; q < CR; ++q) {
      const int e = tid + q * NT;
      if (NRV % NT == 0 || e < NRV) {
        const T* v = reinterpret_cast<const T*>(&r[q]);
        cx<T>* o = buf + slot(e);
#pragma unroll
        for (int h = 0; h < VR / 2; ++h) o[h] = mk<T>(v[2 * h], v[2 * h + 1]);
      }
    }
  }
};

// ---------------------------------------------------------------------------
// Batched forward R2C of real planes.  Plane q is read from
// src + q * sstride as an sh x sw block (row pitch sw) placed at (0, 0) of a
// zero PH x PW grid, and its half spectrum written to dst + q * dstride.
// ---------------------------------------------------------------------------
template <typename T, int PH, int PW, int NT>
__global__ __launch_bounds__(NT) void k_rfft2(const T* __restrict__ src, int sh, int sw, long sstride,
                                              cx<T>* __restrict__ dst, long dstride,
                                              const cx<T>* __restrict__ twH, const cx<T>* __restrict__ twW) {
  using G = PlaneGeom<PH, PW>;
  using IO = PlaneIO<T, PH, PW, NT>;
  __shared__ __align__(16) cx<T> buf[PH * G::LDW];
  __shared__ cx<T> sH[PH], sW[PW];
  const int tid = threadIdx.x;
  const long q = blockIdx.x;
  load_tables<PH, PW, T>(sH, sW, twH, twW, tid, NT);
  const T* s = src + q * sstride;
  if (sh == PH && sw == PW && (sstride % IO::VR) == 0) {
    IO::real_in(buf, s, tid);
  } else {
    for (int e = tid; e < PH * G::M; e += NT) {
      const int r = e / G::M, n = e % G::M, c = 2 * n;
      T a = 0, b = 0;
      if (r < sh) {
        if (c < sw) a = s[r * sw + c];
        if (c + 1 < sw) b = s[r * sw + c + 1];
      }
      buf[r * G::LDW + n] = mk<T>(a, b);
    }
  }
  __syncthreads();
  rfft2_lds<PH, PW, NT, T>(buf, sH, sW, tid);
  IO::spec_out(dst + q * dstride, buf, tid);
}

// ---------------------------------------------------------------------------
// Batched inverse C2R (with the 1/P factor), keeping the top-left oh x ow block
// of each plane (row pitch ow) at dst + q * dstride.
// ---------------------------------------------------------------------------
template <typename T, int PH, int PW, int NT>
__global__ __launch_bounds__(NT) void k_irfft2_crop(const cx<T>* __restrict__ src, long sstride,
                                                    T* __restrict__ dst, int oh, int ow, long dstride,
                                                    const cx<T>* __restrict__ twH,
                                                    const cx<T>* __restrict__ twW) {
  using G = PlaneGeom<PH, PW>;
  using IO = PlaneIO<T, PH, PW, NT>;
  __shared__ __align__(16) cx<T> buf[PH * G::LDW];
  __shared__ cx<T> sH[PH], sW[PW];
  const int tid = threadIdx.x;
  const long q = blockIdx.x;
  load_tables<PH, PW, T>(sH, sW, twH, twW, tid, NT);
  IO::spec_in(buf, src + q * sstride, tid);
  __syncthreads();
  irfft2_lds<PH, PW, NT, T>(buf, sH, sW, tid);
  const T scale = (T)1 / (T)G::P;
  T* d = dst + q * dstride;
  for (int e = tid; e < oh * ow; e += NT) {
    const int r = e / ow, c = e % ow;
    const cx<T> v = buf[r * G::LDW + (c >> 1)];
    d[e] = ((c & 1) ? v.y : v.x) * scale;
  }
}

// ---------------------------------------------------------------------------
// Code update, spatial half of one ADMM iteration, one workgroup per plane:
//   Y = Re F^-1(Zh);  U = S_kappa(Y + W);  W <- Y + W - U;  S = F(U - W).
// first: W = 0 on entry.  last: write U to Uout (if non-null) and stop.
// ---------------------------------------------------------------------------
template <typename T, int PH, int PW, int NT>
__global__ __launch_bounds__(NT) void k_code_plane(const cx<T>* __restrict__ Zh, T* __restrict__ W,
                                                   cx<T>* __restrict__ S, T* __restrict__ Uout,
                                                   const cx<T>* __restrict__ twH,
                                                   const cx<T>* __restrict__ twW, T kappa, int first,
                                                   int last) {
  using G = PlaneGeom<PH, PW>;
  using IO = PlaneIO<T, PH, PW, NT>;
  constexpr int VR = IO::VR, CR = IO::CR, NRV = IO::NRV;
  __shared__ __align__(16) cx<T> buf[PH * G::LDW];
  __shared__ cx<T> sH[PH], sW[PW];
  const int tid = threadIdx.x;
  const long q = blockIdx.x;
  load_tables<PH, PW, T>(sH, sW, twH, twW, tid, NT);
  IO::spec_in(buf, Zh + q * G::PF, tid);
  // the dual W of this plane is fetched while the inverse transform runs
  v4f* wv = reinterpret_cast<v4f*>(W + q * G::P);
  v4f wr[CR];
#pragma unroll
  for (int j = 0; j < CR; ++j) {
    const int e = tid + j * NT;
    if (NRV % NT == 0 || e < NRV) wr[j] = first ? v4f{0, 0, 0, 0} : wv[e];
  }
  __syncthreads();
  irfft2_lds<PH, PW, NT, T>(buf, sH, sW, tid);
  const T scale = (T)1 / (T)G::P;
  v4f* uv = Uout ? reinterpret_cast<v4f*>(Uout + q * G::P) : nullptr;
#pragma unroll
  for (int j = 0; j < CR; ++j) {
    const int e = tid + j * NT;
    if (NRV % NT == 0 || e < NRV) {
      cx<T>* o = buf + IO::slot(e);
      T* w = reinterpret_cast<T*>(&wr[j]);
      v4f uo;
      T* u = reinterpret_cast<T*>(&uo);
#pragma unroll
      for (int h = 0; h < VR / 2; ++h) {
        const cx<T> y = o[h];
        const T v0 = y.x * scale + w[2 * h], v1 = y.y * scale + w[2 * h + 1];
        const T u0 = copysign(fmax(fabs(v0) - kappa, (T)0), v0);
        const T u1 = copysign(fmax(fabs(v1) - kappa, (T)0), v1);
        u[2 * h] = u0;
        u[2 * h + 1] = u1;
        w[2 * h] = v0 - u0;
        w[2 * h + 1] = v1 - u1;
        o[h] = mk<T>(u0 - w[2 * h], u1 - w[2 * h + 1]);
      }
      if (last) {
        if (uv) uv[e] = uo;
      } else {
        wv[e] = wr[j];
      }
    }
  }
  if (last) return;
  __syncthreads();
  rfft2_lds<PH, PW, NT, T>(buf, sH, sW, tid);
  IO::spec_out(S + q * G::PF, buf, tid);
}

// ---------------------------------------------------------------------------
// Code update, frequency half of one ADMM iteration (the Z-step).  At each
// frequency p with a = Dh[:, p], s = S[:, p]:
//   z = s + conj(a) * gam_p * (x_p - a^T s),   gam_p = 1 / (rho + ||a||^2),
// which is the Sherman-Morrison solution of (conj(a) a^T + rho I) z =
// conj(a) x_p + rho s.  A workgroup of 256 threads serves 16 frequencies of
// one sample: thread (kq, f) holds filters k = kq, kq + 16, ... (at most KPT)
// of frequency f in registers, so each filter row is read as one 128-byte
// (FP32) or 256-byte (FP64) segment.  first: s = 0.
// ---------------------------------------------------------------------------
constexpr int ZF = 16;

template <typename T, int KPT>
__global__ __launch_bounds__(256) void k_code_zstep(const cx<T>* __restrict__ Dh,
                                                   const T* __restrict__ gam,
                                                   const cx<T>* __restrict__ xh,
                                                   const cx<T>* __restrict__ S,
                                                   cx<T>* __restrict__ Zh, int K, int Pf,
                                                   int first) {
  __shared__ cx<T> red[16][ZF + 1];
  const int f = threadIdx.x % ZF, kq = threadIdx.x / ZF;
  const int b = blockIdx.y;
  const int p = blockIdx.x * ZF + f;
  const bool ok = p < Pf;
  cx<T> a[KPT], s[KPT];
  cx<T> acc = mk<T>(0, 0);
#pragma unroll
  for (int j = 0; j < KPT; ++j) {
    const int k = kq + j * 16;
    a[j] = mk<T>(0, 0);
    s[j] = mk<T>(0, 0);
    if (ok && k < K) {
      a[j] = Dh[(size_t)k * Pf + p];
      if (!first) s[j] = S[((size_t)b * K + k) * Pf + p];
    }
    acc = cadd<T>(acc, cmul<T>(a[j], s[j]));
  }
  red[kq][f] = acc;
  __syncthreads();
  if (kq == 0) {
    cx<T> tot = red[0][f];
#pragma unroll
    for (int i = 1; i < 16; ++i) tot = cadd<T>(tot, red[i][f]);
    cx<T> qv = mk<T>(0, 0);
    if (ok) qv = cscale<T>(csub<T>(xh[(size_t)b * Pf + p], tot), gam[p]);
    red[0][f] = qv;
  }
  __syncthreads();
  const cx<T> qv = red[0][f];
#pragma unroll
  for (int j = 0; j < KPT; ++j) {
    const int k = kq + j * 16;
    if (ok && k < K) Zh[((size_t)b * K + k) * Pf + p] = cadd<T>(s[j], cmulc<T>(qv, a[j]));
  }
}

// gam_p = 1 / (rho + sum_k |Dh[k][p]|^2)
template <typename T>
__global__ void k_gamma(const cx<T>* __restrict__ Dh, T* __restrict__ gam, T rho, int K, int Pf) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= Pf) return;
  T acc = 0;
  for (int k = 0; k < K; ++k) {
    const cx<T> a = Dh[(long)k * Pf + p];
    acc += a.x * a.x + a.y * a.y;
  }
  gam[p] = (T)1 / (rho + acc);
}

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

// 16-byte vectors of one slot (fpb consecutive frequencies) held by one thread.
constexpr int SWEEP_MAXV = 12;

// 16-byte vectors of one slot per thread: exact for the compile-time
// specialisations, SWEEP_MAXV for the generic kernel.
template <typename T, int KT, int FPB>
__host__ __device__ constexpr int sweep_nvm() {
  if constexpr (KT > 0) {
    constexpr int VR = 16 / (int)sizeof(T);
    constexpr int fs = (KT * (KT + 1) + VR - 1) / VR * VR;
    return (FPB * fs * (int)sizeof(T) / 16 + 255) / 256;
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
template <int NV_MAX>
__device__ __forceinline__ void slot_fetch(v4f (&reg)[NV_MAX], const v4f* __restrict__ src, int nvec, int tid) {
#pragma unroll
  for (int v = 0; v < NV_MAX; ++v) reg[v] = src[min(tid + v * 256, nvec - 1)];
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
// the updated C_p is written back and the right-hand side is the updated G_p
// (the first DictOCSC iterate, from V = Theta = 0).  With rfold (warm start)
// the right-hand side is instead the carried G + rho_d (F(V) - Theta), which
// the fold advances by the same increments as G and writes back.
// dout == nullptr: fold only.
// ---------------------------------------------------------------------------
template <typename T, int KT, int FPB>
__global__ __launch_bounds__(256, 3) void k_dict_sweep(T* __restrict__ Cm, cx<T>* __restrict__ G,
                                                    const cx<T>* __restrict__ rhs,
                                                    const cx<T>* __restrict__ Zh,
                                                    const cx<T>* __restrict__ xh, int nfold,
                                                    cx<T>* __restrict__ rfold,
                                                    cx<T>* __restrict__ dout,
                                                    int K_, int Pf, int fpb_, int fs_, int slots_per_wg,
                                                    int reverse) {
  // KT > 0: K and fpb fixed at compile time (the arguments then equal them)
  constexpr bool CT = KT > 0;
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
  const int s_begin = run * slots_per_wg;
  const int s_end = min(nslots, s_begin + slots_per_wg);
  const int nvec = (int)((size_t)fpb * fs * sizeof(T) / 16);
  const bool plain = dout && nfold == 0;
  v4f reg[NVM];

  auto slot_of = [&](int s) { return reverse ? nslots - 1 - s : s; };
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
    if (plain) {
      // d_p replaces its right-hand side in the run buffer (p - f0 < slots_per_wg * fpb)
      cx<T>* xr = rb + (size_t)(p - f0) * K;
      if constexpr (CT) {
        const cx<T>* const xs[1] = {xr};
        cx<T>* const ys[1] = {xr};
        herm_matvec_ct<T, KT, 256 / FPB, 1>(R, xs, ys, rpart, lt);
      } else {
        herm_matvec<T>(R, K, ld, xr, xr, rpart, lt, tpg, ns);
      }
    } else if (nfold == 1) {
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
      v4f* dst = reinterpret_cast<v4f*>(Cm + (size_t)sl * fpb * fs);
      const v4f* srcv = reinterpret_cast<const v4f*>(Rall);
      for (int e = tid; e < nv; e += 256) dst[e] = srcv[e];
    } else {
      // several samples, folded one after another in sample order
      cx<T> dsum = mk<T>(0, 0);
      for (int b = 0; b < nfold; ++b) {
        if (ok && lt < K) {
          const cx<T> u = cconj<T>(Zh[((size_t)b * K + lt) * Pf + p]);
          const cx<T> du = cmul<T>(u, xh[(size_t)b * Pf + p]);
          xv[lt] = u;
          G[(size_t)lt * Pf + p] = cadd<T>(G[(size_t)lt * Pf + p], du);
          dsum = cadd<T>(dsum, du);
        }
        __syncthreads();
        herm_matvec<T>(R, K, ld, xv, vv, part, lt, tpg, ns);
        T acc = 0;
        if (lt < K) acc = xv[lt].x * vv[lt].x + xv[lt].y * vv[lt].y;   // Re(u^H v)
        acc = group_sum<T>(acc, tpg, wsum);
        herm_rank1<T>(R, K, ld, vv, (T)1 / ((T)1 + acc), lt, tpg, ns);
      }
      v4f* dst = reinterpret_cast<v4f*>(Cm + (size_t)sl * fpb * fs);
      const v4f* srcv = reinterpret_cast<const v4f*>(Rall);
      for (int e = tid; e < nv; e += 256) dst[e] = srcv[e];
      if (rfold && ok && lt < K) {
        const cx<T> rn = cadd<T>(rfold[(size_t)lt * Pf + p], dsum);
        rfold[(size_t)lt * Pf + p] = rn;
        if (dout) xv[lt] = rn;
      } else if (dout && ok && lt < K) {
        xv[lt] = G[(size_t)lt * Pf + p];
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

// ---------------------------------------------------------------------------
// V-step (Proposition 2) by separable pruned DFTs, in two kernels over
// (column block vb of VB spectrum columns, filter k).
//
// k_vstep_alpha: partial sums over the block's columns of
//   alpha_k[m][n] = (1/P) Re sum_{u, v} c_v X[u][v] e^{+2 pi i (u m/PH + v n/PW)},
//   X = d_k + Theta_k,  c_v = 1 at v = 0, PW/2 and 2 otherwise,
// i.e. the crop of the real inverse DFT of a Hermitian spectrum.
// ---------------------------------------------------------------------------
// Columns per block: one 128-byte line of complex values (16 FP32, 8 FP64).
template <typename T> __host__ __device__ constexpr int vblock() { return 128 / (int)(2 * sizeof(T)); }
constexpr int MAXF = 128;   // filter extent bound (filt <= pad <= 128)

template <typename T>
__global__ __launch_bounds__(256) void k_vstep_alpha(const cx<T>* __restrict__ d,
                                                     const cx<T>* __restrict__ Th, T* __restrict__ apart,
                                                     const cx<T>* __restrict__ twH,
                                                     const cx<T>* __restrict__ twW, int PH, int PW,
                                                     int Mh, int Mw, int first) {
  constexpr int VB = vblock<T>();
  __shared__ cx<T> X[MAXF * VB];
  __shared__ cx<T> t[2 * MAXF * VB];
  __shared__ cx<T> sH[MAXF], sW[MAXF];
  const int WC = PW / 2 + 1, Pf = PH * WC;
  const int vb = blockIdx.x, k = blockIdx.y, nvb = gridDim.x;
  const int v0 = vb * VB, nv = min(VB, WC - v0);
  const int tid = threadIdx.x;
  for (int i = tid; i < PH; i += 256) sH[i] = twH[i];
  for (int i = tid; i < PW; i += 256) sW[i] = twW[i];
  const cx<T>* dk = d + (size_t)k * Pf;
  const cx<T>* tk = Th + (size_t)k * Pf;
  constexpr int NQ = MAXF * VB / 256;
  cx<T> xd[NQ], xt[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {   // all loads issued before any use
    const int e = tid + q * 256, u = e / VB, c = e % VB;
    xd[q] = mk<T>(0, 0);
    xt[q] = mk<T>(0, 0);
    if (e < PH * VB && c < nv) {
      xd[q] = dk[u * WC + v0 + c];
      if (!first) xt[q] = tk[u * WC + v0 + c];
    }
  }
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int e = tid + q * 256;
    if (e < PH * VB) X[e] = cadd<T>(xd[q], xt[q]);
  }
  __syncthreads();
  // t[m][c] = sum_u X[u][c] e^{+2 pi i u m / PH}, the u-sum split over two threads
  const int HU = PH / 2;
  for (int e = tid; e < 2 * Mh * VB; e += 256) {
    const int hh = e / (Mh * VB), mc = e % (Mh * VB);
    const int m = mc / VB, c = mc % VB;
    T ar = 0, ai = 0;
    for (int u = hh * HU; u < (hh + 1) * HU; ++u) {
      const cx<T> w = sH[(u * m) & (PH - 1)];   // e^{-2 pi i um/PH}; use its conjugate
      const cx<T> x = X[u * VB + c];
      ar += x.x * w.x + x.y * w.y;
      ai += x.y * w.x - x.x * w.y;
    }
    t[e] = mk<T>(ar, ai);
  }
  __syncthreads();
  for (int e = tid; e < Mh * VB; e += 256) t[e] = cadd<T>(t[e], t[Mh * VB + e]);
  __syncthreads();
  const T invP = (T)1 / (T)(PH * PW);
  T* out = apart + ((size_t)k * nvb + vb) * Mh * Mw;
  for (int e = tid; e < Mh * Mw; e += 256) {
    const int m = e / Mw, n = e % Mw;
    T acc = 0;
    for (int c = 0; c < nv; ++c) {
      const int v = v0 + c;
      const T cv = (v == 0 || 2 * v == PW) ? (T)1 : (T)2;
      const cx<T> w = sW[(v * n) & (PW - 1)];
      const cx<T> tv = t[m * VB + c];
      acc += cv * (tv.x * w.x + tv.y * w.y);   // Re(t * conj(w))
    }
    out[e] = acc * invP;
  }
}

// k_vstep_apply: alpha_k = sum of the partials; V_k = alpha_k / max(||alpha_k||, 1);
// for the block's columns Vh = F(zero-pad V_k) by separable pruned DFTs, then
//   Theta <- Theta + d - Vh  (Theta = 0 on entry when first),
//   rhs   <- G + rho_d (Vh - Theta)   (right-hand side of the next D-step).
template <typename T>
__global__ __launch_bounds__(256) void k_vstep_apply(const cx<T>* __restrict__ d, cx<T>* __restrict__ Th,
                                                     const cx<T>* __restrict__ G, cx<T>* __restrict__ rhs,
                                                     const T* __restrict__ apart, T* __restrict__ V,
                                                     const cx<T>* __restrict__ twH,
                                                     const cx<T>* __restrict__ twW, int PH, int PW,
                                                     int Mh, int Mw, T rho_d, int first) {
  constexpr int VB = vblock<T>();
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* alpha = reinterpret_cast<T*>(smem_raw);                        // [Mh*Mw]
  cx<T>* rr = reinterpret_cast<cx<T>*>(smem_raw + (((size_t)Mh * Mw * sizeof(T) + 15) & ~(size_t)15));
  __shared__ T red[256];
  __shared__ cx<T> sH[MAXF], sW[MAXF];
  const int WC = PW / 2 + 1, Pf = PH * WC;
  const int vb = blockIdx.x, k = blockIdx.y, nvb = gridDim.x;
  const int v0 = vb * VB, nv = min(VB, WC - v0);
  const int tid = threadIdx.x;
  const int MM = Mh * Mw;
  for (int i = tid; i < PH; i += 256) sH[i] = twH[i];
  for (int i = tid; i < PW; i += 256) sW[i] = twW[i];
  const T* ap = apart + (size_t)k * nvb * MM;
  T ss = 0;
  for (int e = tid; e < MM; e += 256) {
    T a = 0;
#pragma unroll 8
    for (int j = 0; j < nvb; ++j) a += ap[(size_t)j * MM + e];
    alpha[e] = a;
    ss += a * a;
  }
  red[tid] = ss;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (tid < s) red[tid] += red[tid + s];
    __syncthreads();
  }
  const T nrm = sqrt(red[0]);
  const T scale = (T)1 / (nrm > (T)1 ? nrm : (T)1);
  for (int e = tid; e < MM; e += 256) {
    const T vval = alpha[e] * scale;
    alpha[e] = vval;
    if (vb == 0) V[(size_t)k * MM + e] = vval;
  }
  __syncthreads();
  // rr[m][c] = sum_n V[m][n] e^{-2 pi i v n / PW}
  for (int e = tid; e < Mh * VB; e += 256) {
    const int m = e / VB, c = e % VB;
    T ar = 0, ai = 0;
    if (c < nv) {
      const int v = v0 + c;
      for (int n = 0; n < Mw; ++n) {
        const cx<T> w = sW[(v * n) & (PW - 1)];
        const T x = alpha[m * Mw + n];
        ar += x * w.x;
        ai += x * w.y;
      }
    }
    rr[e] = mk<T>(ar, ai);
  }
  __syncthreads();
  const size_t base = (size_t)k * Pf;
  constexpr int NQ = MAXF * VB / 256;
  cx<T> dq[NQ], tq[NQ], gq[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {   // all loads issued before any use
    const int e = tid + q * 256, u = e / VB, c = e % VB;
    dq[q] = tq[q] = gq[q] = mk<T>(0, 0);
    if (e < PH * VB && c < nv) {
      const size_t idx = base + (size_t)u * WC + v0 + c;
      dq[q] = d[idx];
      if (!first) tq[q] = Th[idx];
      gq[q] = G[idx];
    }
  }
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int e = tid + q * 256, u = e / VB, c = e % VB;
    if (e >= PH * VB || c >= nv) continue;
    T ar = 0, ai = 0;
    for (int m = 0; m < Mh; ++m) {
      const cx<T> w = sH[(u * m) & (PH - 1)];
      const cx<T> x = rr[m * VB + c];
      ar += x.x * w.x - x.y * w.y;
      ai += x.x * w.y + x.y * w.x;
    }
    const size_t idx = base + (size_t)u * WC + v0 + c;
    const cx<T> th = mk<T>(tq[q].x + dq[q].x - ar, tq[q].y + dq[q].y - ai);
    Th[idx] = th;
    rhs[idx] = mk<T>(gq[q].x + rho_d * (ar - th.x), gq[q].y + rho_d * (ai - th.y));
  }
}

// ---------------------------------------------------------------------------
// Fused V-step (Proposition 2), one workgroup per filter k, for filters of at
// most VF x VF taps.  With X = d_k + Theta_k held in LDS:
//   t[m][v]  = sum_u X[u][v] e^{+2 pi i u m / PH}                   (m < M_h)
//   alpha    = (1/P) Re sum_v c_v t[m][v] e^{+2 pi i v n / PW}        (the crop of
//              the real inverse DFT; c_v = 1 at v = 0, PW/2 and 2 otherwise)
//   V_k      = alpha / max(||alpha||, 1)
//   r[m][v]  = sum_n V_k[m][n] e^{-2 pi i v n / PW};  F(V)[u][v] = sum_m r[m][v] e^{-2 pi i u m / PH}
//   Theta   <- X - F(V)  (= Theta + d - F(V));  rhs <- G + rho_d (F(V) - Theta)
// No other workgroup is involved, so the whole step is one launch.
// ---------------------------------------------------------------------------
constexpr int VF = 16;

template <typename T, int PH, int PW, int NT, int NQ>
__global__ __launch_bounds__(NT) void k_vstep_filter(const cx<T>* __restrict__ d, cx<T>* __restrict__ Th,
                                                     const cx<T>* __restrict__ G, cx<T>* __restrict__ rhs,
                                                     T* __restrict__ V, const cx<T>* __restrict__ twH,
                                                     const cx<T>* __restrict__ twW, int Mh, int Mw, T rho_d,
                                                     int first) {
  using Gm = PlaneGeom<PH, PW>;
  constexpr int WC = Gm::WC, PF = Gm::PF;
  constexpr int FPT = (PF + NT - 1) / NT;   // frequencies per thread in the update
  __shared__ __align__(16) cx<T> X[PF];
  __shared__ cx<T> tq[NQ * VF * WC];       // partial t over u-quarters; later r
  __shared__ cx<T> sH[PH], sW[PW];
  __shared__ T al[VF * VF];
  __shared__ T red[NT / 64];
  const int k = blockIdx.x, tid = threadIdx.x;
  const size_t base = (size_t)k * PF;
  // G of this thread's frequencies is fetched now and used at the end
  cx<T> gq[FPT];
#pragma unroll
  for (int j = 0; j < FPT; ++j) {
    const int e = min(tid + j * NT, PF - 1);
    gq[j] = G[base + e];
  }
  load_tables<PH, PW, T>(sH, sW, twH, twW, tid, NT);
  {
    cx<T> dq[FPT], tqv[FPT];
#pragma unroll
    for (int j = 0; j < FPT; ++j) {
      const int e = min(tid + j * NT, PF - 1);
      dq[j] = d[base + e];
      tqv[j] = first ? mk<T>(0, 0) : Th[base + e];
    }
#pragma unroll
    for (int j = 0; j < FPT; ++j) {
      const int e = tid + j * NT;
      if (PF % NT == 0 || e < PF) X[e] = cadd<T>(dq[j], tqv[j]);
    }
  }
  __syncthreads();
  // t over NQ slices of u
  constexpr int US = PH / NQ;
  for (int task = tid; task < NQ * Mh * WC; task += NT) {
    const int q = task / (Mh * WC), r = task - q * (Mh * WC);
    const int m = r / WC, v = r - m * WC;
    T ar = 0, ai = 0;
#pragma unroll 8
    for (int u = q * US; u < (q + 1) * US; ++u) {
      const cx<T> w = sH[(u * m) & (PH - 1)];   // e^{-2 pi i um/PH}; its conjugate is used
      const cx<T> x = X[u * WC + v];
      ar += x.x * w.x + x.y * w.y;
      ai += x.y * w.x - x.x * w.y;
    }
    tq[(q * VF + m) * WC + v] = mk<T>(ar, ai);
  }
  __syncthreads();
  const T invP = (T)1 / (T)(PH * PW);
  T ss = 0;
  for (int task = tid; task < Mh * Mw; task += NT) {
    const int m = task / Mw, n = task - m * Mw;
    T acc = 0;
    for (int v = 0; v < WC; ++v) {
      cx<T> tv = tq[m * WC + v];
#pragma unroll
      for (int q = 1; q < NQ; ++q) tv = cadd<T>(tv, tq[(q * VF + m) * WC + v]);
      const cx<T> w = sW[(v * n) & (PW - 1)];
      const T cv = (v == 0 || 2 * v == PW) ? (T)1 : (T)2;
      acc += cv * (tv.x * w.x + tv.y * w.y);   // Re(t * conj(w))
    }
    acc *= invP;
    al[task] = acc;
    ss += acc * acc;
  }
  for (int off = 32; off > 0; off >>= 1) ss += __shfl_xor(ss, off, 64);
  if ((tid & 63) == 0) red[tid >> 6] = ss;
  __syncthreads();
  T nrm2 = 0;
#pragma unroll
  for (int w = 0; w < NT / 64; ++w) nrm2 += red[w];
  const T nrm = sqrt(nrm2);
  const T scale = (T)1 / (nrm > (T)1 ? nrm : (T)1);
  for (int task = tid; task < Mh * Mw; task += NT) {
    const T vv = al[task] * scale;
    al[task] = vv;
    V[(size_t)k * Mh * Mw + task] = vv;
  }
  __syncthreads();
  // r[m][v] = sum_n V[m][n] e^{-2 pi i v n / PW}   (into tq)
  for (int task = tid; task < Mh * WC; task += NT) {
    const int m = task / WC, v = task - m * WC;
    T ar = 0, ai = 0;
    for (int n = 0; n < Mw; ++n) {
      const cx<T> w = sW[(v * n) & (PW - 1)];
      const T x = al[m * Mw + n];
      ar += x * w.x;
      ai += x * w.y;
    }
    tq[m * WC + v] = mk<T>(ar, ai);
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < FPT; ++j) {
    const int e = tid + j * NT;
    if (PF % NT != 0 && e >= PF) continue;
    const int u = e / WC, v = e - u * WC;
    T ar = 0, ai = 0;
    for (int m = 0; m < Mh; ++m) {
      const cx<T> w = sH[(u * m) & (PH - 1)];
      const cx<T> x = tq[m * WC + v];
      ar += x.x * w.x - x.y * w.y;
      ai += x.x * w.y + x.y * w.x;
    }
    const cx<T> xv = X[e];
    const cx<T> th = mk<T>(xv.x - ar, xv.y - ai);
    Th[base + e] = th;
    rhs[base + e] = mk<T>(gq[j].x + rho_d * (ar - th.x), gq[j].y + rho_d * (ai - th.y));
  }
}

// ---------------------------------------------------------------------------
// Objective (eq. csc) through Parseval: per sample b
//   sum_p c_v |x_p - sum_k Dh_k(p) Uh_bk(p)|^2 / P  and  sum |U_b|,
// accumulated in double.  Partials per block, then a final reduction.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_obj_resid(const cx<T>* __restrict__ xh, const cx<T>* __restrict__ Dh,
                                                   const cx<T>* __restrict__ Uh, double* __restrict__ part,
                                                   int K, int PW, int Pf) {
  __shared__ double red[256];
  const int WC = PW / 2 + 1;
  const int b = blockIdx.y;
  const int p = blockIdx.x * 256 + threadIdx.x;
  double acc = 0;
  if (p < Pf) {
    cx<T> r = xh[(size_t)b * Pf + p];
    for (int k = 0; k < K; ++k) r = csub<T>(r, cmul<T>(Dh[(size_t)k * Pf + p], Uh[((size_t)b * K + k) * Pf + p]));
    const int v = p % WC;
    const double cv = (v == 0 || 2 * v == PW) ? 1.0 : 2.0;
    acc = cv * ((double)r.x * r.x + (double)r.y * r.y);
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[(size_t)b * gridDim.x + blockIdx.x] = red[0];
}

template <typename T>
__global__ __launch_bounds__(256) void k_abs_sum(const T* __restrict__ U, double* __restrict__ part, long n) {
  __shared__ double red[256];
  const int b = blockIdx.y;
  const T* u = U + (size_t)b * n;
  double acc = 0;
  for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long)gridDim.x * 256) acc += fabs((double)u[i]);
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[(size_t)b * gridDim.x + blockIdx.x] = red[0];
}

__global__ void k_obj_final(const double* __restrict__ rpart, int nr, const double* __restrict__ lpart, int nl,
                            double* __restrict__ out, double invP, double lam, int terms) {
  __shared__ double a[256], c[256];
  const int b = blockIdx.x;
  double s1 = 0, s2 = 0;
  for (int i = threadIdx.x; i < nr; i += 256) s1 += rpart[(size_t)b * nr + i];
  for (int i = threadIdx.x; i < nl; i += 256) s2 += lpart[(size_t)b * nl + i];
  a[threadIdx.x] = s1;
  c[threadIdx.x] = s2;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      a[threadIdx.x] += a[threadIdx.x + s];
      c[threadIdx.x] += c[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    if (terms) {
      out[2 * b] = 0.5 * a[0] * invP;
      out[2 * b + 1] = c[0];
    } else {
      out[b] = 0.5 * a[0] * invP + lam * c[0];
    }
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

template <typename T>
__global__ void k_fill_zero(T* __restrict__ x, size_t n) {
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) x[e] = (T)0;
}

}  // namespace ocsc
