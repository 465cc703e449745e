// bigplane.hpp -- plane transforms and the fused code-plane step for grids
// whose half spectrum does not fit in LDS (256 x 256 up to 512 x 512).
//
// A 2-D transform is split into a row pass and a column pass, each a launch
// over (block, plane) workgroups that stage their block in LDS:
//   row pass:    RB consecutive rows of one plane (real <-> half spectrum)
//   column pass: a block of CB spectrum columns of one plane, all PH rows
//                (CB complex = 128, 256 or 512 bytes per row segment)
// The code-plane step takes CB and RB from the context's launch shape; the
// per-column and per-row arithmetic does not depend on them.
// Spectra keep the layout of the small-grid path: cx[plane][PH][PW/2 + 1].
#pragma once
#include "common.hpp"

// the passes below compute the same bits wherever they are inlined
#pragma clang fp contract(off)

namespace ocsc {

constexpr int BIG_RB = 8;   // rows per row-pass workgroup of the sample and objective transforms
template <typename T> __host__ __device__ constexpr int big_cb() { return 128 / (int)(2 * sizeof(T)); }
// threads of a column-pass workgroup: PH / 16 (FP32) or PH / 32 (FP64) values each
template <typename T, int CB> __host__ __device__ constexpr int big_cols_nt() { return CB * 16 * (int)sizeof(T) / 4; }

// ---------------------------------------------------------------------------
// Column pass: length-PH DFT (forward or inverse, unnormalised) of columns
// [c0, c0 + CB) of each plane, src -> dst (may alias).  Columns past PW/2
// are computed on clamped copies and not stored.
// ---------------------------------------------------------------------------
// The body serves column block bx of plane q with LDS buf (PH * CB complex,
// buf[u * CB + c]) and table sH.
template <typename T, int PH, int PW, bool INV, int CB, int NT>
__device__ __forceinline__ void big_cols_body(cx<T>* buf, cx<T>* sH, int bx, long q, const cx<T>* __restrict__ src,
                                              cx<T>* __restrict__ dst, const cx<T>* __restrict__ twH) {
  constexpr int WC = PW / 2 + 1;
  constexpr int NE = PH * CB, EPT = (NE + NT - 1) / NT;
  static_assert(NE % NT == 0, "column block must be a multiple of the workgroup");
  const int tid = threadIdx.x;
  const int c0 = bx * CB;
  const size_t pb = (size_t)q * PH * WC;
  {
    // the table and the block are fetched together and stored after all
    // loads are issued (one memory round trip)
    constexpr int NTH = (PH + NT - 1) / NT;
    T thx[NTH], thy[NTH];   // real and imaginary parts apart: kept in registers
    cx<T> r[EPT];
#pragma unroll
    for (int i = 0; i < NTH; ++i)
      if (PH % NT == 0 || tid + i * NT < PH) {
        const cx<T> v = twH[tid + i * NT];
        thx[i] = v.x;
        thy[i] = v.y;
      }
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
      const int e = tid + j * NT;
      const int u = e / CB, c = min(c0 + (e % CB), WC - 1);
      r[j] = src[pb + (size_t)u * WC + c];
    }
#pragma unroll
    for (int i = 0; i < NTH; ++i)
      if (PH % NT == 0 || tid + i * NT < PH) sH[tid + i * NT] = mk<T>(thx[i], thy[i]);
#pragma unroll
    for (int j = 0; j < EPT; ++j) buf[tid + j * NT] = r[j];
  }
  __syncthreads();
  fft_lines<PH, CB, 1, CB, 1, true, INV, NT, T>(buf, sH, tid);
#pragma unroll
  for (int j = 0; j < EPT; ++j) {
    const int e = tid + j * NT;
    const int u = e / CB, c = c0 + (e % CB);
    if (c < WC) dst[pb + (size_t)u * WC + c] = buf[e];
  }
}

template <typename T, int PH, int PW, bool INV, int CB = big_cb<T>()>
__global__ __launch_bounds__((big_cols_nt<T, CB>())) void k_big_cols(const cx<T>* __restrict__ src,
                                                                  cx<T>* __restrict__ dst,
                                                                  const cx<T>* __restrict__ twH) {
  __shared__ __align__(16) cx<T> buf[PH * CB];
  __shared__ cx<T> sH[PH];
  big_cols_body<T, PH, PW, INV, CB, big_cols_nt<T, CB>()>(buf, sH, blockIdx.x, blockIdx.y, src, dst, twH);
}

// ---------------------------------------------------------------------------
// Row pass, forward: rows [r0, r0 + RB) of each real plane (an sh x sw block
// at (0, 0) of the zero PH x PW grid, row pitch sw, plane q at src + q *
// sstride) -> their half spectra (rows of dst + q * dstride).
// ---------------------------------------------------------------------------
template <typename T, int PH, int PW>
__global__ __launch_bounds__(256) void k_big_rows_fwd(const T* __restrict__ src, int sh, int sw, long sstride,
                                                      cx<T>* __restrict__ dst, long dstride,
                                                      const cx<T>* __restrict__ twW) {
  constexpr int M = PW / 2, WC = M + 1, NT = 256, RB = BIG_RB;
  __shared__ __align__(16) cx<T> buf[RB * WC];
  __shared__ cx<T> sW[PW];
  const int tid = threadIdx.x;
  const int r0 = blockIdx.x * RB;
  const long q = blockIdx.y;
  for (int i = tid; i < PW; i += NT) sW[i] = twW[i];
  const T* s = src + q * sstride;
  for (int e = tid; e < RB * M; e += NT) {
    const int rr = e / M, n = e % M, u = r0 + rr, c = 2 * n;
    T a = 0, b = 0;
    if (u < sh) {
      if (c < sw) a = s[(size_t)u * sw + c];
      if (c + 1 < sw) b = s[(size_t)u * sw + c + 1];
    }
    buf[rr * WC + n] = mk<T>(a, b);
  }
  __syncthreads();
  rows_r2c_lds<RB, PW, NT, T>(buf, sW, tid);
  cx<T>* d = dst + q * dstride + (size_t)r0 * WC;
  for (int e = tid; e < RB * WC; e += NT) d[e] = buf[e];
}

// ---------------------------------------------------------------------------
// Row pass, inverse with crop: rows of the column-inverted spectra -> real
// rows (with the 1/P factor), keeping the top-left oh x ow block of each
// plane (row pitch ow) at dst + q * dstride.  Row blocks past oh exit.
// ---------------------------------------------------------------------------
template <typename T, int PH, int PW>
__global__ __launch_bounds__(256) void k_big_rows_inv_crop(const cx<T>* __restrict__ src, long sstride,
                                                           T* __restrict__ dst, int oh, int ow, long dstride,
                                                           const cx<T>* __restrict__ twW) {
  constexpr int M = PW / 2, WC = M + 1, NT = 256, RB = BIG_RB;
  __shared__ __align__(16) cx<T> buf[RB * WC];
  __shared__ cx<T> sW[PW];
  const int tid = threadIdx.x;
  const int r0 = blockIdx.x * RB;
  const long q = blockIdx.y;
  if (r0 >= oh) return;
  for (int i = tid; i < PW; i += NT) sW[i] = twW[i];
  const cx<T>* s = src + q * sstride + (size_t)r0 * WC;
  for (int e = tid; e < RB * WC; e += NT) buf[e] = s[e];
  __syncthreads();
  rows_c2r_lds<RB, PW, NT, T>(buf, sW, tid);
  const T scale = (T)1 / (T)(PH * PW);
  T* d = dst + q * dstride;
  const int nr = min(RB, oh - r0);
  for (int e = tid; e < nr * ow; e += NT) {
    const int rr = e / ow, c = e % ow;
    const cx<T> v = buf[rr * WC + (c >> 1)];
    d[(size_t)(r0 + rr) * ow + c] = ((c & 1) ? v.y : v.x) * scale;
  }
}

// ---------------------------------------------------------------------------
// Code-plane row pass (eq. fcsc_code, U-step and dual) on rows [r0, r0 + RB)
// of plane q = b*K + k, after the column pass has inverted Zh into Y:
//   y = rows of Re F^-1(Zh);  U = S_kappa(y + W);  W <- W + y - U;
//   rows of (U - W) are transformed forward into S (the column pass then
//   completes S = F(U - W)).  On the last iteration only U is stored.
// W = 0 on entry when first.
// ---------------------------------------------------------------------------
// The body serves row block bx of plane q with LDS buf (RB * (PW/2 + 1)
// complex) and table sW.
template <typename T, int PH, int PW, int RB, int NT>
__device__ __forceinline__ void big_code_rows_body(cx<T>* buf, cx<T>* sW, int bx, size_t q,
                                                   const cx<T>* __restrict__ Y, T* __restrict__ W,
                                                   cx<T>* __restrict__ S, T* __restrict__ Uout,
                                                   const cx<T>* __restrict__ twW, T kappa, int first, int last) {
  constexpr int M = PW / 2, WC = M + 1;
  constexpr int NE = RB * WC, NR = RB * PW;
  const int tid = threadIdx.x;
  const int r0 = bx * RB;
  const size_t so = q * PH * WC + (size_t)r0 * WC;   // spectrum rows
  const size_t ro = q * PH * PW + (size_t)r0 * PW;   // real rows
  // the table and the rows are fetched into registers and stored after all
  // loads (with this thread's W values, used after the inverse) are issued
  constexpr int NTW = (PW + NT - 1) / NT, NEV = (NE + NT - 1) / NT;
  T twx[NTW], twy[NTW], yx[NEV], yy[NEV];   // real and imaginary parts apart: kept in registers
#pragma unroll
  for (int i = 0; i < NTW; ++i)
    if (PW % NT == 0 || tid + i * NT < PW) {
      const cx<T> v = twW[tid + i * NT];
      twx[i] = v.x;
      twy[i] = v.y;
    }
#pragma unroll
  for (int j = 0; j < NEV; ++j)
    if (NE % NT == 0 || tid + j * NT < NE) {
      const cx<T> v = Y[so + tid + j * NT];
      yx[j] = v.x;
      yy[j] = v.y;
    }
  constexpr int WPT = (NR + NT - 1) / NT;
  T wv[WPT];
#pragma unroll
  for (int j = 0; j < WPT; ++j) {
    const int e = tid + j * NT;
    wv[j] = (first || e >= NR) ? (T)0 : W[ro + min(e, NR - 1)];
  }
#pragma unroll
  for (int i = 0; i < NTW; ++i)
    if (PW % NT == 0 || tid + i * NT < PW) sW[tid + i * NT] = mk<T>(twx[i], twy[i]);
#pragma unroll
  for (int j = 0; j < NEV; ++j)
    if (NE % NT == 0 || tid + j * NT < NE) buf[tid + j * NT] = mk<T>(yx[j], yy[j]);
  __syncthreads();
  rows_c2r_lds<RB, PW, NT, T>(buf, sW, tid);
  const T scale = (T)1 / (T)(PH * PW);
  T tv[WPT];
#pragma unroll
  for (int j = 0; j < WPT; ++j) {
    const int e = tid + j * NT;
    if (NR % NT != 0 && e >= NR) continue;
    const int rr = e / PW, c = e % PW;
    const cx<T> v = buf[rr * WC + (c >> 1)];
    const T a = fma((c & 1) ? v.y : v.x, scale, wv[j]);   // y + W, y the inverse transform
    const T u = copysign(fmax(fabs(a) - kappa, (T)0), a);
    const T wn = a - u;   // W + y - U
    if (last) {
      if (Uout) Uout[ro + e] = u;
    } else {
      W[ro + e] = wn;
    }
    tv[j] = u - wn;
  }
  if (last) return;   // the codes are final; no further Z-step needs S
  __syncthreads();   // every thread has read its inverse values
#pragma unroll
  for (int j = 0; j < WPT; ++j) {
    const int e = tid + j * NT;
    if (NR % NT != 0 && e >= NR) continue;
    const int rr = e / PW, c = e % PW;
    T* slot = reinterpret_cast<T*>(&buf[rr * WC + (c >> 1)]);
    slot[c & 1] = tv[j];
  }
  __syncthreads();
  rows_r2c_lds<RB, PW, NT, T>(buf, sW, tid);
  for (int e = tid; e < NE; e += NT) S[so + e] = buf[e];
}

template <typename T, int PH, int PW, int RB = BIG_RB>
__global__ __launch_bounds__(256) void k_big_code_rows(const cx<T>* __restrict__ Y, T* __restrict__ W,
                                                       cx<T>* __restrict__ S, T* __restrict__ Uout,
                                                       const cx<T>* __restrict__ twW, T kappa, int first,
                                                       int last) {
  __shared__ __align__(16) cx<T> buf[RB * (PW / 2 + 1)];
  __shared__ cx<T> sW[PW];
  big_code_rows_body<T, PH, PW, RB, 256>(buf, sW, blockIdx.x, blockIdx.y, Y, W, S, Uout, twW, kappa, first, last);
}

}  // namespace ocsc

#pragma clang fp contract(fast)
