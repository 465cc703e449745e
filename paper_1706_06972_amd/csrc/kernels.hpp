// kernels.hpp -- gfx950 kernels of the OCSC hot path (templated on the real type).
//
// Layouts in HBM (Pf = PH * (PW/2+1) stored frequencies, P = PH * PW):
//   spectra     cx[plane][Pf]          plane = b*K + k (codes) or k (dictionary)
//   real planes T[plane][PH][PW]
//   inverse C   T[Pf][K][K]            R-form: R[i][j] = Re C_ij (j >= i),
//                                              R[j][i] = Im C_ij (j > i)
#pragma once
#include "common.hpp"
#include "dstep.hpp"
#include "vstep.hpp"

// the code-update bodies below compute the same bits wherever they are inlined
#pragma clang fp contract(off)

namespace ocsc {

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

// The twiddle tables through registers: fetch() issues their loads first, and
// put() writes them to LDS after the plane's own loads have been issued, so
// that waiting for the tables does not wait for those loads, and the two
// fetches take one memory round trip instead of two.
template <typename T, int PH, int PW, int NT>
struct TableStage {
  static constexpr int NH = (PH + NT - 1) / NT, NW = (PW + NT - 1) / NT;
  T hx[NH], hy[NH], wx[NW], wy[NW];   // real and imaginary parts apart: kept in registers
  __device__ __forceinline__ void fetch(const cx<T>* __restrict__ twH, const cx<T>* __restrict__ twW, int tid) {
#pragma unroll
    for (int i = 0; i < NH; ++i)
      if (PH % NT == 0 || tid + i * NT < PH) {
        const cx<T> v = twH[tid + i * NT];
        hx[i] = v.x;
        hy[i] = v.y;
      }
#pragma unroll
    for (int i = 0; i < NW; ++i)
      if (PW % NT == 0 || tid + i * NT < PW) {
        const cx<T> v = twW[tid + i * NT];
        wx[i] = v.x;
        wy[i] = v.y;
      }
  }
  __device__ __forceinline__ void put(cx<T>* sH, cx<T>* sW, int tid) const {
#pragma unroll
    for (int i = 0; i < NH; ++i)
      if (PH % NT == 0 || tid + i * NT < PH) sH[tid + i * NT] = mk<T>(hx[i], hy[i]);
#pragma unroll
    for (int i = 0; i < NW; ++i)
      if (PW % NT == 0 || tid + i * NT < PW) sW[tid + i * NT] = mk<T>(wx[i], wy[i]);
  }
};

// ---------------------------------------------------------------------------
// Code update, spatial half of one ADMM iteration, one workgroup per plane:
//   Y = Re F^-1(Zh);  U = S_kappa(Y + W);  W <- Y + W - U;  S = F(U - W).
// first: W = 0 on entry.  last: write U to Uout (if non-null) and stop.
// The body serves plane q with the workgroup's LDS buf (PH * LDW complex)
// and tables sH, sW; the caller separates successive planes by a barrier.
// ---------------------------------------------------------------------------
template <typename T, int PH, int PW, int NT>
__device__ __forceinline__ void code_plane_body(cx<T>* buf, cx<T>* sH, cx<T>* sW, long q,
                                                const cx<T>* __restrict__ Zh, T* __restrict__ W,
                                                cx<T>* __restrict__ S, T* __restrict__ Uout,
                                                const cx<T>* __restrict__ twH, const cx<T>* __restrict__ twW,
                                                T kappa, int first, int last) {
  using G = PlaneGeom<PH, PW>;
  using IO = PlaneIO<T, PH, PW, NT>;
  constexpr int VR = IO::VR, CR = IO::CR, NRV = IO::NRV;
  const int tid = threadIdx.x;
  TableStage<T, PH, PW, NT> tab;
  tab.fetch(twH, twW, tid);
  IO::spec_in(buf, Zh + q * G::PF, tid);
  // the dual W of this plane is fetched while the inverse transform runs
  v4f* wv = reinterpret_cast<v4f*>(W + q * G::P);
  v4f wr[CR];
  if (first) {   // outside the loop, so that the loads are not waited for one by one
#pragma unroll
    for (int j = 0; j < CR; ++j) wr[j] = v4f{0, 0, 0, 0};
  } else {
#pragma unroll
    for (int j = 0; j < CR; ++j) {
      const int e = tid + j * NT;
      if (NRV % NT == 0 || e < NRV) wr[j] = wv[e];
    }
  }
  tab.put(sH, sW, tid);
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
        const T v0 = fma(y.x, scale, w[2 * h]), v1 = fma(y.y, scale, w[2 * h + 1]);
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

template <typename T, int PH, int PW, int NT>
__global__ __launch_bounds__(NT) void k_code_plane(const cx<T>* __restrict__ Zh, T* __restrict__ W,
                                                   cx<T>* __restrict__ S, T* __restrict__ Uout,
                                                   const cx<T>* __restrict__ twH,
                                                   const cx<T>* __restrict__ twW, T kappa, int first,
                                                   int last) {
  __shared__ __align__(16) cx<T> buf[PH * PlaneGeom<PH, PW>::LDW];
  __shared__ cx<T> sH[PH], sW[PW];
  code_plane_body<T, PH, PW, NT>(buf, sH, sW, (long)blockIdx.x, Zh, W, S, Uout, twH, twW, kappa, first, last);
}

// ---------------------------------------------------------------------------
// The same step with each plane split over F workgroups by row residue
// (workgroup e = 0 .. F-1 takes rows r = F m + e): for batches too small to
// fill the chip with one workgroup per plane (F = 2), and for planes too
// large for one workgroup's LDS (256 and 512 grids: F = 2 to 16, so that a
// slice of PH/F rows fits).  A column DFT of length PH is one radix-F step
// over F DFTs of length PH/F on the rows of each residue (decimation in time):
//   forward  X[h] = sum_e w^{h e} E_e[h mod PH/F],  w = e^{-2 pi i/PH};
//   inverse  rows F m + e of the inverse column DFT of Y are the inverse
//            DFTs of length PH/F of
//            conj(w^{h' e}) sum_j Y[h' + j PH/F] e^{+2 pi i j e/F}.
// Workgroup e forms its length-PH/F spectrum from Zh on the way into LDS,
// runs the transforms of its PH/F rows, the U-step and the dual on them, and
// writes E_e (the column DFTs of length PH/F of its rows of U - W) to rows
// [e PH/F, (e + 1) PH/F) of the plane's slot of S.  The Z-step forms
// F(U - W) from E_0 .. E_{F-1} (zstep_body with SPLIT).
// ---------------------------------------------------------------------------
// Row residues per plane: 2 on one-pass grids, else the fewest whose slice
// (and the twiddle tables) fits in 150 KB of LDS.
__host__ __device__ constexpr int split_rows(int real_bytes, int ph, int pw) {
  int f = 2;
  if (ph > 128 || pw > 128)
    while (f < 16 && (long)(ph / f) * (pw / 2 + 1) * 2 * real_bytes + (long)(ph + pw) * 2 * real_bytes > 150 * 1024)
      f *= 2;
  return f;
}

// 2-D transforms of one row residue of a PH x PW plane (PHS = PH/F rows):
// column DFTs of length PHS, with twH the length-PH table read at stride F.
template <int PHS, int F, int PW, int NT, typename T>
__device__ void rfft2_slice_lds(cx<T>* buf, const cx<T>* twH, const cx<T>* twW, int tid) {
  constexpr int WC = PW / 2 + 1;
  rows_r2c_lds<PHS, PW, NT, T>(buf, twW, tid);
  fft_lines<PHS, WC, 1, WC, F, true, false, NT, T>(buf, twH, tid);
}

template <int PHS, int F, int PW, int NT, typename T>
__device__ void irfft2_slice_lds(cx<T>* buf, const cx<T>* twH, const cx<T>* twW, int tid) {
  constexpr int WC = PW / 2 + 1;
  fft_lines<PHS, WC, 1, WC, F, true, true, NT, T>(buf, twH, tid);
  rows_c2r_lds<PHS, PW, NT, T>(buf, twW, tid);
}

// v * e^{+2 pi i k/16}, 0 <= k < 16 (exact for k a multiple of 4)
template <typename T>
__device__ __forceinline__ cx<T> rot16_inv(cx<T> v, int k) {
  const cx<T> r = rot16<true, T>(v, k & 7);
  return k < 8 ? r : mk<T>(-r.x, -r.y);
}

template <typename T, int PH, int PW, int NT>
__device__ __forceinline__ void code_plane_split_body(cx<T>* buf, cx<T>* sH, cx<T>* sW, long q, int e,
                                                      const cx<T>* __restrict__ Zh, T* __restrict__ W,
                                                      cx<T>* __restrict__ S, T* __restrict__ Uout,
                                                      const cx<T>* __restrict__ twH,
                                                      const cx<T>* __restrict__ twW, T kappa, int first,
                                                      int last) {
  using G = PlaneGeom<PH, PW>;
  constexpr int F = split_rows((int)sizeof(T), PH, PW);
  constexpr int PHS = PH / F;
  constexpr int VR = 16 / (int)sizeof(T);    // reals per vector
  constexpr int CV = VR / 2;                 // complex values per vector
  static_assert((PHS * G::WC) % CV == 0, "slice spectrum in whole vectors");
  constexpr int NSV = PHS * G::WC / CV;      // vectors per slice spectrum
  constexpr int NRV = PHS * PW / VR;         // vectors per slice of the real plane
  constexpr int CS = (NSV + NT - 1) / NT, CR = (NRV + NT - 1) / NT;
  constexpr int U0 = 16 / F > 0 ? 16 / F : 1;
  constexpr int U = CS < U0 ? CS : U0;       // vectors per thread per round of spectrum loads
  constexpr int NR = (CS + U - 1) / U;       // rounds
  const int tid = threadIdx.x;
  TableStage<T, PH, PW, NT> tab;
  tab.fetch(twH, twW, tid);
  // spectrum rows h' + j PH/F (j < F) of the plane, U vectors per thread at a time
  const v4f* zs = reinterpret_cast<const v4f*>(Zh + q * G::PF);
  v4f zin[U][F];
  auto fetch = [&](int r) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int v = (r * U + u) * NT + tid;
      if (v < NSV) {
#pragma unroll
        for (int j = 0; j < F; ++j) zin[u][j] = zs[v + j * NSV];
      }
    }
  };
  fetch(0);
  // the dual on this workgroup's rows
  T* const Wq = W + q * G::P;
  v4f wr[CR];
  if (first) {   // outside the loop, so that the loads are not waited for one by one
#pragma unroll
    for (int j = 0; j < CR; ++j) wr[j] = v4f{0, 0, 0, 0};
  } else {
#pragma unroll
    for (int j = 0; j < CR; ++j) {
      const int v = tid + j * NT;
      if (NRV % NT == 0 || v < NRV) {
        const int i = v * VR, m = i / PW;
        wr[j] = *reinterpret_cast<const v4f*>(Wq + (F * m + e) * PW + i % PW);
      }
    }
  }
  tab.put(sH, sW, tid);
  __syncthreads();   // tables
  v4f* d = reinterpret_cast<v4f*>(buf);
#pragma unroll 1
  for (int r = 0; r < NR; ++r) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int v = (r * U + u) * NT + tid;
      if (v < NSV) {
        v4f o;
        cx<T>* oc = reinterpret_cast<cx<T>*>(&o);
#pragma unroll
        for (int c = 0; c < CV; ++c) {
          cx<T> acc = reinterpret_cast<const cx<T>*>(&zin[u][0])[c];
#pragma unroll
          for (int j = 1; j < F; ++j)
            acc = cadd<T>(acc, rot16_inv<T>(reinterpret_cast<const cx<T>*>(&zin[u][j])[c], (j * e * (16 / F)) & 15));
          oc[c] = e == 0 ? acc : cmulc<T>(acc, sH[(((v * CV + c) / G::WC) * e) % PH]);
        }
        d[v] = o;
      }
    }
    if (r + 1 < NR) fetch(r + 1);
  }
  __syncthreads();
  irfft2_slice_lds<PHS, F, PW, NT, T>(buf, sH, sW, tid);
  const T scale = (T)1 / (T)G::P;
#pragma unroll
  for (int j = 0; j < CR; ++j) {
    const int v = tid + j * NT;
    if (NRV % NT == 0 || v < NRV) {
      const int i = v * VR, m = i / PW, col = i % PW;
      cx<T>* o = buf + m * G::LDW + (col >> 1);
      T* w = reinterpret_cast<T*>(&wr[j]);
      v4f uo;
      T* u = reinterpret_cast<T*>(&uo);
#pragma unroll
      for (int h = 0; h < VR / 2; ++h) {
        const cx<T> y = o[h];
        const T v0 = fma(y.x, scale, w[2 * h]), v1 = fma(y.y, scale, w[2 * h + 1]);
        const T u0 = copysign(fmax(fabs(v0) - kappa, (T)0), v0);
        const T u1 = copysign(fmax(fabs(v1) - kappa, (T)0), v1);
        u[2 * h] = u0;
        u[2 * h + 1] = u1;
        w[2 * h] = v0 - u0;
        w[2 * h + 1] = v1 - u1;
        o[h] = mk<T>(u0 - w[2 * h], u1 - w[2 * h + 1]);
      }
      const long off = (long)(F * m + e) * PW + col;
      if (last) {
        if (Uout) *reinterpret_cast<v4f*>(Uout + q * G::P + off) = uo;
      } else {
        *reinterpret_cast<v4f*>(Wq + off) = wr[j];
      }
    }
  }
  if (last) return;
  __syncthreads();
  rfft2_slice_lds<PHS, F, PW, NT, T>(buf, sH, sW, tid);
  v4f* so = reinterpret_cast<v4f*>(S + q * G::PF + (long)e * PHS * G::WC);
  for (int v = tid; v < NSV; v += NT) so[v] = d[v];
}

// Block b of F n -> (plane q, residue e).  The F workgroups of a plane are
// eight blocks apart, so they run on the same XCD and the repeated reads of
// the plane's spectrum can come from its L2.  A bijection on [0, F n).
__device__ __forceinline__ void split_block(int b, int n, int F, int& q, int& e) {
  const int full = n >> 3;
  if (b < full * 8 * F) {
    q = (b / (8 * F)) * 8 + (b & 7);
    e = (b >> 3) % F;
  } else {
    const int t = b - full * 8 * F, r = n - full * 8;
    q = full * 8 + t % r;
    e = t / r;
  }
}

template <typename T, int PH, int PW, int NT>
__global__ __launch_bounds__(NT) void k_code_plane_split(const cx<T>* __restrict__ Zh, T* __restrict__ W,
                                                         cx<T>* __restrict__ S, T* __restrict__ Uout,
                                                         const cx<T>* __restrict__ twH,
                                                         const cx<T>* __restrict__ twW, T kappa, int first,
                                                         int last, int nplanes) {
  constexpr int F = split_rows((int)sizeof(T), PH, PW);
  __shared__ __align__(16) cx<T> buf[(PH / F) * PlaneGeom<PH, PW>::LDW];
  __shared__ cx<T> sH[PH], sW[PW];
  int q, e;
  split_block((int)blockIdx.x, nplanes, F, q, e);
  code_plane_split_body<T, PH, PW, NT>(buf, sH, sW, (long)q, e, Zh, W, S, Uout, twH, twW, kappa, first, last);
}

// ---------------------------------------------------------------------------
// Code update, frequency half of one ADMM iteration (the Z-step).  At each
// frequency p with a = Dh[:, p], s = S[:, p]:
//   z = s + conj(a) * gam_p * (x_p - a^T s),   gam_p = 1 / (rho + ||a||^2),
// which is the Sherman-Morrison solution of (conj(a) a^T + rho I) z =
// conj(a) x_p + rho s.  A workgroup of 16 * ZF threads serves ZF frequencies
// of SB consecutive samples: thread (kq, f) holds filters k = kq, kq + 16, ...
// (at most KPT) of frequency f in registers, so a wave reads 64 / ZF filter
// rows per load, each as one run of ZF complex values; the filter values are
// read once for the SB samples.  The sums over filters are taken in the same
// order for every ZF and SB (per thread over j, then over the 16 threads of a
// frequency in kq order), so every launch shape gives the same bits.
// first: s = 0.
// SPLIT: S holds, per plane, the column DFTs E_0 .. E_{F-1} of the split
// plane step (rows [e PH/F, (e + 1) PH/F)), and s = sum_e w^{h e} E_e[h']
// (h' = h mod PH/F) is formed here (twH[i] = e^{-2 pi i i/PH}, WC stored
// columns).  A workgroup then serves ZF/F frequencies in each of the F row
// blocks, at the same h' and column, which read the same E values.
// ---------------------------------------------------------------------------
// The body serves frequency block bx of sample block by with the LDS
// reduction buffer red (16 * (ZF + 1) complex).
template <typename T, int KPT, int ZF, int SB, bool SPLIT = false>
__device__ __forceinline__ void zstep_body(cx<T> (*red)[ZF + 1], int bx, int by, const cx<T>* __restrict__ Dh,
                                           const T* __restrict__ gam, const cx<T>* __restrict__ xh,
                                           const cx<T>* __restrict__ S, cx<T>* __restrict__ Zh, int K, int Pf,
                                           int B, int first, cx<T>* __restrict__ Zt, int ldt, int bt0,
                                           const cx<T>* __restrict__ twH = nullptr, int WC = 1, int F = 1) {
  // Zt (optional): the same values frequency-major, Zt[(p * ldt + bt0 + b) * K + k]
  const int f = threadIdx.x % ZF, kq = threadIdx.x / ZF;
  const int zb = ZF / F;              // SPLIT: frequencies per row block
  const int part = Pf / F;            // SPLIT: values per E_e
  const int jh = bx * zb + f % zb;    // SPLIT: index within E_e
  const int p = SPLIT ? jh + (f / zb) * part : bx * ZF + f;
  const bool ok = SPLIT ? jh < part : p < Pf;
  const int ph = Pf / WC, h = p / WC;
  const cx<T> tw1 = (SPLIT && ok) ? twH[h] : mk<T>(0, 0);   // w^h
  // gam_p and x~_p are read by the threads that finish the reduction; they
  // are fetched with the other loads, not after the barrier
  const bool fin = kq == 0 && ok;
  const T gp = fin ? gam[p] : (T)0;
  cx<T> a[KPT];
#pragma unroll
  for (int j = 0; j < KPT; ++j) {
    const int k = kq + j * 16;
    a[j] = (ok && k < K) ? Dh[(size_t)k * Pf + p] : mk<T>(0, 0);
  }
  for (int sb = 0; sb < SB; ++sb) {
    const int b = by * SB + sb;
    if (b >= B) break;   // the same for the whole workgroup
    const cx<T> xv = fin ? xh[(size_t)b * Pf + p] : mk<T>(0, 0);
    cx<T> s[KPT];
    if (SPLIT) {
      // every filter's E_0 and E_1 loads are issued before the first is used
      // (a wait per filter would make KPT memory round trips of one)
      cx<T> s1[KPT];
#pragma unroll
      for (int j = 0; j < KPT; ++j) {
        const int k = kq + j * 16;
        const bool v = ok && k < K && !first;
        const cx<T>* e0 = S + ((size_t)b * K + k) * Pf + jh;
        s[j] = v ? e0[0] : mk<T>(0, 0);
        s1[j] = v ? e0[part] : mk<T>(0, 0);
      }
#pragma unroll
      for (int j = 0; j < KPT; ++j) s[j] = cadd<T>(s[j], cmul<T>(s1[j], tw1));
      if (F > 2) {
        // one residue at a time, every filter's load issued before the first
        // is used (each filter still adds its terms in the order r = 2, 3, ..)
        for (int r = 2, i = h; r < F; ++r) {   // i = h r mod PH
          i += h;
          if (i >= ph) i -= ph;
          const cx<T> twr = ok ? twH[i] : mk<T>(0, 0);
          cx<T> er[KPT];
#pragma unroll
          for (int j = 0; j < KPT; ++j) {
            const int k = kq + j * 16;
            er[j] = (ok && k < K && !first) ? S[((size_t)b * K + k) * Pf + jh + (size_t)r * part] : mk<T>(0, 0);
          }
#pragma unroll
          for (int j = 0; j < KPT; ++j) {
            const int k = kq + j * 16;
            if (ok && k < K && !first) s[j] = cadd<T>(s[j], cmul<T>(er[j], twr));
          }
        }
      }
    } else {
#pragma unroll
      for (int j = 0; j < KPT; ++j) {
        const int k = kq + j * 16;
        s[j] = (ok && k < K && !first) ? S[((size_t)b * K + k) * Pf + p] : mk<T>(0, 0);
      }
    }
    cx<T> acc = mk<T>(0, 0);
#pragma unroll
    for (int j = 0; j < KPT; ++j) acc = cadd<T>(acc, cmul<T>(a[j], s[j]));
    red[kq][f] = acc;
    __syncthreads();
    if (kq == 0) {
      cx<T> tot = red[0][f];
#pragma unroll
      for (int i = 1; i < 16; ++i) tot = cadd<T>(tot, red[i][f]);
      cx<T> qv = mk<T>(0, 0);
      if (ok) qv = cscale<T>(csub<T>(xv, tot), gp);
      red[0][f] = qv;
    }
    __syncthreads();
    const cx<T> qv = red[0][f];
#pragma unroll
    for (int j = 0; j < KPT; ++j) {
      const int k = kq + j * 16;
      if (ok && k < K) {
        const cx<T> z = cadd<T>(s[j], cmulc<T>(qv, a[j]));
        Zh[((size_t)b * K + k) * Pf + p] = z;
        if (Zt) Zt[((size_t)p * ldt + bt0 + b) * K + k] = z;
      }
    }
    if (SB > 1) __syncthreads();   // red is reused by the next sample
  }
}

template <typename T, int KPT, int ZF, int SB, bool SPLIT>
__global__ __launch_bounds__(16 * ZF) void k_code_zstep(const cx<T>* __restrict__ Dh,
                                                        const T* __restrict__ gam,
                                                        const cx<T>* __restrict__ xh,
                                                        const cx<T>* __restrict__ S,
                                                        cx<T>* __restrict__ Zh, int K, int Pf, int B,
                                                        int first, cx<T>* __restrict__ Zt, int ldt, int bt0,
                                                        const cx<T>* __restrict__ twH, int WC, int F) {
  __shared__ cx<T> red[16][ZF + 1];
  // SPLIT: a block's runs in each E_e can be shorter than a cache line, so
  // neighbouring blocks go to the same XCD and share its L2
  const int bx = SPLIT ? xcd_block((int)blockIdx.x, (int)gridDim.x) : (int)blockIdx.x;
  zstep_body<T, KPT, ZF, SB, SPLIT>(red, bx, blockIdx.y, Dh, gam, xh, S, Zh, K, Pf, B, first, Zt, ldt, bt0, twH,
                                    WC, F);
}

// gam_p = 1 / (rho + sum_k |Dh[k][p]|^2): 64 frequencies per workgroup, the
// sum over filters split four ways so that a thread's loads are independent.
template <typename T>
__global__ __launch_bounds__(256) void k_gamma(const cx<T>* __restrict__ Dh, T* __restrict__ gam, T rho, int K,
                                               int Pf) {
  __shared__ T part[4][64];
  const int f = threadIdx.x & 63, sl = threadIdx.x >> 6;
  const int p = blockIdx.x * 64 + f;
  T acc = 0;
  if (p < Pf) {
#pragma unroll 5
    for (int k = sl; k < K; k += 4) {
      const cx<T> a = Dh[(size_t)k * Pf + p];
      acc += a.x * a.x + a.y * a.y;
    }
  }
  part[sl][f] = acc;
  __syncthreads();
  if (sl == 0 && p < Pf) gam[p] = (T)1 / (rho + ((part[0][f] + part[1][f]) + (part[2][f] + part[3][f])));
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

}  // namespace ocsc

#pragma clang fp contract(fast)
