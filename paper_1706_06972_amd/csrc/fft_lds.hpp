// fft_lds.hpp -- LDS-resident 2-D real DFTs of small planes for gfx950.
//
// A plane of PH x PW reals lives in LDS as PH rows of PW/2+1 complex values
// (the non-redundant half spectrum, row pitch LDW).  The forward transform
// (R2C) runs a complex FFT of length PW/2 along each row on the packed pairs
// (x[2n], x[2n+1]), splits it into the half spectrum of the real row, then
// runs complex FFTs of length PH down the PW/2+1 columns.  The inverse (C2R)
// undoes these steps in reverse order; it is unnormalised and leaves
// P * (x[2n], x[2n+1]) in row r, slot n.
//
// Each 1-D FFT is a two-stage Stockham autosort transform with radices of at
// most 16; a stage reads R values per butterfly into registers, applies the
// stage twiddles, runs an in-register radix-R DFT and writes the results back
// to their Stockham positions.  All threads finish reading before any writes
// (one barrier in between), so a stage works in place.
//
// Floating-point contraction is off in this file and in the code-update
// bodies (kernels.hpp, bigplane.hpp): every fused multiply-add is written
// out, so a body computes the same bits wherever the compiler inlines it
// (separate kernels, launch shapes, the grouped persistent launch).
#pragma once
#include <hip/hip_runtime.h>

#pragma clang fp contract(off)

namespace ocsc {

template <typename T> struct cplx_t;
template <> struct cplx_t<float> { using type = float2; };
template <> struct cplx_t<double> { using type = double2; };
template <typename T> using cx = typename cplx_t<T>::type;

template <typename T> __device__ __forceinline__ cx<T> mk(T a, T b) { cx<T> r; r.x = a; r.y = b; return r; }
template <typename T> __device__ __forceinline__ cx<T> cadd(cx<T> a, cx<T> b) { return mk<T>(a.x + b.x, a.y + b.y); }
template <typename T> __device__ __forceinline__ cx<T> csub(cx<T> a, cx<T> b) { return mk<T>(a.x - b.x, a.y - b.y); }
template <typename T> __device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
  return mk<T>(fma(a.x, b.x, -(a.y * b.y)), fma(a.x, b.y, a.y * b.x));
}
// a * conj(b)
template <typename T> __device__ __forceinline__ cx<T> cmulc(cx<T> a, cx<T> b) {
  return mk<T>(fma(a.x, b.x, a.y * b.y), fma(a.y, b.x, -(a.x * b.y)));
}
template <typename T> __device__ __forceinline__ cx<T> cconj(cx<T> a) { return mk<T>(a.x, -a.y); }
template <typename T> __device__ __forceinline__ cx<T> cscale(cx<T> a, T s) { return mk<T>(a.x * s, a.y * s); }

// ---------------------------------------------------------------------------
// In-register DFT of size R in {2, 4, 8, 16}: radix-2 decimation in time with
// compile-time twiddles (16th roots of unity).  Sign: forward e^{-2 pi i/R}.
// ---------------------------------------------------------------------------
__device__ constexpr double kCos16[8] = {
    1.0, 0.92387953251128675613, 0.70710678118654752440, 0.38268343236508977173,
    0.0, -0.38268343236508977173, -0.70710678118654752440, -0.92387953251128675613};
__device__ constexpr double kSin16[8] = {
    0.0, 0.38268343236508977173, 0.70710678118654752440, 0.92387953251128675613,
    1.0, 0.92387953251128675613, 0.70710678118654752440, 0.38268343236508977173};

// v * w16^e with w16 = e^{-+2 pi i/16} (forward / inverse), 0 <= e < 8.
template <bool INV, typename T>
__device__ __forceinline__ cx<T> rot16(cx<T> v, int e) {
  if (e == 0) return v;
  if (e == 4) return INV ? mk<T>(-v.y, v.x) : mk<T>(v.y, -v.x);
  const T c = (T)kCos16[e];
  const T s = INV ? (T)kSin16[e] : -(T)kSin16[e];
  return mk<T>(fma(v.x, c, -(v.y * s)), fma(v.x, s, v.y * c));
}

__host__ __device__ constexpr int ilog2(int n) { return n <= 1 ? 0 : 1 + ilog2(n >> 1); }
__host__ __device__ constexpr int bitrev(int i, int bits) {
  int r = 0;
  for (int b = 0; b < bits; ++b) r |= ((i >> b) & 1) << (bits - 1 - b);
  return r;
}

template <int R, bool INV, typename T>
__device__ __forceinline__ void dft_reg(cx<T>* x) {
  constexpr int L = ilog2(R);
#pragma unroll
  for (int i = 0; i < R; ++i) {
    const int j = bitrev(i, L);
    if (j > i) { cx<T> t = x[i]; x[i] = x[j]; x[j] = t; }
  }
#pragma unroll
  for (int len = 2; len <= R; len <<= 1) {
#pragma unroll
    for (int i = 0; i < R; i += len) {
#pragma unroll
      for (int j = 0; j < len / 2; ++j) {
        cx<T> u = x[i + j];
        cx<T> v = rot16<INV, T>(x[i + j + len / 2], j * (16 / len));
        x[i + j] = cadd<T>(u, v);
        x[i + j + len / 2] = csub<T>(u, v);
      }
    }
  }
}

// Radix plans (two or three stages) for the 1-D lengths of the plane kernels.
template <int N> struct Plan;
template <> struct Plan<16> { static constexpr int R1 = 4, R2 = 4, R3 = 1; };
template <> struct Plan<32> { static constexpr int R1 = 8, R2 = 4, R3 = 1; };
template <> struct Plan<64> { static constexpr int R1 = 8, R2 = 8, R3 = 1; };
template <> struct Plan<128> { static constexpr int R1 = 16, R2 = 8, R3 = 1; };
template <> struct Plan<256> { static constexpr int R1 = 16, R2 = 16, R3 = 1; };
template <> struct Plan<512> { static constexpr int R1 = 8, R2 = 8, R3 = 8; };

// One Stockham stage of radix R on NLINES lines of length N in LDS.
// Element n of line l is buf[l * LSTR + n * ESTR].  L is the product of the
// radices of earlier stages.  tab[e * TS] = e^{-2 pi i e / N} for 0 <= e < N.
// LINE_FAST: consecutive threads take consecutive lines; otherwise
// consecutive butterflies of one line.  Both sweeps use LINE_FAST: along a
// row the lines are LDW complex apart, which spreads a wave over the banks.
template <int R, int N, int L, int NLINES, int LSTR, int ESTR, int TS, bool LINE_FAST, bool INV,
          int NT, typename T>
__device__ __forceinline__ void stockham_stage(cx<T>* buf, const cx<T>* tab, int tid) {
  constexpr int NB = N / R;
  constexpr int TASKS = NLINES * NB;
  constexpr int TPT = (TASKS + NT - 1) / NT;
  constexpr int TWS = N / (L * R);  // twiddle index step: w_{LR}^{rk} = w_N^{rk * TWS}
  cx<T> v[TPT][R];
#pragma unroll
  for (int q = 0; q < TPT; ++q) {
    const int task = tid + q * NT;
    if (TASKS % NT == 0 || task < TASKS) {
      const int line = LINE_FAST ? task % NLINES : task / NB;
      const int j = LINE_FAST ? task / NLINES : task % NB;
      const int k = j % L;
      cx<T>* base = buf + line * LSTR;
#pragma unroll
      for (int r = 0; r < R; ++r) v[q][r] = base[(j + r * NB) * ESTR];
      if (L > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          const cx<T> w = tab[(r * k * TWS) * TS];
          v[q][r] = INV ? cmulc<T>(v[q][r], w) : cmul<T>(v[q][r], w);
        }
      }
      dft_reg<R, INV, T>(v[q]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < TPT; ++q) {
    const int task = tid + q * NT;
    if (TASKS % NT == 0 || task < TASKS) {
      const int line = LINE_FAST ? task % NLINES : task / NB;
      const int j = LINE_FAST ? task / NLINES : task % NB;
      const int k = j % L;
      cx<T>* base = buf + line * LSTR;
      const int o = (j / L) * L * R + k;
#pragma unroll
      for (int s = 0; s < R; ++s) base[(o + s * L) * ESTR] = v[q][s];
    }
  }
  __syncthreads();
}

template <int N, int NLINES, int LSTR, int ESTR, int TS, bool LINE_FAST, bool INV, int NT, typename T>
__device__ __forceinline__ void fft_lines(cx<T>* buf, const cx<T>* tab, int tid) {
  constexpr int R1 = Plan<N>::R1, R2 = Plan<N>::R2, R3 = Plan<N>::R3;
  stockham_stage<R1, N, 1, NLINES, LSTR, ESTR, TS, LINE_FAST, INV, NT, T>(buf, tab, tid);
  stockham_stage<R2, N, R1, NLINES, LSTR, ESTR, TS, LINE_FAST, INV, NT, T>(buf, tab, tid);
  if constexpr (R3 > 1) stockham_stage<R3, N, R1 * R2, NLINES, LSTR, ESTR, TS, LINE_FAST, INV, NT, T>(buf, tab, tid);
}

// Geometry of a PH x PW real plane held as a half spectrum in LDS.
template <int PH, int PW> struct PlaneGeom {
  static constexpr int M = PW / 2;    // complex row length of the packed real row
  static constexpr int WC = M + 1;    // stored spectrum columns
  static constexpr int LDW = WC;      // LDS row pitch (complex elements)
  static constexpr int PF = PH * WC;  // stored frequencies
  static constexpr int P = PH * PW;
};

// Forward R2C: buf rows hold (x[2n], x[2n+1]) in slots 0..M-1 on entry and the
// half spectrum in slots 0..M on exit.  twH[e] = e^{-2 pi i e/PH} (e < PH),
// twW[e] = e^{-2 pi i e/PW} (e < PW), both in LDS.
// Forward R2C of NROWS real rows of length PW: rows of pitch PW/2 + 1 hold
// (x[2n], x[2n+1]) in slots 0..PW/2-1 on entry and the row's half spectrum
// in slots 0..PW/2 on exit.  twW[e] = e^{-2 pi i e/PW} in LDS.
template <int NROWS, int PW, int NT, typename T>
__device__ void rows_r2c_lds(cx<T>* buf, const cx<T>* twW, int tid) {
  constexpr int M = PW / 2, LDW = M + 1;
  fft_lines<M, NROWS, LDW, 1, 2, true, false, NT, T>(buf, twW, tid);
  // split the packed spectrum of each row into the spectrum of the real row
  constexpr int HALF = M / 2 + 1;
  for (int task = tid; task < NROWS * HALF; task += NT) {
    const int r = task / HALF, k = task % HALF;
    cx<T>* row = buf + r * LDW;
    if (k == 0) {
      const cx<T> z = row[0];
      row[0] = mk<T>(z.x + z.y, (T)0);
      row[M] = mk<T>(z.x - z.y, (T)0);
    } else if (k == M / 2) {
      row[k] = cconj<T>(row[k]);
    } else {
      const cx<T> zk = row[k], zm = row[M - k];
      const cx<T> e = mk<T>((zk.x + zm.x) * (T)0.5, (zk.y - zm.y) * (T)0.5);   // (zk + conj zm)/2
      const cx<T> o = mk<T>((zk.y + zm.y) * (T)0.5, (zm.x - zk.x) * (T)0.5);   // (zk - conj zm)/(2i)
      const cx<T> wo = cmul<T>(twW[k], o);
      row[k] = cadd<T>(e, wo);
      row[M - k] = cconj<T>(csub<T>(e, wo));
    }
  }
  __syncthreads();
}

// Unnormalised inverse C2R of NROWS rows: half spectra in, PW * (x[2n], x[2n+1]) out.
// The imaginary parts of columns 0 and PW/2 are ignored.
template <int NROWS, int PW, int NT, typename T>
__device__ void rows_c2r_lds(cx<T>* buf, const cx<T>* twW, int tid) {
  constexpr int M = PW / 2, LDW = M + 1;
  constexpr int HALF = M / 2 + 1;
  for (int task = tid; task < NROWS * HALF; task += NT) {
    const int r = task / HALF, k = task % HALF;
    cx<T>* row = buf + r * LDW;
    if (k == 0) {
      const T x0 = row[0].x, xm = row[M].x;
      row[0] = mk<T>(x0 + xm, x0 - xm);
    } else {
      const cx<T> xk = row[k], xm = row[M - k];
      const cx<T> e = mk<T>(xk.x + xm.x, xk.y - xm.y);                 // xk + conj xm
      const cx<T> o = cmulc<T>(mk<T>(xk.x - xm.x, xk.y + xm.y), twW[k]); // (xk - conj xm) w^-k
      row[k] = mk<T>(e.x - o.y, e.y + o.x);                            // e + i o
      if (k != M / 2) row[M - k] = mk<T>(e.x + o.y, o.x - e.y);        // conj e + i conj o
    }
  }
  __syncthreads();
  fft_lines<M, NROWS, LDW, 1, 2, true, true, NT, T>(buf, twW, tid);
}

template <int PH, int PW, int NT, typename T>
__device__ void rfft2_lds(cx<T>* buf, const cx<T>* twH, const cx<T>* twW, int tid) {
  using G = PlaneGeom<PH, PW>;
  rows_r2c_lds<PH, PW, NT, T>(buf, twW, tid);
  fft_lines<PH, G::WC, 1, G::LDW, 1, true, false, NT, T>(buf, twH, tid);
}

// Unnormalised inverse C2R: half spectrum in, P * (x[2n], x[2n+1]) out.
// The imaginary parts of columns 0 and PW/2 are ignored after the column pass.
template <int PH, int PW, int NT, typename T>
__device__ void irfft2_lds(cx<T>* buf, const cx<T>* twH, const cx<T>* twW, int tid) {
  using G = PlaneGeom<PH, PW>;
  fft_lines<PH, G::WC, 1, G::LDW, 1, true, true, NT, T>(buf, twH, tid);
  rows_c2r_lds<PH, PW, NT, T>(buf, twW, tid);
}

}  // namespace ocsc

#pragma clang fp contract(fast)
