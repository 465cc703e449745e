// vstep.hpp -- V-step of DictOCSC (Proposition 2), Theta update and the next
// D-step right-hand side, by pruned DFTs (only the filter support is formed).
#pragma once
#include "common.hpp"

namespace ocsc {

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
constexpr int MAXF = 128;   // filter extent bound of these kernels
constexpr int VCH = 8;      // loads per thread issued together

// MAXP: bound on PH and PW (128, or 512 for the two-pass grids).
template <typename T, int MAXP>
__global__ __launch_bounds__(256) void k_vstep_alpha(const cx<T>* __restrict__ d,
                                                     const cx<T>* __restrict__ Th, T* __restrict__ apart,
                                                     const cx<T>* __restrict__ twH,
                                                     const cx<T>* __restrict__ twW, int PH, int PW,
                                                     int Mh, int Mw, int first) {
  constexpr int VB = vblock<T>();
  __shared__ cx<T> X[MAXP * VB];
  __shared__ cx<T> t[2 * MAXF * VB];
  __shared__ cx<T> sH[MAXP], sW[MAXP];
  const int WC = PW / 2 + 1, Pf = PH * WC;
  const int vb = blockIdx.x, k = blockIdx.y, nvb = gridDim.x;
  const int v0 = vb * VB, nv = min(VB, WC - v0);
  const int tid = threadIdx.x;
  for (int i = tid; i < PH; i += 256) sH[i] = twH[i];
  for (int i = tid; i < PW; i += 256) sW[i] = twW[i];
  const cx<T>* dk = d + (size_t)k * Pf;
  const cx<T>* tk = Th + (size_t)k * Pf;
  for (int e0 = 0; e0 < PH * VB; e0 += VCH * 256) {
    cx<T> xd[VCH], xt[VCH];
#pragma unroll
    for (int q = 0; q < VCH; ++q) {   // a chunk's loads are issued before any use
      const int e = e0 + tid + q * 256, u = e / VB, c = e % VB;
      xd[q] = mk<T>(0, 0);
      xt[q] = mk<T>(0, 0);
      if (e < PH * VB && c < nv) {
        xd[q] = dk[u * WC + v0 + c];
        if (!first) xt[q] = tk[u * WC + v0 + c];
      }
    }
#pragma unroll
    for (int q = 0; q < VCH; ++q) {
      const int e = e0 + tid + q * 256;
      if (e < PH * VB) X[e] = cadd<T>(xd[q], xt[q]);
    }
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
// apart == nullptr: V is given (the consensus V-step of several grids) and
// only read.
template <typename T, int MAXP>
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
  __shared__ cx<T> sH[MAXP], sW[MAXP];
  const int WC = PW / 2 + 1, Pf = PH * WC;
  const int vb = blockIdx.x, k = blockIdx.y, nvb = gridDim.x;
  const int v0 = vb * VB, nv = min(VB, WC - v0);
  const int tid = threadIdx.x;
  const int MM = Mh * Mw;
  for (int i = tid; i < PH; i += 256) sH[i] = twH[i];
  for (int i = tid; i < PW; i += 256) sW[i] = twW[i];
  if (apart) {
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
  } else {
    for (int e = tid; e < MM; e += 256) alpha[e] = V[(size_t)k * MM + e];
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
  for (int e0 = 0; e0 < PH * VB; e0 += VCH * 256) {
    cx<T> dq[VCH], tq[VCH], gq[VCH];
#pragma unroll
    for (int q = 0; q < VCH; ++q) {   // a chunk's loads are issued before any use
      const int e = e0 + tid + q * 256, u = e / VB, c = e % VB;
      dq[q] = tq[q] = gq[q] = mk<T>(0, 0);
      if (e < PH * VB && c < nv) {
        const size_t idx = base + (size_t)u * WC + v0 + c;
        dq[q] = d[idx];
        if (!first) tq[q] = Th[idx];
        gq[q] = G[idx];
      }
    }
#pragma unroll
    for (int q = 0; q < VCH; ++q) {
      const int e = e0 + tid + q * 256, u = e / VB, c = e % VB;
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
    for (int j = 0; j < FPT; ++j) dq[j] = d[base + min(tid + j * NT, PF - 1)];
    if (first) {   // outside the loop, so that the loads are not waited for one by one
#pragma unroll
      for (int j = 0; j < FPT; ++j) tqv[j] = mk<T>(0, 0);
    } else {
#pragma unroll
      for (int j = 0; j < FPT; ++j) tqv[j] = Th[base + min(tid + j * NT, PF - 1)];
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
// V-step on the matrix cores (FP32), one workgroup of 16 waves per filter k,
// filters of at most 16 x 16 taps.  The two large pruned DFTs are dense
// complex products, done as four real products each with
// v_mfma_f32_16x16x4_f32 (operand A[i][kk] in lane i + 16 kk, B[kk][j] in
// lane j + 16 kk, result D[i][j] in lane j + 16 (i / 4), register i % 4):
//   t  = W X:   W[m][u] = e^{+2 pi i u m / PH} (16 x PH),  X = d_k + Theta_k (PH x PW/2)
//   FV = W' r:  W'[u][m] = e^{-2 pi i u m / PH} (PH x 16), r (16 x PW/2)
// with r[m][v] = sum_n V_k[m][n] e^{-2 pi i v n / PW} (zero for m >= M_h).  The
// Nyquist column v = PW/2 of both products, alpha (the crop of the real
// inverse DFT), the ball projection and r are small and stay on the VALU.
//   alpha[m][n] = (1/P) sum_v c_v Re(t[m][v] e^{+2 pi i v n / PW}),
//   V_k = alpha / max(||alpha||, 1);  Theta <- X - FV;  rhs <- G + rho_d (FV - Theta).
// ---------------------------------------------------------------------------
template <int PH, int PW>
struct VGeo {
  static constexpr int WC = PW / 2 + 1;
  static constexpr int PF = PH * WC;
  static constexpr int NVT = (PW / 2) / 16;                 // 16-column tiles below the Nyquist column
  static constexpr int NUT = PH / 16;                       // 16-row tiles
  static constexpr int KS = PH / 4;                         // k-steps of t = W X
  static constexpr int WPT0 = 16 / NVT;
  static constexpr int WPT = WPT0 < KS ? WPT0 : KS;         // waves per column tile in t = W X
  static constexpr int SPW = KS / WPT;                      // k-steps per wave
  static constexpr int NTILE = NUT * NVT;                   // tiles of FV = W' r
  static constexpr int TPW = (NTILE + 15) / 16;             // tiles per wave
};

__device__ __forceinline__ v4f mfma4(float a, float b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <int PH, int PW>
__global__ __launch_bounds__(1024) void k_vstep_mfma(const float2* __restrict__ d, float2* __restrict__ Th,
                                                    const float2* __restrict__ G, float2* __restrict__ rhs,
                                                    float* __restrict__ V, const float2* __restrict__ twH,
                                                    const float2* __restrict__ twW, int Mh, int Mw, float rho_d,
                                                    int first) {
  using Gm = VGeo<PH, PW>;
  constexpr int WC = Gm::WC, PF = Gm::PF, NVT = Gm::NVT, WPT = Gm::WPT, SPW = Gm::SPW, TPW = Gm::TPW;
  constexpr int NT = 1024;
  static_assert(PH <= NT && PW <= NT, "one twiddle of each table per thread");
  static_assert(WPT * NVT >= 8, "part holds the 16 partial alpha products");
  constexpr int FPT = (PF + NT - 1) / NT;
  constexpr int NYQ = PW / 2;
  __shared__ __align__(16) float2 xs[PF];               // X[u][v]
  __shared__ __align__(16) float2 part[WPT * NVT * 256]; // partial t tiles [wave slot][16 x 16]
  __shared__ float2 ts[16 * WC];                        // t, then r
  __shared__ float2 sH[PH], sW[PW];
  __shared__ float al[VF * VF];
  __shared__ float red[16];
  const int k = blockIdx.x, tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int li = lane & 15, lk = lane >> 4;
  const size_t base = (size_t)k * PF;

  // X = d + Theta first; then G for this wave's output tiles and the Nyquist
  // column, which is used at the end and arrives during the products
  float2 gq[TPW][4], gny;
  {
    const float2 th = twH[min(tid, PH - 1)], tw = twW[min(tid, PW - 1)];
    float2 dq[FPT], tq[FPT];
#pragma unroll
    for (int j = 0; j < FPT; ++j) dq[j] = d[base + min(tid + j * NT, PF - 1)];
    // the test of first stays outside the loop: a branch around each load
    // made the compiler wait for all loads in flight at every join
    if (first) {
#pragma unroll
      for (int j = 0; j < FPT; ++j) tq[j] = make_float2(0.f, 0.f);
    } else {
#pragma unroll
      for (int j = 0; j < FPT; ++j) tq[j] = Th[base + min(tid + j * NT, PF - 1)];
    }
#pragma unroll
    for (int tt = 0; tt < TPW; ++tt) {
      const int tile = min(wave + 16 * tt, Gm::NTILE - 1);
      const int ut = tile / NVT, vt = tile - ut * NVT;
#pragma unroll
      for (int j = 0; j < 4; ++j) gq[tt][j] = G[base + (size_t)(ut * 16 + 4 * lk + j) * WC + vt * 16 + li];
    }
    gny = G[base + (size_t)min(tid, PH - 1) * WC + NYQ];
    if (tid < PH) sH[tid] = th;
    if (tid < PW) sW[tid] = tw;
#pragma unroll
    for (int j = 0; j < FPT; ++j) {
      const int e = tid + j * NT;
      if (PF % NT == 0 || e < PF) xs[e] = make_float2(dq[j].x + tq[j].x, dq[j].y + tq[j].y);
    }
  }
  __syncthreads();

  // ---- t = W X on the matrix cores: wave -> (column tile vt, slice of u)
  if (wave < WPT * NVT) {
    const int vt = wave / WPT, sl = wave - vt * WPT;
    // three real products per complex one: p1 = Re W Re X, p2 = Im W Im X,
    // p3 = (Re W + Im W)(Re X + Im X); Re t = p1 - p2, Im t = p3 - p1 - p2
    v4f p1 = {0, 0, 0, 0}, p2 = {0, 0, 0, 0}, p3 = {0, 0, 0, 0};
#pragma unroll 4
    for (int s = 0; s < SPW; ++s) {
      const int u = (sl * SPW + s) * 4 + lk;
      const float2 w = sH[(u * li) & (PH - 1)];         // e^{-2 pi i u m/PH}, m = li; W is its conjugate
      const float2 x = xs[u * WC + vt * 16 + li];
      p1 = mfma4(w.x, x.x, p1);
      p2 = mfma4(-w.y, x.y, p2);                         // Im W = -w.y
      p3 = mfma4(w.x - w.y, x.x + x.y, p3);
    }
    float2* pp = part + (size_t)wave * 256;
#pragma unroll
    for (int j = 0; j < 4; ++j) pp[(4 * lk + j) * 16 + li] = make_float2(p1[j] - p2[j], p3[j] - p1[j] - p2[j]);
  }
  // Nyquist column of t on the VALU: wave m sums over u
  if (wave < 16) {
    const int m = wave;
    float ar = 0.f, ai = 0.f;
    for (int u = lane; u < PH; u += 64) {
      const float2 w = sH[(u * m) & (PH - 1)];
      const float2 x = xs[u * WC + NYQ];
      ar += x.x * w.x + x.y * w.y;
      ai += x.y * w.x - x.x * w.y;
    }
    for (int off = 32; off > 0; off >>= 1) {
      ar += __shfl_xor(ar, off, 64);
      ai += __shfl_xor(ai, off, 64);
    }
    if (lane == 0) ts[m * WC + NYQ] = make_float2(ar, ai);
  }
  __syncthreads();
  for (int e = tid; e < 16 * NYQ; e += NT) {
    const int m = e / NYQ, v = e - m * NYQ;
    const int vt = v >> 4, c = v & 15;
    float2 acc = make_float2(0.f, 0.f);
#pragma unroll
    for (int sl = 0; sl < WPT; ++sl) {
      const float2 q = part[(size_t)(vt * WPT + sl) * 256 + m * 16 + c];
      acc.x += q.x;
      acc.y += q.y;
    }
    ts[m * WC + v] = acc;
  }
  __syncthreads();

  // ---- alpha on the matrix cores, as the real product (16 x 2 WC)(2 WC x 16):
  //   A[m][2v + c] = (Re, Im)[c] t[m][v],  B[2v + c][n] = c_v (Re, Im)[c] e^{-2 pi i v n / PW}
  // (c_v = 1 at v = 0 and v = PW/2, else 2; the sum is Re(t conj(w)) over v).  Its k-steps
  // are dealt out to the 16 waves; their partial 16 x 16 products are added in wave order.
  {
    constexpr int KSA = (2 * WC + 3) / 4;
    v4f acc = {0, 0, 0, 0};
    for (int s = wave; s < KSA; s += 16) {
      const int kk = 4 * s + lk, v = kk >> 1;
      float a = 0.f, b = 0.f;
      if (v < WC) {
        const float2 tv = ts[li * WC + v];
        const float2 w = sW[(v * li) & (PW - 1)];
        const float cv = (v == 0 || 2 * v == PW) ? 1.f : 2.f;
        a = (kk & 1) ? tv.y : tv.x;
        b = cv * ((kk & 1) ? w.y : w.x);
      }
      acc = mfma4(a, b, acc);
    }
    float* pa = reinterpret_cast<float*>(part) + wave * 256;
#pragma unroll
    for (int j = 0; j < 4; ++j) pa[(4 * lk + j) * 16 + li] = acc[j];   // D[4 lk + j][li]
  }
  __syncthreads();
  const float invP = 1.f / (float)(PH * PW);
  float ss = 0.f;
  for (int o = tid; o < Mh * Mw; o += NT) {
    const int m = o / Mw, n = o - m * Mw;
    const float* pa = reinterpret_cast<const float*>(part) + m * 16 + n;
    float acc = 0.f;
#pragma unroll
    for (int w = 0; w < 16; ++w) acc += pa[w * 256];
    acc *= invP;
    al[o] = acc;
    ss += acc * acc;
  }
  for (int off = 32; off > 0; off >>= 1) ss += __shfl_xor(ss, off, 64);
  if (lane == 0) red[wave] = ss;
  __syncthreads();
  float nrm2 = 0.f;
#pragma unroll
  for (int w = 0; w < 16; ++w) nrm2 += red[w];
  const float nrm = sqrtf(nrm2);
  const float scale = 1.f / (nrm > 1.f ? nrm : 1.f);
  for (int task = tid; task < Mh * Mw; task += NT) {
    const float vv = al[task] * scale;
    al[task] = vv;
    V[(size_t)k * Mh * Mw + task] = vv;
  }
  __syncthreads();
  // r[m][v] = sum_n V[m][n] e^{-2 pi i v n / PW}, zero rows below M_h (into ts)
  for (int task = tid; task < 16 * WC; task += NT) {
    const int m = task / WC, v = task - m * WC;
    float ar = 0.f, ai = 0.f;
    if (m < Mh) {
      for (int n = 0; n < Mw; ++n) {
        const float2 w = sW[(v * n) & (PW - 1)];
        const float x = al[m * Mw + n];
        ar += x * w.x;
        ai += x * w.y;
      }
    }
    ts[task] = make_float2(ar, ai);
  }
  __syncthreads();

  // ---- FV = W' r on the matrix cores, then Theta and rhs for each output
#pragma unroll
  for (int tt = 0; tt < TPW; ++tt) {
    const int tile = wave + 16 * tt;
    if (tile < Gm::NTILE) {
      const int ut = tile / NVT, vt = tile - ut * NVT;
      const int u = ut * 16 + li;
      // three real products per complex one, as for t
      v4f p1 = {0, 0, 0, 0}, p2 = {0, 0, 0, 0}, p3 = {0, 0, 0, 0};
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int m = s * 4 + lk;
        const float2 w = sH[(u * m) & (PH - 1)];         // W'[u][m]
        const float2 x = ts[m * WC + vt * 16 + li];     // r[m][v]
        p1 = mfma4(w.x, x.x, p1);
        p2 = mfma4(w.y, x.y, p2);
        p3 = mfma4(w.x + w.y, x.x + x.y, p3);
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int uo = ut * 16 + 4 * lk + j, v = vt * 16 + li;
        const int e = uo * WC + v;
        const float fr = p1[j] - p2[j], fi = p3[j] - p1[j] - p2[j];
        const float2 xv = xs[e];
        const float2 th = make_float2(xv.x - fr, xv.y - fi);
        Th[base + e] = th;
        rhs[base + e] = make_float2(gq[tt][j].x + rho_d * (fr - th.x), gq[tt][j].y + rho_d * (fi - th.y));
      }
    }
  }
  // Nyquist column of FV on the VALU
  if (tid < PH) {
    const int u = tid;
    float ar = 0.f, ai = 0.f;
    for (int m = 0; m < Mh; ++m) {
      const float2 w = sH[(u * m) & (PH - 1)];
      const float2 x = ts[m * WC + NYQ];
      ar += x.x * w.x - x.y * w.y;
      ai += x.x * w.y + x.y * w.x;
    }
    const int e = u * WC + NYQ;
    const float2 xv = xs[e];
    const float2 th = make_float2(xv.x - ar, xv.y - ai);
    Th[base + e] = th;
    rhs[base + e] = make_float2(gny.x + rho_d * (ar - th.x), gny.y + rho_d * (ai - th.y));
  }
}

// ---------------------------------------------------------------------------
// Consensus V-step of several grids sharing one dictionary (one workgroup per
// filter k): alpha = sum_s w_s alpha_s / sum_s w_s with alpha_s the sum of the
// column-block partials of grid s (k_vstep_alpha) and w_s = P_s; then
// V_k = alpha / max(||alpha||, 1), written to every grid's V.
// ---------------------------------------------------------------------------
constexpr int GROUP_MAX = 8;

template <typename T>
struct GroupArgs {
  const T* apart[GROUP_MAX];
  T* V[GROUP_MAX];
  int nvb[GROUP_MAX];
  T w[GROUP_MAX];
  int n;
};

template <typename T>
__global__ __launch_bounds__(256) void k_vstep_group_v(GroupArgs<T> a, int MM) {
  __shared__ T red[256];
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* alpha = reinterpret_cast<T*>(smem_raw);   // [MM]
  const int k = blockIdx.x, tid = threadIdx.x;
  T wsum = 0;
  for (int s = 0; s < a.n; ++s) wsum += a.w[s];
  T ss = 0;
  for (int e = tid; e < MM; e += 256) {
    T acc = 0;
    for (int s = 0; s < a.n; ++s) {
      const T* ap = a.apart[s] + (size_t)k * a.nvb[s] * MM;
      T part = 0;
      for (int j = 0; j < a.nvb[s]; ++j) part += ap[(size_t)j * MM + e];
      acc += a.w[s] * part;
    }
    acc /= wsum;
    alpha[e] = acc;
    ss += acc * acc;
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
    const T v = alpha[e] * scale;
    for (int s = 0; s < a.n; ++s) a.V[s][(size_t)k * MM + e] = v;
  }
}

}  // namespace ocsc
