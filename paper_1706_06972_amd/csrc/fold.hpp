// fold.hpp -- history fold of several pending samples on the FP32 matrix cores
// (eqs. B_update and C_update, FP32 contexts, K <= 128).
//
// C_p = (H_p + rho_d I)^-1 takes the rank-one terms u_b u_b^H, u_b = conj(z_bp),
// of the pending samples in sample order.  Taken sixteen at a time, the
// recursion of eq. C_update is the block identity
//   (A + U U^H)^-1 = C - Y S^-1 Y^H,   Y = C U,  S = I + U^H Y,
// with C = A^-1 and U the K x 16 block (exact in exact arithmetic; zero
// columns pad the last block).  Per frequency, one workgroup of four waves:
//   1. C_p (R-form: R[i][j] = Re C_ij for j >= i, -Im C_ij for j < i; rows of
//      pitch K + 1) is staged in LDS;
//   2. per block: U from the frequency-major copy of the code spectra, G_p
//      (and the warm-start right-hand side) += u_b x_bp in sample order;
//      Y = C U, M = U^H Y, S^-1 by Gauss-Jordan elimination (S is Hermitian
//      positive definite, its eigenvalues are >= 1), W = Y S^-1, and
//      C <- C - W Y^H on the 16 x 16 tiles on and above the diagonal;
//   3. C_p is written back.
// The products run on v_mfma_f32_16x16x4_f32 (operand A[i][kk] in lane
// i + 16 kk, B[kk][j] in lane j + 16 kk, result D[i][j] in lane j + 16 (i / 4),
// register i % 4), four real products per complex one.  U, Y and W are held
// sample-major, [16][K rounded up to 16, plus 1], so that the 16 rows or
// samples one operand load touches fall in different banks.
#pragma once
#include "common.hpp"

namespace ocsc {

constexpr int FM_B = 16;    // samples per block
constexpr int FM_NT = 256;  // threads per workgroup

__device__ __forceinline__ v4f fm_mfma(float a, float b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// LDS of k_fold_mfma in bytes: R (fs reals), U and Y (re, im; 16 rows of
// KP + 1), S (16 x 16, re and im), the block's x (16 complex)
__host__ __device__ inline size_t fold_mfma_lds(int K, int fs) {
  const int kpp = (K + 15) / 16 * 16 + 1;
  return ((size_t)fs + 4 * (size_t)FM_B * kpp + 2 * 256 + 2 * FM_B) * sizeof(float);
}

// C[r][c] from the R-form (zero outside K x K)
__device__ __forceinline__ void fm_centry(const float* R, int ld, int K, int r, int c, float& cr, float& ci) {
  cr = 0.f;
  ci = 0.f;
  if (r < K && c < K) {
    if (r < c) {
      cr = R[r * ld + c];
      ci = R[c * ld + r];
    } else if (r > c) {
      cr = R[c * ld + r];
      ci = -R[r * ld + c];
    } else {
      cr = R[r * ld + r];
    }
  }
}

// One frequency per workgroup (blockIdx.x = p).  Cm: R-forms of pitch fs;
// G, rfold (optional): complex [K][Pf]; Zt[(p * ldt + b) * K + k]: the code
// spectra of the nfold pending samples; xh[b * Pf + p]: their sample spectra.
template <int KP>
__global__ __launch_bounds__(FM_NT, 2) void k_fold_mfma(float* __restrict__ Cm, int fs, int K, int Pf,
                                                        float2* __restrict__ G, float2* __restrict__ rfold,
                                                        const float2* __restrict__ Zt, int ldt,
                                                        const float2* __restrict__ xh, int nfold) {
  constexpr int NB = KP / 16;           // 16-row tiles of C
  constexpr int KPP = KP + 1;           // pitch of U, Y, W
  constexpr int NTI = NB * (NB + 1) / 2;  // tiles on and above the diagonal
  extern __shared__ __align__(16) float fm_smem[];
  float* R = fm_smem;
  float* Ur = R + fs;                   // U, then W
  float* Ui = Ur + FM_B * KPP;
  float* Yr = Ui + FM_B * KPP;
  float* Yi = Yr + FM_B * KPP;
  float* Sr = Yi + FM_B * KPP;
  float* Si = Sr + 256;
  float2* xs = reinterpret_cast<float2*>(Si + 256);
  const int p = blockIdx.x, tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int li = lane & 15, lk = lane >> 4;
  const int ld = K + 1;

  {
    const v4f* src = reinterpret_cast<const v4f*>(Cm + (size_t)p * fs);
    v4f* dst = reinterpret_cast<v4f*>(R);
    for (int v = tid; v < fs / 4; v += FM_NT) dst[v] = __builtin_nontemporal_load(src + v);
  }
  float2 gacc = make_float2(0.f, 0.f), racc = make_float2(0.f, 0.f);
  if (tid < K) {
    gacc = G[(size_t)tid * Pf + p];
    if (rfold) racc = rfold[(size_t)tid * Pf + p];
  }
  const float2* zt = Zt + (size_t)p * ldt * K;

  for (int b0 = 0; b0 < nfold; b0 += FM_B) {
    __syncthreads();   // C staged or updated; U, Y and S free
    if (tid < FM_B) xs[tid] = b0 + tid < nfold ? xh[(size_t)(b0 + tid) * Pf + p] : make_float2(0.f, 0.f);
    for (int e = tid; e < FM_B * KP; e += FM_NT) {
      const int q = e / KP, k = e - q * KP;   // consecutive threads: consecutive k of one sample
      float2 z = make_float2(0.f, 0.f);
      if (k < K && b0 + q < nfold) z = zt[(size_t)(b0 + q) * K + k];
      Ur[q * KPP + k] = z.x;   // u = conj(z)
      Ui[q * KPP + k] = -z.y;
    }
    __syncthreads();
    if (tid < K) {   // G_p[k] (and the carried right-hand side) += u_bk x_bp, in sample order
      for (int q = 0; q < FM_B && b0 + q < nfold; ++q) {
        const float ur = Ur[q * KPP + tid], ui = Ui[q * KPP + tid];
        const float2 x = xs[q];
        const float dr = ur * x.x - ui * x.y, di = ur * x.y + ui * x.x;
        gacc.x += dr;
        gacc.y += di;
        racc.x += dr;
        racc.y += di;
      }
    }
    // Y = C U: wave -> row tiles I
    for (int I = wave; I < NB; I += 4) {
      v4f yr = {0.f, 0.f, 0.f, 0.f}, yi = {0.f, 0.f, 0.f, 0.f};
      const int r = I * 16 + li;
#pragma unroll 4
      for (int ks = 0; ks < KP / 4; ++ks) {
        const int c = ks * 4 + lk;
        float cr, ci;
        fm_centry(R, ld, K, r, c, cr, ci);                  // A[i][kk] = C[r][c]
        const float ur = Ur[li * KPP + c], ui = Ui[li * KPP + c];   // B[kk][j] = U[c][j]
        yr = fm_mfma(cr, ur, yr);
        yr = fm_mfma(-ci, ui, yr);
        yi = fm_mfma(cr, ui, yi);
        yi = fm_mfma(ci, ur, yi);
      }
#pragma unroll
      for (int e = 0; e < 4; ++e) {   // D[i][j]: row I * 16 + 4 lk + e, sample li
        Yr[li * KPP + I * 16 + 4 * lk + e] = yr[e];
        Yi[li * KPP + I * 16 + 4 * lk + e] = yi[e];
      }
    }
    __syncthreads();
    // S = I + U^H Y on wave 0
    if (wave == 0) {
      v4f mr = {0.f, 0.f, 0.f, 0.f}, mi = {0.f, 0.f, 0.f, 0.f};
#pragma unroll 4
      for (int ks = 0; ks < KP / 4; ++ks) {
        const int c = ks * 4 + lk;
        const float ar = Ur[li * KPP + c], ai = -Ui[li * KPP + c];   // A[a][kk] = conj(U[c][a])
        const float br = Yr[li * KPP + c], bi = Yi[li * KPP + c];    // B[kk][b] = Y[c][b]
        mr = fm_mfma(ar, br, mr);
        mr = fm_mfma(-ai, bi, mr);
        mi = fm_mfma(ar, bi, mi);
        mi = fm_mfma(ai, br, mi);
      }
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int a = 4 * lk + e;
        Sr[a * 16 + li] = mr[e] + (a == li ? 1.f : 0.f);
        Si[a * 16 + li] = mi[e];
      }
    }
    // S^-1 in place by Gauss-Jordan elimination, thread (i, j) = (tid / 16, tid % 16)
    {
      const int i = tid >> 4, j = tid & 15;
      for (int k = 0; k < 16; ++k) {
        __syncthreads();
        const float aikr = Sr[i * 16 + k], aiki = Si[i * 16 + k];
        const float akjr = Sr[k * 16 + j], akji = Si[k * 16 + j];
        const float akkr = Sr[k * 16 + k], akki = Si[k * 16 + k];
        const float aijr = Sr[tid], aiji = Si[tid];
        __syncthreads();
        const float den = akkr * akkr + akki * akki;
        const float ivr = akkr / den, ivi = -akki / den;   // 1 / a_kk
        const float tr = akjr * ivr - akji * ivi, ti = akjr * ivi + akji * ivr;   // a_kj / a_kk
        float nr, ni;
        if (i == k && j == k) {
          nr = ivr;
          ni = ivi;
        } else if (i == k) {
          nr = tr;
          ni = ti;
        } else if (j == k) {
          nr = -(aikr * ivr - aiki * ivi);
          ni = -(aikr * ivi + aiki * ivr);
        } else {
          nr = aijr - (aikr * tr - aiki * ti);
          ni = aiji - (aikr * ti + aiki * tr);
        }
        Sr[tid] = nr;
        Si[tid] = ni;
      }
    }
    __syncthreads();
    // W = Y S^-1 into U's place
    for (int I = wave; I < NB; I += 4) {
      v4f wr = {0.f, 0.f, 0.f, 0.f}, wi = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) {
        const int q = ks * 4 + lk;
        const float ar = Yr[q * KPP + I * 16 + li], ai = Yi[q * KPP + I * 16 + li];   // A[i][kk] = Y[I*16+i][q]
        const float br = Sr[q * 16 + li], bi = Si[q * 16 + li];                       // B[kk][j] = S^-1[q][j]
        wr = fm_mfma(ar, br, wr);
        wr = fm_mfma(-ai, bi, wr);
        wi = fm_mfma(ar, bi, wi);
        wi = fm_mfma(ai, br, wi);
      }
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        Ur[li * KPP + I * 16 + 4 * lk + e] = wr[e];
        Ui[li * KPP + I * 16 + 4 * lk + e] = wi[e];
      }
    }
    __syncthreads();
    // C <- C - W Y^H on the tiles (I, J), I <= J
    for (int t = wave; t < NTI; t += 4) {
      int I = 0, tt = t;
      while (tt >= NB - I) {
        tt -= NB - I;
        ++I;
      }
      const int J = I + tt;
      v4f pr = {0.f, 0.f, 0.f, 0.f}, pi = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) {
        const int q = ks * 4 + lk;
        const float ar = Ur[q * KPP + I * 16 + li], ai = Ui[q * KPP + I * 16 + li];    // A[i][kk] = W[I*16+i][q]
        const float br = Yr[q * KPP + J * 16 + li], bi = -Yi[q * KPP + J * 16 + li];   // B[kk][j] = conj(Y[J*16+j][q])
        pr = fm_mfma(ar, br, pr);
        pr = fm_mfma(-ai, bi, pr);
        pi = fm_mfma(ar, bi, pi);
        pi = fm_mfma(ai, br, pi);
      }
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int r = I * 16 + 4 * lk + e, c = J * 16 + li;
        if (r < K && c < K) {
          if (r < c) {
            R[r * ld + c] -= pr[e];   // Re C_rc
            R[c * ld + r] -= pi[e];   // Im C_rc
          } else if (r == c) {
            R[r * ld + r] -= pr[e];
          }
        }
      }
    }
  }
  __syncthreads();
  {
    v4f* dst = reinterpret_cast<v4f*>(Cm + (size_t)p * fs);
    const v4f* src = reinterpret_cast<const v4f*>(R);
    for (int v = tid; v < fs / 4; v += FM_NT) __builtin_nontemporal_store(src[v], dst + v);
  }
  if (tid < K) {
    G[(size_t)tid * Pf + p] = gacc;
    if (rfold) rfold[(size_t)tid * Pf + p] = racc;
  }
}

}  // namespace ocsc
