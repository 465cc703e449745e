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
//      Y = C U, M = U^H Y, S^-1 by Gauss-Jordan elimination without pivoting
//      (S is Hermitian positive definite, its eigenvalues are >= 1), W =
//      Y S^-1, and C <- C - W Y^H on the 16 x 16 tiles on and above the
//      diagonal;
//   3. C_p is written back.
// The products run on v_mfma_f32_16x16x4_f32 (operand A[i][kk] in lane
// i + 16 kk, B[kk][j] in lane j + 16 kk, result D[i][j] in lane j + 16 (i / 4),
// register i % 4), three real products per complex one.  U, Y and W are held
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
// KP + 1), S (16 x 16, re and im), four partial products U^H Y (re, im), the
// block's x (16 complex)
// (at least the staging stores of C: whole rounds of 256 16-byte vectors)
__host__ __device__ inline size_t fold_mfma_lds(int K, int fs) {
  const int kp = (K + 15) / 16 * 16, kpp = kp + 1;
  const size_t need = ((size_t)fs + 4 * (size_t)FM_B * kpp + 2 * 256 + 4 * 2 * 256 + 2 * FM_B) * sizeof(float);
  const size_t stage = (size_t)((kp * (kp + 1) / 4 + FM_NT - 1) / FM_NT) * FM_NT * 16;
  return need > stage ? need : stage;
}

// C[r][c] from the R-form (zero outside K x K), without branches: the two
// loads read R[min][max] and R[max][min] (address 0 outside K x K)
__device__ __forceinline__ void fm_centry(const float* R, int ld, int K, int r, int c, float& cr, float& ci) {
  const bool up = r < c, ok = r < K && c < K;
  const int lo = up ? r : c, hi = up ? c : r;
  const float a = R[ok ? lo * ld + hi : 0], b = R[ok ? hi * ld + lo : 0];
  cr = ok ? a : 0.f;
  ci = (!ok || r == c) ? 0.f : (up ? b : -b);
}

// A complex product accumulated as three real ones: p1 += ar br, p2 += ai bi,
// p3 += (ar + ai)(br + bi); then Re = p1 - p2, Im = p3 - p1 - p2.
struct FmAcc {
  v4f p1, p2, p3;
};
__device__ __forceinline__ FmAcc fm_zero() { return FmAcc{{0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}}; }
__device__ __forceinline__ void fm_cmac(FmAcc& a, float ar, float ai, float br, float bi) {
  a.p1 = fm_mfma(ar, br, a.p1);
  a.p2 = fm_mfma(ai, bi, a.p2);
  a.p3 = fm_mfma(ar + ai, br + bi, a.p3);
}
__device__ __forceinline__ float fm_re(const FmAcc& a, int e) { return a.p1[e] - a.p2[e]; }
__device__ __forceinline__ float fm_im(const FmAcc& a, int e) { return a.p3[e] - a.p1[e] - a.p2[e]; }

// One frequency per workgroup (blockIdx.x = p).  Cm: R-forms of pitch fs;
// G, rfold (optional): complex [K][Pf]; Zt[(p * ldt + b) * K + k]: the code
// spectra of the nfold pending samples; xh[b * Pf + p]: their sample spectra.
// Per block: the code spectra were fetched into registers during the previous
// block (thread k holds row k of U); Y = C U with a wave's row tiles
// interleaved; M = U^H Y as four partial sums (one per wave), added in a
// fixed order; S^-1 by one wave in registers (a column per lane); W = Y S^-1;
// the update tiles two at a time.
template <int KP>
__global__ __launch_bounds__(FM_NT, 2) void k_fold_mfma(float* __restrict__ Cm, int fs, int K, int Pf,
                                                        float2* __restrict__ G, float2* __restrict__ rfold,
                                                        const float2* __restrict__ Zt, int ldt,
                                                        const float2* __restrict__ xh, int nfold) {
  constexpr int NB = KP / 16;             // 16-row tiles of C
  constexpr int KPP = KP + 1;             // pitch of U, Y, W
  constexpr int TPW = (NB + 3) / 4;       // row tiles per wave
  constexpr int NTI = NB * (NB + 1) / 2;  // update tiles on and above the diagonal
  extern __shared__ __align__(16) float fm_smem[];
  float* R = fm_smem;
  float* Ur = R + fs;                     // U, then W
  float* Ui = Ur + FM_B * KPP;
  float* Yr = Ui + FM_B * KPP;
  float* Yi = Yr + FM_B * KPP;
  float* Sr = Yi + FM_B * KPP;            // S, then S^-1
  float* Si = Sr + 256;
  float* Mp = Si + 256;                   // [4][2][256]: partial products U^H Y
  float2* xs = reinterpret_cast<float2*>(Mp + 4 * 2 * 256);
  const int p = blockIdx.x, tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int li = lane & 15, lk = lane >> 4;
  const int ld = K + 1;
  const float2* zt = Zt + (size_t)p * ldt * K;

  // this thread's row of U for the block at b0 (thread k < KP; zero past K or nfold)
  float2 zn[FM_B];
  float2 xn = make_float2(0.f, 0.f);
  auto fetch = [&](int b0) {
    if (tid < KP) {
#pragma unroll
      for (int q = 0; q < FM_B; ++q)
        zn[q] = (tid < K && b0 + q < nfold) ? zt[(size_t)(b0 + q) * K + tid] : make_float2(0.f, 0.f);
    }
    if (tid < FM_B) xn = b0 + tid < nfold ? xh[(size_t)(b0 + tid) * Pf + p] : make_float2(0.f, 0.f);
  };
  fetch(0);
  {
    // every load issued before the first store: indices past C_p are clamped
    // to its last vector, and their stores land in the U / Y area (written
    // before it is read)
    constexpr int NVM = (KP * (KP + 1) / 4 + FM_NT - 1) / FM_NT;
    const int nv = fs / 4;
    const v4f* src = reinterpret_cast<const v4f*>(Cm + (size_t)p * fs);
    v4f* dst = reinterpret_cast<v4f*>(R);
    v4f cv[NVM];
#pragma unroll
    for (int m = 0; m < NVM; ++m) cv[m] = __builtin_nontemporal_load(src + min(tid + m * FM_NT, nv - 1));
#pragma unroll
    for (int m = 0; m < NVM; ++m) dst[tid + m * FM_NT] = cv[m];
  }
  float2 gacc = make_float2(0.f, 0.f), racc = make_float2(0.f, 0.f);
  if (tid < K) {
    gacc = G[(size_t)tid * Pf + p];
    if (rfold) racc = rfold[(size_t)tid * Pf + p];
  }

  for (int b0 = 0; b0 < nfold; b0 += FM_B) {
    __syncthreads();   // C staged or updated; U, Y, S and the partials free
    if (tid < KP) {
#pragma unroll
      for (int q = 0; q < FM_B; ++q) {
        Ur[q * KPP + tid] = zn[q].x;   // u = conj(z)
        Ui[q * KPP + tid] = -zn[q].y;
      }
    }
    if (tid < FM_B) xs[tid] = xn;
    __syncthreads();
    if (tid < K) {   // G_p[k] (and the carried right-hand side) += u_bk x_bp, in sample order
#pragma unroll
      for (int q = 0; q < FM_B; ++q) {
        if (b0 + q < nfold) {
          const float ur = zn[q].x, ui = -zn[q].y;
          const float2 x = xs[q];
          const float dr = ur * x.x - ui * x.y, di = ur * x.y + ui * x.x;
          gacc.x += dr;
          gacc.y += di;
          racc.x += dr;
          racc.y += di;
        }
      }
    }
    if (b0 + FM_B < nfold) fetch(b0 + FM_B);   // in flight during this block
    // Y = C U: the wave's row tiles I = wave, wave + 4, ... in one k loop
    {
      FmAcc ya[TPW];
#pragma unroll
      for (int t = 0; t < TPW; ++t) ya[t] = fm_zero();
#pragma unroll 2
      for (int ks = 0; ks < KP / 4; ++ks) {
        const int c = ks * 4 + lk;
        const float ur = Ur[li * KPP + c], ui = Ui[li * KPP + c];   // B[kk][j] = U[c][j]
#pragma unroll
        for (int t = 0; t < TPW; ++t) {
          const int I = wave + 4 * t;
          if (I < NB) {
            float cr, ci;
            fm_centry(R, ld, K, I * 16 + li, c, cr, ci);           // A[i][kk] = C[I*16+i][c]
            fm_cmac(ya[t], cr, ci, ur, ui);
          }
        }
      }
#pragma unroll
      for (int t = 0; t < TPW; ++t) {
        const int I = wave + 4 * t;
        if (I < NB) {
#pragma unroll
          for (int e = 0; e < 4; ++e) {   // D[i][j]: row I * 16 + 4 lk + e, sample li
            Yr[li * KPP + I * 16 + 4 * lk + e] = fm_re(ya[t], e);
            Yi[li * KPP + I * 16 + 4 * lk + e] = fm_im(ya[t], e);
          }
        }
      }
    }
    __syncthreads();
    // partial M_w = sum over the wave's row tiles of U_I^H Y_I
    {
      FmAcc ma = fm_zero();
#pragma unroll
      for (int t = 0; t < TPW; ++t) {
        const int I = wave + 4 * t;
        if (I < NB) {
#pragma unroll
          for (int ks = 0; ks < 4; ++ks) {
            const int c = I * 16 + ks * 4 + lk;
            fm_cmac(ma, Ur[li * KPP + c], -Ui[li * KPP + c], Yr[li * KPP + c], Yi[li * KPP + c]);
          }
        }
      }
#pragma unroll
      for (int e = 0; e < 4; ++e) {   // M[a][b]: a = 4 lk + e, b = li
        Mp[(wave * 2) * 256 + (4 * lk + e) * 16 + li] = fm_re(ma, e);
        Mp[(wave * 2 + 1) * 256 + (4 * lk + e) * 16 + li] = fm_im(ma, e);
      }
    }
    __syncthreads();
    if (wave == 0) {
      // S = I + sum of the partials (fixed order), then S^-1 by Gauss-Jordan
      // elimination on this wave alone: lane j + 16 g holds rows 4g .. 4g+3 of
      // column j of S in registers; in step k each lane takes its rows of the
      // pivot column from lane k + 16 g and its element of the pivot row,
      // a_kj, from lane j + 16 (k / 4) by lane shuffles, a_kk by readlane
      const int j = li, g = lk;
      float cr[4], ci[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        const int i = 4 * g + a, idx = i * 16 + j;
        float sr = i == j ? 1.f : 0.f, si = 0.f;
#pragma unroll
        for (int w = 0; w < 4; ++w) {
          sr += Mp[(w * 2) * 256 + idx];
          si += Mp[(w * 2 + 1) * 256 + idx];
        }
        cr[a] = sr;
        ci[a] = si;
      }
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        const int kg = k >> 2, ka = k & 3;
        // this lane's element in row slot ka (row 4 g + ka)
        const float skr = ka == 0 ? cr[0] : ka == 1 ? cr[1] : ka == 2 ? cr[2] : cr[3];
        const float ski = ka == 0 ? ci[0] : ka == 1 ? ci[1] : ka == 2 ? ci[2] : ci[3];
        // a_kj of this lane's column, from the lane holding row k of it
        const float akr = __shfl(skr, j + 16 * kg, 64), aki = __shfl(ski, j + 16 * kg, 64);
        // a_kk, and this lane's rows of column k (from lane k + 16 g)
        const float pkr = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(skr), k + 16 * kg));
        const float pki = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(ski), k + 16 * kg));
        float qr4[4], qi4[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          qr4[a] = __shfl(cr[a], k + 16 * g, 64);
          qi4[a] = __shfl(ci[a], k + 16 * g, 64);
        }
        const float den = pkr * pkr + pki * pki;
        const float ivr = pkr / den, ivi = -pki / den;   // 1 / a_kk
        const float tr = akr * ivr - aki * ivi, ti = akr * ivi + aki * ivr;   // a_kj / a_kk
        const bool pivcol = j == k;
        const float fr = pivcol ? ivr : tr, fi = pivcol ? ivi : ti;
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          const int i = 4 * g + a;
          const float qpr = qr4[a], qpi = qi4[a];   // a_ik
          if (i == k) {
            cr[a] = fr;
            ci[a] = fi;
          } else {
            // column k: -a_ik / a_kk;  elsewhere: a_ij - a_ik a_kj / a_kk
            const float qr = qpr * fr - qpi * fi, qi = qpr * fi + qpi * fr;
            cr[a] = pivcol ? -qr : cr[a] - qr;
            ci[a] = pivcol ? -qi : ci[a] - qi;
          }
        }
      }
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        Sr[(4 * g + a) * 16 + j] = cr[a];
        Si[(4 * g + a) * 16 + j] = ci[a];
      }
    }
    __syncthreads();   // S^-1 in (Sr, Si)
    // W = Y S^-1 into U's place
    {
      FmAcc wa[TPW];
#pragma unroll
      for (int t = 0; t < TPW; ++t) wa[t] = fm_zero();
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) {
        const int q = ks * 4 + lk;
        const float br = Sr[q * 16 + li], bi = Si[q * 16 + li];   // B[kk][j] = S^-1[q][j]
#pragma unroll
        for (int t = 0; t < TPW; ++t) {
          const int I = wave + 4 * t;
          if (I < NB) fm_cmac(wa[t], Yr[q * KPP + I * 16 + li], Yi[q * KPP + I * 16 + li], br, bi);
        }
      }
#pragma unroll
      for (int t = 0; t < TPW; ++t) {
        const int I = wave + 4 * t;
        if (I < NB) {
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            Ur[li * KPP + I * 16 + 4 * lk + e] = fm_re(wa[t], e);
            Ui[li * KPP + I * 16 + 4 * lk + e] = fm_im(wa[t], e);
          }
        }
      }
    }
    __syncthreads();
    // C <- C - W Y^H on the tiles (I, J), I <= J, two at a time
    for (int t0 = wave; t0 < NTI; t0 += 8) {
      int ti[2], tj[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        int I = 0, tt = min(t0 + 4 * h, NTI - 1);
        while (tt >= NB - I) {
          tt -= NB - I;
          ++I;
        }
        ti[h] = I;
        tj[h] = I + tt;
      }
      const bool two = t0 + 4 < NTI;
      FmAcc pa[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) pa[h] = fm_zero();
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) {
        const int q = ks * 4 + lk;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          if (h == 0 || two)   // A[i][kk] = W[I*16+i][q], B[kk][j] = conj(Y[J*16+j][q])
            fm_cmac(pa[h], Ur[q * KPP + ti[h] * 16 + li], Ui[q * KPP + ti[h] * 16 + li],
                    Yr[q * KPP + tj[h] * 16 + li], -Yi[q * KPP + tj[h] * 16 + li]);
        }
      }
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        if (h == 1 && !two) break;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int r = ti[h] * 16 + 4 * lk + e, c = tj[h] * 16 + li;
          if (r < K && c < K) {
            if (r < c) {
              R[r * ld + c] -= fm_re(pa[h], e);    // Re C_rc
              R[c * ld + r] -= fm_im(pa[h], e);    // Im C_rc
            } else if (r == c) {
              R[r * ld + r] -= fm_re(pa[h], e);
            }
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
