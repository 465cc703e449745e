// chol.hpp -- precision form of the history (FP32 contexts, K <= 128):
//   H_p += sum_b conj(z_bp) z_bp^T and G_p += sum_b conj(z_bp) x_bp for a
//   minibatch, the products on the BF16 matrix cores with FP32 accumulation
//   and a split-precision correction (z = hi + lo, both BF16; the products
//   hi*hi + hi*lo + lo*hi, dropping lo*lo), then
//   C_p = (H_p + rho_d I)^-1 recomputed per frequency in FP64 through a
//   Cholesky factor (eqs. A_update, B_update; C_update without the
//   Sherman-Morrison recursion).
#pragma once
#include "common.hpp"

namespace ocsc {

typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

constexpr int HERK_B = 64;            // samples per chunk (two k-steps of 32)
constexpr int HERK_LD = HERK_B + 8;   // LDS row pitch (bf16) of the transposed parts

__device__ __forceinline__ v4f mfma_bf16(v8bf a, v8bf b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// One workgroup (4 waves) per frequency p.  Zt[(p * ldt + b) * K + k] holds
// the nb pending code spectra frequency-major; xh[b * Pf + p] the sample
// spectra.  H_p (R-form, rows of pitch K + 1 at Hm + p * fs) and G[k][p] are
// updated in place.  The product tiles on and above the diagonal are spread
// over the waves; operand layout of v_mfma_f32_16x16x32_bf16: A[i][8g..8g+7]
// in lane i + 16 g, B[8g..8g+7][j] in lane j + 16 g, D[i][j] in lane
// j + 16 (i / 4), register i % 4.
template <int KP>
__global__ __launch_bounds__(256) void k_herk_bf16(const float2* __restrict__ Zt, int ldt, int nb,
                                                  const float2* __restrict__ xh, int Pf, float* __restrict__ Hm,
                                                  int fs, float2* __restrict__ G, int K) {
  constexpr int NTD = KP / 16;                    // tiles per dimension
  constexpr int NTILE = NTD * (NTD + 1) / 2;      // tiles on or above the diagonal
  constexpr int TPW = (NTILE + 3) / 4;            // tiles per wave
  __shared__ __align__(16) __bf16 zrh[KP * HERK_LD], zrl[KP * HERK_LD], zih[KP * HERK_LD], zil[KP * HERK_LD];
  const int p = blockIdx.x;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, li = lane & 15, lg = lane >> 4;
  int tri[TPW], trj[TPW];
#pragma unroll
  for (int tt = 0; tt < TPW; ++tt) {   // upper-triangular tile enumeration (row-major)
    int t = min(wave + 4 * tt, NTILE - 1), i = 0;
    while (t >= NTD - i) {
      t -= NTD - i;
      ++i;
    }
    tri[tt] = i;
    trj[tt] = i + t;
  }
  v4f re[TPW], im1[TPW], im2[TPW];
#pragma unroll
  for (int tt = 0; tt < TPW; ++tt) re[tt] = im1[tt] = im2[tt] = v4f{0, 0, 0, 0};
  float gr = 0.f, gi = 0.f;
  const float2* zp = Zt + (size_t)p * ldt * K;
  for (int b0 = 0; b0 < nb; b0 += HERK_B) {
    const int cb = min(HERK_B, nb - b0);
    __syncthreads();   // the previous chunk's operands are no longer read
    for (int e = tid; e < HERK_B * KP; e += 256) {
      const int b = e / KP, k = e - b * KP;   // consecutive threads read consecutive k
      float2 z = make_float2(0.f, 0.f);
      if (b < cb && k < K) z = zp[(size_t)(b0 + b) * K + k];
      const __bf16 rh = (__bf16)z.x, ih = (__bf16)z.y;
      const int o = k * HERK_LD + b;
      zrh[o] = rh;
      zrl[o] = (__bf16)(z.x - (float)rh);
      zih[o] = ih;
      zil[o] = (__bf16)(z.y - (float)ih);
    }
    if (tid < K) {   // G_p[k] += sum_b conj(z_bk) x_b (FP32)
      for (int b = 0; b < cb; ++b) {
        const float2 z = zp[(size_t)(b0 + b) * K + tid];
        const float2 x = xh[(size_t)(b0 + b) * Pf + p];
        gr += z.x * x.x + z.y * x.y;
        gi += z.x * x.y - z.y * x.x;
      }
    }
    __syncthreads();
#pragma unroll
    for (int tt = 0; tt < TPW; ++tt) {
      if (wave + 4 * tt >= NTILE) continue;
      const int ra = (tri[tt] * 16 + li) * HERK_LD, rb = (trj[tt] * 16 + li) * HERK_LD;
#pragma unroll
      for (int ks = 0; ks < HERK_B; ks += 32) {
        const int bo = ks + 8 * lg;
        const v8bf arh = *reinterpret_cast<const v8bf*>(&zrh[ra + bo]);
        const v8bf arl = *reinterpret_cast<const v8bf*>(&zrl[ra + bo]);
        const v8bf aih = *reinterpret_cast<const v8bf*>(&zih[ra + bo]);
        const v8bf ail = *reinterpret_cast<const v8bf*>(&zil[ra + bo]);
        const v8bf brh = *reinterpret_cast<const v8bf*>(&zrh[rb + bo]);
        const v8bf brl = *reinterpret_cast<const v8bf*>(&zrl[rb + bo]);
        const v8bf bih = *reinterpret_cast<const v8bf*>(&zih[rb + bo]);
        const v8bf bil = *reinterpret_cast<const v8bf*>(&zil[rb + bo]);
        // Re H_ij = sum_b zr_i zr_j + zi_i zi_j
        re[tt] = mfma_bf16(arh, brh, re[tt]);
        re[tt] = mfma_bf16(arh, brl, re[tt]);
        re[tt] = mfma_bf16(arl, brh, re[tt]);
        re[tt] = mfma_bf16(aih, bih, re[tt]);
        re[tt] = mfma_bf16(aih, bil, re[tt]);
        re[tt] = mfma_bf16(ail, bih, re[tt]);
        // Im H_ij = sum_b zr_i zi_j - zi_i zr_j
        im1[tt] = mfma_bf16(arh, bih, im1[tt]);
        im1[tt] = mfma_bf16(arh, bil, im1[tt]);
        im1[tt] = mfma_bf16(arl, bih, im1[tt]);
        im2[tt] = mfma_bf16(aih, brh, im2[tt]);
        im2[tt] = mfma_bf16(aih, brl, im2[tt]);
        im2[tt] = mfma_bf16(ail, brh, im2[tt]);
      }
    }
  }
  float* R = Hm + (size_t)p * fs;
  const int ld = K + 1;
#pragma unroll
  for (int tt = 0; tt < TPW; ++tt) {
    if (wave + 4 * tt >= NTILE) continue;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = tri[tt] * 16 + 4 * lg + r, j = trj[tt] * 16 + li;
      if (i < K && j < K && i <= j) {
        R[i * ld + j] += re[tt][r];
        if (i < j) R[j * ld + i] += im1[tt][r] - im2[tt][r];
      }
    }
  }
  if (tid < K) {
    float2 g = G[(size_t)tid * Pf + p];
    g.x += gr;
    g.y += gi;
    G[(size_t)tid * Pf + p] = g;
  }
}

// ---------------------------------------------------------------------------
// C_p = (H_p + rho_d I)^-1 in FP64, one workgroup per frequency, the lower
// triangle in LDS (packed, element (i, j) at i(i+1)/2 + j):
//   1. A = H + rho_d I (lower triangle, A_ij = conj(H_ji) for i > j);
//   2. Cholesky A = L L^H, right-looking: per column j, L_.j = A_.j / sqrt(A_jj),
//      then the trailing update A_ik -= L_ij conj(L_kj);
//   3. X = L^-1 in place, right-looking on [L | I]: per step k, row k of X is
//      B_k. / L_kk, then B_ij -= L_ik X_kj for i > k, j <= k (B starts as I;
//      column k of L is copied out before its slots take B);
//   4. C = X^H X, C_ij = sum_{k >= max(i, j)} conj(X_ki) X_kj, rounded to FP32
//      in the R-form of C (rows of pitch K + 1 at Cm + p * fs).
// Dynamic LDS: (K(K+1)/2 + K) complex doubles.  The trailing loops run on a
// (CHOL_NT / 16) x 16 thread tiling.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int tri_idx(int i, int j) { return i * (i + 1) / 2 + j; }

constexpr int CHOL_NT = 1024;   // threads per workgroup: 16 waves share each step's work

__global__ __launch_bounds__(CHOL_NT) void k_chol_inv(const float* __restrict__ Hm, float* __restrict__ Cm, int K,
                                                 int fs, double rho_d) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double2* L = reinterpret_cast<double2*>(smem_raw);
  double2* col = L + K * (K + 1) / 2;
  const int p = blockIdx.x, tid = threadIdx.x;
  constexpr int NY = CHOL_NT / 16;
  const int ty = tid >> 4, tx = tid & 15;
  const int ld = K + 1;
  const float* R = Hm + (size_t)p * fs;
  for (int i = ty; i < K; i += NY)
    for (int j = tx; j <= i; j += 16)
      L[tri_idx(i, j)] = (i == j) ? make_double2((double)R[i * ld + i] + rho_d, 0.0)
                                  : make_double2((double)R[j * ld + i], -(double)R[i * ld + j]);
  __syncthreads();
  // 2. Cholesky
  for (int j = 0; j < K; ++j) {
    const double d = sqrt(L[tri_idx(j, j)].x);
    const double inv = 1.0 / d;
    for (int i = j + tid; i < K; i += CHOL_NT) {
      const double2 v = L[tri_idx(i, j)];
      col[i] = (i == j) ? make_double2(d, 0.0) : make_double2(v.x * inv, v.y * inv);
    }
    __syncthreads();
    for (int i = j + tid; i < K; i += CHOL_NT) L[tri_idx(i, j)] = col[i];
    for (int i = j + 1 + ty; i < K; i += NY) {
      const double2 a = col[i];
      for (int k = j + 1 + tx; k <= i; k += 16) {   // A_ik -= L_ij conj(L_kj)
        const double2 b = col[k];
        double2 v = L[tri_idx(i, k)];
        v.x -= a.x * b.x + a.y * b.y;
        v.y -= a.y * b.x - a.x * b.y;
        L[tri_idx(i, k)] = v;
      }
    }
    __syncthreads();
  }
  // 3. X = L^-1 in place
  for (int k = 0; k < K; ++k) {
    // X_kk stays in a register until the end of the step: slot (k, k) still
    // holds L_kk for the threads that read it at the start
    const double xkk = 1.0 / L[tri_idx(k, k)].x;
    for (int i = k + 1 + tid; i < K; i += CHOL_NT) col[i] = L[tri_idx(i, k)];   // column k of L
    for (int j = tid; j < k; j += CHOL_NT) {                                    // row k of X
      const double2 bkj = L[tri_idx(k, j)];
      L[tri_idx(k, j)] = make_double2(bkj.x * xkk, bkj.y * xkk);
    }
    __syncthreads();
    for (int i = k + 1 + ty; i < K; i += NY) {
      const double2 l = col[i];
      for (int j = tx; j <= k; j += 16) {   // B_ij -= L_ik X_kj (B_ik starts at 0)
        const double2 x = (j == k) ? make_double2(xkk, 0.0) : L[tri_idx(k, j)];
        double2 v = (j == k) ? make_double2(0.0, 0.0) : L[tri_idx(i, j)];
        v.x -= l.x * x.x - l.y * x.y;
        v.y -= l.x * x.y + l.y * x.x;
        L[tri_idx(i, j)] = v;
      }
    }
    if (tid == 0) L[tri_idx(k, k)] = make_double2(xkk, 0.0);
    __syncthreads();
  }
  // 4. C = X^H X (upper triangle and its imaginary parts)
  float* Co = Cm + (size_t)p * fs;
  for (int i = ty; i < K; i += NY) {
    for (int j = i + tx; j < K; j += 16) {
      double sr = 0.0, si = 0.0;
      for (int k = j; k < K; ++k) {
        const double2 a = L[tri_idx(k, i)], b = L[tri_idx(k, j)];   // conj(X_ki) X_kj
        sr += a.x * b.x + a.y * b.y;
        si += a.x * b.y - a.y * b.x;
      }
      Co[i * ld + j] = (float)sr;
      if (i < j) Co[j * ld + i] = (float)si;
    }
  }
}

}  // namespace ocsc
