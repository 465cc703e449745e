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


__device__ __forceinline__ v4f mfma_bf16(v8bf a, v8bf b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// -x for eight BF16 values (sign bits flipped; exact)
__device__ __forceinline__ v8bf bf_neg(v8bf x) {
  typedef unsigned int v4u __attribute__((ext_vector_type(4)));
  v4u u = __builtin_bit_cast(v4u, x);
  u ^= 0x80008000u;
  return __builtin_bit_cast(v8bf, u);
}

// NW waves per workgroup, NSPLIT workgroups per frequency p (blockIdx.x = p,
// blockIdx.y = share of the tiles); CH samples per staged chunk (a multiple
// of 32: one k-step of the products per 32).  Up to K = 112 with 8 waves the
// registers are held to 128 per lane (chunks of 32 samples), so that two
// workgroups share a CU and cover each other's load and write phases; with
// the whole register file one workgroup per CU ran alone.  Zt[(p * ldt + b) * K + k] holds the nb
// pending code spectra frequency-major; xh[b * Pf + p] the sample spectra.
// H_p (R-form, rows of pitch K + 1 at Hm + p * fs) and G[k][p] are updated in
// place.  The product tiles on and above the diagonal are spread over the
// workgroups and waves (tile = y + NSPLIT (wave + NW tt)); operand layout of
// v_mfma_f32_16x16x32_bf16: A[i][8g..8g+7] in lane i + 16 g,
// B[8g..8g+7][j] in lane j + 16 g, D[i][j] in lane j + 16 (i / 4),
// register i % 4.
template <int KP, int NW, int NSPLIT, int CH>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(NW <= 8 && KP <= 112 ? 4 : 1))) void k_herk_bf16(const float2* __restrict__ Zt, int ldt, int nb,
                                                      const float2* __restrict__ xh, int Pf, float* __restrict__ Hm,
                                                      int fs, float2* __restrict__ G, int K) {
  constexpr int HERK_B = CH;            // samples per chunk
  constexpr int HERK_LD = HERK_B + 8;   // LDS row pitch (bf16) of the transposed parts
  constexpr int NT = 64 * NW;
  constexpr int NTD = KP / 16;                    // tiles per dimension
  constexpr int NTILE = NTD * (NTD + 1) / 2;      // tiles on or above the diagonal
  constexpr int TPW = (NTILE + NW * NSPLIT - 1) / (NW * NSPLIT);   // tiles per wave
  __shared__ __align__(16) __bf16 zrh[KP * HERK_LD], zrl[KP * HERK_LD], zih[KP * HERK_LD], zil[KP * HERK_LD];
  // G: GS threads per filter k, each summing every GS-th sample of a chunk; x_b staged in LDS
  constexpr int GS = NT / KP > 8 ? 8 : NT / KP;
  __shared__ float2 xs[HERK_B], gpart[GS * KP];
  const int p = blockIdx.x, split = blockIdx.y;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, li = lane & 15, lg = lane >> 4;
  auto tile_of = [&](int tt) { return split + NSPLIT * (wave + NW * tt); };
  int tri[TPW], trj[TPW];
#pragma unroll
  for (int tt = 0; tt < TPW; ++tt) {   // upper-triangular tile enumeration (row-major)
    int t = min(tile_of(tt), NTILE - 1), i = 0;
    while (t >= NTD - i) {
      t -= NTD - i;
      ++i;
    }
    tri[tt] = i;
    trj[tt] = i + t;
  }
  v4f re[TPW], im[TPW];
#pragma unroll
  for (int tt = 0; tt < TPW; ++tt) re[tt] = im[tt] = v4f{0, 0, 0, 0};

  float gr = 0.f, gi = 0.f;
  const int gk = tid % KP, gsl = tid / KP;   // this thread's filter and sample slice for G
  const float2* zp = Zt + (size_t)p * ldt * K;
  for (int b0 = 0; b0 < nb; b0 += HERK_B) {
    const int cb = min(HERK_B, nb - b0);
    __syncthreads();   // the previous chunk's operands are no longer read
    if (tid < HERK_B) xs[tid] = tid < cb ? xh[(size_t)(b0 + tid) * Pf + p] : make_float2(0.f, 0.f);
    // NW <= 8 (K <= 128): every load of the chunk is issued before the first
    // conversion, and the loads for G likewise (measured at K = 100: 875 ->
    // 703 us per launch).  With 16 waves the registers allow four loads in
    // flight per thread.
    if constexpr (NW > 8) {
      constexpr int QL = 4;
      for (int e0 = tid; e0 < HERK_B * KP; e0 += QL * NT) {
        float2 zv[QL];
#pragma unroll
        for (int q = 0; q < QL; ++q) {
          const int e = e0 + q * NT, b = e / KP, k = e - b * KP;   // consecutive threads read consecutive k
          zv[q] = (e < HERK_B * KP && b < cb && k < K) ? zp[(size_t)(b0 + b) * K + k] : make_float2(0.f, 0.f);
        }
#pragma unroll
        for (int q = 0; q < QL; ++q) {
          const int e = e0 + q * NT, b = e / KP, k = e - b * KP;
          if (e < HERK_B * KP) {
            const float2 z = zv[q];
            const __bf16 rh = (__bf16)z.x, ih = (__bf16)z.y;
            const int o = k * HERK_LD + b;
            zrh[o] = rh;
            zrl[o] = (__bf16)(z.x - (float)rh);
            zih[o] = ih;
            zil[o] = (__bf16)(z.y - (float)ih);
          }
        }
      }
    } else {
      constexpr int SPT = (HERK_B * KP + NT - 1) / NT;
      float2 zv[SPT];
#pragma unroll
      for (int q = 0; q < SPT; ++q) {
        const int e = tid + q * NT, b = e / KP, k = e - b * KP;   // consecutive threads read consecutive k
        zv[q] = (e < HERK_B * KP && b < cb && k < K) ? zp[(size_t)(b0 + b) * K + k] : make_float2(0.f, 0.f);
      }
#pragma unroll
      for (int q = 0; q < SPT; ++q) {
        const int e = tid + q * NT, b = e / KP, k = e - b * KP;
        if (HERK_B * KP % NT == 0 || e < HERK_B * KP) {
          const float2 z = zv[q];
          const __bf16 rh = (__bf16)z.x, ih = (__bf16)z.y;
          const int o = k * HERK_LD + b;
          zrh[o] = rh;
          zrl[o] = (__bf16)(z.x - (float)rh);
          zih[o] = ih;
          zil[o] = (__bf16)(z.y - (float)ih);
        }
      }
    }
    __syncthreads();
    if (NW > 8 && split == 0 && gsl < GS && gk < K) {   // G_p[k] += sum_b conj(z_bk) x_b (FP32), samples gsl, gsl + GS, ...
      constexpr int QL = 4;
      for (int bb = gsl; bb < cb; bb += QL * GS) {
        float2 zg[QL];
#pragma unroll
        for (int q = 0; q < QL; ++q) {   // four loads in flight
          const int b = bb + q * GS;
          zg[q] = b < cb ? zp[(size_t)(b0 + b) * K + gk] : make_float2(0.f, 0.f);
        }
#pragma unroll
        for (int q = 0; q < QL; ++q) {
          const int b = bb + q * GS;
          if (b < cb) {
            const float2 x = xs[b];
            gr += zg[q].x * x.x + zg[q].y * x.y;
            gi += zg[q].x * x.y - zg[q].y * x.x;
          }
        }
      }
    }
    if (NW <= 8 && split == 0 && gsl < GS && gk < K) {   // the same sums, loads issued together
      constexpr int GB = HERK_B / GS;
      float2 zg[GB];
#pragma unroll
      for (int q = 0; q < GB; ++q) {   // loads issued together
        const int b = gsl + q * GS;
        zg[q] = b < cb ? zp[(size_t)(b0 + b) * K + gk] : make_float2(0.f, 0.f);
      }
#pragma unroll
      for (int q = 0; q < GB; ++q) {
        const int b = gsl + q * GS;
        if (b < cb) {
          const float2 z = zg[q];
          const float2 x = xs[b];
          gr += z.x * x.x + z.y * x.y;
          gi += z.x * x.y - z.y * x.x;
        }
      }
    }
#pragma unroll
    for (int tt = 0; tt < TPW; ++tt) {
      if (tile_of(tt) >= NTILE) continue;
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
        // Im H_ij = sum_b zr_i zi_j - zi_i zr_j, formed transposed (row j,
        // column i: the j-block as operand A) so that the lower triangle of
        // the R-form, which holds it, is written row by row; the second sum
        // enters with its A operand negated, so one accumulator holds both
        im[tt] = mfma_bf16(bih, arh, im[tt]);
        im[tt] = mfma_bf16(bil, arh, im[tt]);
        im[tt] = mfma_bf16(bih, arl, im[tt]);
        const v8bf nbrh = bf_neg(brh), nbrl = bf_neg(brl);
        im[tt] = mfma_bf16(nbrh, aih, im[tt]);
        im[tt] = mfma_bf16(nbrl, aih, im[tt]);
        im[tt] = mfma_bf16(nbrh, ail, im[tt]);
      }
    }
  }
  float* R = Hm + (size_t)p * fs;
  const int ld = K + 1;
#pragma unroll
  for (int tt = 0; tt < TPW; ++tt) {
    if (tile_of(tt) >= NTILE) continue;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = tri[tt] * 16 + 4 * lg + r, j = trj[tt] * 16 + li;   // Re H_ij at R[i][j], i <= j
      if (i < K && j < K && i <= j) R[i * ld + j] += re[tt][r];
      const int jt = trj[tt] * 16 + 4 * lg + r, it = tri[tt] * 16 + li;  // Im H_it,jt at R[jt][it], it < jt
      if (it < K && jt < K && it < jt) R[jt * ld + it] += im[tt][r];
    }
  }
  if (split == 0) {
    if (gsl < GS) gpart[gsl * KP + gk] = make_float2(gr, gi);
    __syncthreads();
    if (tid < K) {
      float2 g = G[(size_t)tid * Pf + p];
#pragma unroll
      for (int sl = 0; sl < GS; ++sl) {
        g.x += gpart[sl * KP + tid].x;
        g.y += gpart[sl * KP + tid].y;
      }
      G[(size_t)tid * Pf + p] = g;
    }
  }
}

// ---------------------------------------------------------------------------
// C_p = (H_p + rho_d I)^-1 in FP64, one workgroup per frequency, the lower
// triangle in LDS (packed, element (i, j) at i(i+1)/2 + j):
//   1. A = H + rho_d I (lower triangle, A_ij = conj(H_ji) for i > j);
//   2. Cholesky A = L L^H, right-looking, CHOL_B columns per step;
//   3. X = L^-1 in place, right-looking on [L | I], CHOL_B rows per step;
//   4. C = X^H X, C_ij = sum_{k >= max(i, j)} conj(X_ki) X_kj, rounded to FP32
//      in the R-form of C (rows of pitch K + 1 at Cm + p * fs).
// Blocking by CHOL_B cuts the barrier phases and the passes over the
// trailing triangle by CHOL_B; the small diagonal blocks are factorised and
// inverted redundantly by every thread in registers.
// Dynamic LDS: (N(N+1)/2 + 2 CHOL_B^2) complex doubles, N = K rounded up to
// CHOL_B (81 KB at K = 100, so that two workgroups of NT = 512 share a CU and
// cover each other's serial diagonal-block phases).  The trailing updates are
// flat lists of 2 x 2 tiles shared by all threads, so every step keeps the
// threads evenly busy.
// FULL = true: the input is A itself, a full Hermitian n x n block in FP64
// (row pitch CB_N, block p at Ain + p * CB_N * CB_N), and the output is the
// full inverse in the same layout (the blocks of the K > 128 form below).
// ---------------------------------------------------------------------------
__device__ __forceinline__ int tri_idx(int i, int j) { return i * (i + 1) / 2 + j; }

// v - a conj(b), v - a b and v + conj(a) b as four fused multiply-adds
__device__ __forceinline__ double2 zsub_mulc(double2 v, double2 a, double2 b) {
  return make_double2(fma(-a.x, b.x, fma(-a.y, b.y, v.x)), fma(-a.y, b.x, fma(a.x, b.y, v.y)));
}
__device__ __forceinline__ double2 zsub_mul(double2 v, double2 a, double2 b) {
  return make_double2(fma(-a.x, b.x, fma(a.y, b.y, v.x)), fma(-a.x, b.y, fma(-a.y, b.x, v.y)));
}
__device__ __forceinline__ double2 zadd_cmul(double2 v, double2 a, double2 b) {
  return make_double2(fma(a.x, b.x, fma(a.y, b.y, v.x)), fma(a.x, b.y, fma(-a.y, b.x, v.y)));
}

constexpr int CHOL_NT = 1024;   // threads per workgroup: 16 waves share each step's work
constexpr int CHOL_B = 4;       // columns (rows) per step of the factorisation (inverse)
constexpr int CB_N = 128;       // block size of the K > 128 form

template <bool FULL, int NT>
__global__ __launch_bounds__(NT) void k_chol_inv_t(const float* __restrict__ Hm, float* __restrict__ Cm,
                                                   const double2* __restrict__ Ain, double2* __restrict__ Cout,
                                                   int K, int fs, double rho_d, int* __restrict__ breakdown) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  // the factorisation runs on N = K rounded up to CHOL_B, padded with the
  // identity (which stays outside the top-left K x K of the inverse)
  const int N = (K + CHOL_B - 1) / CHOL_B * CHOL_B;
  double2* L = reinterpret_cast<double2*>(smem_raw);
  double2* xdb = L + N * (N + 1) / 2;   // 2 x [CHOL_B][CHOL_B]: factor (step 2) / inverses (step 3) of diagonal blocks
  const int p = blockIdx.x, tid = threadIdx.x;
  const int ld = K + 1;
  for (int e = tid; e < N * (N + 1) / 2; e += NT) {
    int i = (int)((sqrtf(8.f * (float)e + 1.f) - 1.f) * 0.5f);
    while (tri_idx(i + 1, 0) <= e) ++i;
    while (tri_idx(i, 0) > e) --i;
    const int j = e - tri_idx(i, 0);
    double2 v;
    if (i >= K) {
      v = make_double2(i == j ? 1.0 : 0.0, 0.0);
    } else if constexpr (FULL) {
      v = Ain[(size_t)p * CB_N * CB_N + i * CB_N + j];
    } else {
      const float* R = Hm + (size_t)p * fs;
      v = (i == j) ? make_double2((double)R[i * ld + i] + rho_d, 0.0)
                   : make_double2((double)R[j * ld + i], -(double)R[i * ld + j]);
    }
    L[e] = v;
  }
  __syncthreads();
  // 2. Cholesky A = L L^H, CHOL_B columns per step (right-looking):
  //    one wave factors the CHOL_B x CHOL_B diagonal block D and shares it
  //    through LDS; each row below solves l_i D^H = a_i in place; then the
  //    trailing triangle takes the rank-CHOL_B update
  //    A_ik -= sum_c l_ic conj(l_kc) in 2 x 2 tiles.
  //    Look-ahead: the next diagonal block needs only this step's update of
  //    its own entries.  Wave 0 applies that update in registers and factors
  //    the block while the other waves update the rest of the trailing
  //    triangle (its L entries are stale until the factor overwrites them in
  //    the next step); the factors alternate between two LDS buffers.
  auto factor_block = [&](const double2 (&a)[CHOL_B][CHOL_B], double2* dst) {   // a: lower triangle
    double2 d[CHOL_B][CHOL_B];
#pragma unroll
    for (int c = 0; c < CHOL_B; ++c)
#pragma unroll
      for (int r = 0; r < CHOL_B; ++r) d[r][c] = make_double2(0.0, 0.0);
#pragma unroll
    for (int c = 0; c < CHOL_B; ++c) {
      double sdiag = a[c][c].x;
#pragma unroll
      for (int m = 0; m < c; ++m) sdiag -= d[c][m].x * d[c][m].x + d[c][m].y * d[c][m].y;
      // a pivot that is not positive (or not a number): the matrix is not
      // Hermitian positive definite; the factor goes on with NaN, and the
      // context reports the breakdown at its next call that waits
      if (!(sdiag > 0.0) && tid == 0) atomicOr(breakdown, 1);
      const double dc = sqrt(sdiag), ic = 1.0 / dc;
      d[c][c] = make_double2(dc, ic);   // the diagonal is real; its .y carries 1 / d_cc
#pragma unroll
      for (int r = c + 1; r < CHOL_B; ++r) {
        double2 v = a[r][c];
#pragma unroll
        for (int m = 0; m < c; ++m) v = zsub_mulc(v, d[r][m], d[c][m]);
        d[r][c] = make_double2(v.x * ic, v.y * ic);
      }
    }
    if (tid == 0)
#pragma unroll
      for (int r = 0; r < CHOL_B; ++r)
#pragma unroll
        for (int c = 0; c < CHOL_B; ++c) dst[r * CHOL_B + c] = d[r][c];
  };
  if (tid < 64) {
    double2 a[CHOL_B][CHOL_B];
#pragma unroll
    for (int r = 0; r < CHOL_B; ++r)
#pragma unroll
      for (int c = 0; c < CHOL_B; ++c) a[r][c] = c <= r ? L[tri_idx(r, c)] : make_double2(0.0, 0.0);
    factor_block(a, xdb);
  }
  __syncthreads();
  for (int j = 0, cur = 0; j < N; j += CHOL_B, cur ^= 1) {
    const double2* xc = xdb + cur * CHOL_B * CHOL_B;   // this block's factor
    double2* xn = xdb + (cur ^ 1) * CHOL_B * CHOL_B;   // the next block's
    double2 d[CHOL_B][CHOL_B];
    double dinv[CHOL_B];
#pragma unroll
    for (int r = 0; r < CHOL_B; ++r)
#pragma unroll
      for (int c = 0; c < CHOL_B; ++c) d[r][c] = xc[r * CHOL_B + c];
#pragma unroll
    for (int c = 0; c < CHOL_B; ++c) {
      dinv[c] = d[c][c].y;
      d[c][c].y = 0.0;
    }
    // panel rows in place (each thread reads and writes its own rows)
    for (int i = j + CHOL_B + tid; i < N; i += NT) {
      const int ri = tri_idx(i, 0) + j;
      double2 l[CHOL_B];
#pragma unroll
      for (int c = 0; c < CHOL_B; ++c) {
        double2 v = L[ri + c];
#pragma unroll
        for (int m = 0; m < c; ++m) v = zsub_mulc(v, l[m], d[c][m]);
        l[c] = make_double2(v.x * dinv[c], v.y * dinv[c]);
      }
#pragma unroll
      for (int c = 0; c < CHOL_B; ++c) L[ri + c] = l[c];
    }
    if (tid == 0) {
#pragma unroll
      for (int r = 0; r < CHOL_B; ++r)
#pragma unroll
        for (int c = 0; c <= r; ++c) L[tri_idx(j + r, j + c)] = d[r][c];
    }
    __syncthreads();
    const int j0 = j + CHOL_B;
    if (tid < 64) {
      if (j0 < N) {   // the next diagonal block: this step's update, then its factor
        double2 a[CHOL_B][CHOL_B];
#pragma unroll
        for (int r = 0; r < CHOL_B; ++r) {
#pragma unroll
          for (int c = 0; c < CHOL_B; ++c) {
            double2 v = make_double2(0.0, 0.0);
            if (c <= r) {
              v = L[tri_idx(j0 + r, j0 + c)];
#pragma unroll
              for (int q = 0; q < CHOL_B; ++q)
                v = zsub_mulc(v, L[tri_idx(j0 + r, j + q)], L[tri_idx(j0 + c, j + q)]);
            }
            a[r][c] = v;
          }
        }
        factor_block(a, xn);
      }
    } else {
      // the rest of the trailing triangle in 2 x 2 tiles, a flat list over
      // waves 1..; tiles 0..2 are the next diagonal block
      const int t2 = (N - j0) / 2;
      for (int t = 3 + tid - 64; t < t2 * (t2 + 1) / 2; t += NT - 64) {
        int ti = (int)((sqrtf(8.f * (float)t + 1.f) - 1.f) * 0.5f);
        while (tri_idx(ti + 1, 0) <= t) ++ti;
        while (tri_idx(ti, 0) > t) --ti;
        const int tk = t - tri_idx(ti, 0);
        const int i = j0 + 2 * ti, k = j0 + 2 * tk;   // rows i, i+1; columns k, k+1 (k <= i)
        const int r0 = tri_idx(i, 0), r1 = tri_idx(i + 1, 0), q0 = tri_idx(k, 0), q1 = tri_idx(k + 1, 0);
        double2 a[2][CHOL_B], b[2][CHOL_B];
#pragma unroll
        for (int c = 0; c < CHOL_B; ++c) {
          a[0][c] = L[r0 + j + c];
          a[1][c] = L[r1 + j + c];
          b[0][c] = L[q0 + j + c];
          b[1][c] = L[q1 + j + c];
        }
        double2 v00 = L[r0 + k], v10 = L[r1 + k], v11 = L[r1 + k + 1];
        double2 v01 = (k + 1 <= i) ? L[r0 + k + 1] : make_double2(0.0, 0.0);
#pragma unroll
        for (int c = 0; c < CHOL_B; ++c) {   // A_ik -= sum_c l_ic conj(l_kc)
          v00 = zsub_mulc(v00, a[0][c], b[0][c]);
          v01 = zsub_mulc(v01, a[0][c], b[1][c]);
          v10 = zsub_mulc(v10, a[1][c], b[0][c]);
          v11 = zsub_mulc(v11, a[1][c], b[1][c]);
        }
        L[r0 + k] = v00;
        L[r1 + k] = v10;
        L[r1 + k + 1] = v11;
        if (k + 1 <= i) L[r0 + k + 1] = v01;
      }
    }
    __syncthreads();
  }
  // 3. X = L^-1 in place, CHOL_B rows per step (right-looking on [L | I]):
  //    B starts as I; per step one wave inverts the diagonal block (Xd, shared
  //    through LDS), rows k.. of B become rows of X, then the rows below take
  //    B_ij -= sum_c L_i,k+c X_k+c,j: first for the columns left of the block
  //    (which read the block's column of L), then for the block's own columns
  //    (which overwrite it; one thread per row pair).  Slot (i, j) holds L
  //    until column j is consumed, then B, then X.
  //    Look-ahead: the inverse of the next diagonal block (final L, untouched
  //    by this step) is formed by wave 0 while the other waves update the
  //    rows below; the two inverses alternate between two LDS buffers.
  auto inv_diag = [&](int k, double2* dst) {   // every lane of wave 0 alike; lane 0 stores
    double2 xd[CHOL_B][CHOL_B];
#pragma unroll
    for (int c = 0; c < CHOL_B; ++c)
#pragma unroll
      for (int r = 0; r < CHOL_B; ++r) xd[r][c] = make_double2(0.0, 0.0);
#pragma unroll
    for (int c = 0; c < CHOL_B; ++c) {
      xd[c][c] = make_double2(1.0 / L[tri_idx(k + c, k + c)].x, 0.0);
#pragma unroll
      for (int r = c + 1; r < CHOL_B; ++r) {
        // xd[r][c] = -(sum_{m=c}^{r-1} L_{k+r,k+m} xd[m][c]) / L_{k+r,k+r}
        double2 v = make_double2(0.0, 0.0);
#pragma unroll
        for (int m = c; m < r; ++m) v = zsub_mul(v, L[tri_idx(k + r, k + m)], xd[m][c]);
        const double ir = 1.0 / L[tri_idx(k + r, k + r)].x;
        xd[r][c] = make_double2(v.x * ir, v.y * ir);
      }
    }
    if (tid == 0)
#pragma unroll
      for (int r = 0; r < CHOL_B; ++r)
#pragma unroll
        for (int c = 0; c < CHOL_B; ++c) dst[r * CHOL_B + c] = xd[r][c];
  };
  if (tid < 64) inv_diag(0, xdb);
  __syncthreads();
  for (int k = 0, cur = 0; k < N; k += CHOL_B, cur ^= 1) {
    const double2* xc = xdb + cur * CHOL_B * CHOL_B;         // this block's inverse
    double2* xn = xdb + (cur ^ 1) * CHOL_B * CHOL_B;         // the next block's
    for (int jj = tid; jj < k; jj += NT) {   // rows k.. of X, columns left of the block
      double2 xd[CHOL_B][CHOL_B];
#pragma unroll
      for (int r = 0; r < CHOL_B; ++r)
#pragma unroll
        for (int c = 0; c <= r; ++c) xd[r][c] = xc[r * CHOL_B + c];
      double2 bq[CHOL_B];
#pragma unroll
      for (int m = 0; m < CHOL_B; ++m) bq[m] = L[tri_idx(k + m, jj)];
#pragma unroll
      for (int r = 0; r < CHOL_B; ++r) {
        double2 x = make_double2(0.0, 0.0);
#pragma unroll
        for (int m = 0; m <= r; ++m) x = zsub_mul(x, make_double2(-xd[r][m].x, -xd[r][m].y), bq[m]);
        L[tri_idx(k + r, jj)] = x;
      }
    }
    if (tid == 0) {
#pragma unroll
      for (int r = 0; r < CHOL_B; ++r)
#pragma unroll
        for (int c = 0; c <= r; ++c) L[tri_idx(k + r, k + c)] = xc[r * CHOL_B + c];
    }
    __syncthreads();
    if (tid < 64) {
      if (k + CHOL_B < N) inv_diag(k + CHOL_B, xn);
    } else {
      // rows below the block x columns left of it, in 2 x 2 tiles (waves 1..)
      const int nr = (N - k - CHOL_B) / 2, nc = k / 2;
      for (int t = tid - 64; t < nr * nc; t += NT - 64) {
        const int i = k + CHOL_B + 2 * (t / nc), jj = 2 * (t % nc);
        const int r0 = tri_idx(i, 0), r1 = tri_idx(i + 1, 0);
        double2 a[2][CHOL_B], x[CHOL_B][2];
#pragma unroll
        for (int c = 0; c < CHOL_B; ++c) {
          a[0][c] = L[r0 + k + c];
          a[1][c] = L[r1 + k + c];
          const int rx = tri_idx(k + c, 0) + jj;   // X rows k.. (written above)
          x[c][0] = L[rx];
          x[c][1] = L[rx + 1];
        }
        double2 v[2][2];
#pragma unroll
        for (int rr = 0; rr < 2; ++rr)
#pragma unroll
          for (int q = 0; q < 2; ++q) v[rr][q] = L[(rr ? r1 : r0) + jj + q];
#pragma unroll
        for (int c = 0; c < CHOL_B; ++c)
#pragma unroll
          for (int rr = 0; rr < 2; ++rr)
#pragma unroll
            for (int q = 0; q < 2; ++q) v[rr][q] = zsub_mul(v[rr][q], a[rr][c], x[c][q]);
#pragma unroll
        for (int rr = 0; rr < 2; ++rr)
#pragma unroll
          for (int q = 0; q < 2; ++q) L[(rr ? r1 : r0) + jj + q] = v[rr][q];
      }
    }
    __syncthreads();
    // the block's own columns: B_i,k+q = -sum_{c >= q} L_i,k+c Xd[c][q] (B starts at 0)
    for (int i = k + CHOL_B + 2 * tid; i < N; i += 2 * NT) {
#pragma unroll
      for (int rr = 0; rr < 2; ++rr) {
        const int ri = tri_idx(i + rr, 0) + k;
        double2 a[CHOL_B];
#pragma unroll
        for (int c = 0; c < CHOL_B; ++c) a[c] = L[ri + c];
#pragma unroll
        for (int q = 0; q < CHOL_B; ++q) {
          double2 v = make_double2(0.0, 0.0);
#pragma unroll
          for (int c = q; c < CHOL_B; ++c) v = zsub_mul(v, a[c], xc[c * CHOL_B + q]);   // Xd from LDS
          L[ri + q] = v;
        }
      }
    }
    __syncthreads();
  }
  // 4. C = X^H X, C_ij = sum_{m >= j} conj(X_mi) X_mj for i <= j, in 2 x 2
  //    blocks (four loads for four products per m).  X is block diagonal
  //    with the identity padding, so the sums may run to N; only m = j0 meets
  //    the zero upper triangle (X_m,j0+1 for m = j0).
  const int n2 = N / 2, ntile = n2 * (n2 + 1) / 2;
  // the sums get shorter along the tile list (m runs from j0 + 1 to N), so
  // the rounds alternate direction and each thread's tiles even out
  for (int rd = 0; rd * NT < ntile; ++rd) {
    const int t = (rd & 1) ? (rd + 1) * NT - 1 - tid : rd * NT + tid;
    if (t >= ntile) continue;
    int r = (int)((sqrtf(8.f * (float)t + 1.f) - 1.f) * 0.5f);   // t = r (r + 1) / 2 + c, c <= r
    while (tri_idx(r + 1, 0) <= t) ++r;
    while (tri_idx(r, 0) > t) --r;
    const int i0 = 2 * (t - tri_idx(r, 0)), j0 = 2 * r;   // tile rows i0, i0 + 1 <= columns j0, j0 + 1
    double2 acc[2][2];
    {
      const int r0 = tri_idx(j0, 0);   // m = j0: X_j0,j0+1 = 0
      const double2 xi0 = L[r0 + i0], xi1 = (i0 + 1 <= j0) ? L[r0 + i0 + 1] : make_double2(0.0, 0.0);
      const double2 xj0 = L[r0 + j0];
      acc[0][0] = zadd_cmul(make_double2(0.0, 0.0), xi0, xj0);
      acc[1][0] = zadd_cmul(make_double2(0.0, 0.0), xi1, xj0);
      acc[0][1] = make_double2(0.0, 0.0);
      acc[1][1] = make_double2(0.0, 0.0);
    }
    for (int m = j0 + 1; m < N; ++m) {
      const int rm = tri_idx(m, 0);
      const double2 xi[2] = {L[rm + i0], L[rm + i0 + 1]};
      const double2 xj[2] = {L[rm + j0], L[rm + j0 + 1]};
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = zadd_cmul(acc[a][b], xi[a], xj[b]);   // + conj(xi) xj
    }
#pragma unroll
    for (int a = 0; a < 2; ++a) {
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const int i = i0 + a, jx = j0 + b;
        if (i >= K || jx >= K || i > jx) continue;
        const double sr = acc[a][b].x, si = acc[a][b].y;
        if constexpr (FULL) {
          double2* Co = Cout + (size_t)p * CB_N * CB_N;
          Co[i * CB_N + jx] = make_double2(sr, si);
          Co[jx * CB_N + i] = make_double2(sr, -si);
        } else {
          float* Co = Cm + (size_t)p * fs;
          Co[i * ld + jx] = (float)sr;
          if (i < jx) Co[jx * ld + i] = (float)si;
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// C_p = (H_p + rho_d I)^-1 in FP64 on the matrix cores, one workgroup of 8
// waves per frequency, for N = K rounded up to 16 <= 128 (NB <= 8 blocks of
// 16 x 16).  Used for the 128-blocks of the K > 128 form (FULL): 1.05 ms per
// 2048 frequencies against 1.46 ms for k_chol_inv_t.  At K = 100 its 122 KB
// of LDS leave one workgroup per CU, and k_chol_inv_t, two per CU, is
// faster there (2.56 against 3.18 ms).  The lower triangle of blocks lives in LDS (each block 16 rows of
// pitch 17 complex doubles, so that the 16 rows read by one operand load
// fall in different banks).  Every block product is a 16 x 16 x 16 complex
// product on v_mfma_f64_16x16x4_f64 (operand A[i][k] in lane i + 16 k,
// B[k][j] in lane j + 16 k, result D[i][j] in lane j + 16 (i % 4), element
// i / 4 -- the rows of a lane's four results are strided, unlike the FP32
// form; checked by an in-bounds probe), three real products per complex one:
//   P1 = Ar Br, P2 = Ai Bi, P3 = (Ar + Ai)(Br + Bi);  Re = P1 - P2, Im = P3 - P1 - P2.
//   1. A = H + rho_d I (identity padding beyond K).
//   2. Blocked right-looking Cholesky A = L L^H: per block column j, the
//      diagonal block is factorised and inverted by one wave (W_jj = L_jj^-1,
//      kept in place of L_jj), the panel becomes L_ij = A_ij W_jj^H, and the
//      trailing blocks take A_ik -= L_ij L_kj^H.  Look-ahead: wave 0 first
//      updates the next diagonal block and factorises it while the other waves
//      update the rest of the trailing triangle.
//   3. X = L^-1, right-looking per block column k: row k becomes
//      X_kj = W_kk B_kj; then the rows below take B_ij -= L_ik X_kj (j < k)
//      and, once those have read L_ik, B_ik = -L_ik W_kk (B holds the rows
//      below).
//   4. C = X^H X: C_ij = sum_{m >= j} X_mi^H X_mj for the blocks on and above
//      the diagonal, written to the R-form (FP32) or, FULL, to a dense
//      128 x 128 FP64 block (both triangles).
// The diagonal blocks: in 4 x 4 steps, every lane of the wave factorises the
// 4 x 4 diagonal piece in registers, the rows below solve against it, the
// rest of the block takes the rank-4 update; then each of 16 lanes forms one
// column of W_jj by forward substitution.
// ---------------------------------------------------------------------------
typedef double v4d __attribute__((ext_vector_type(4)));
constexpr int CM_P = 17;            // LDS row pitch of a block (complex doubles)
constexpr int CM_BS = 16 * CM_P;    // complex doubles per stored block
constexpr int CM_NT = 512;          // 8 waves (up to 256 registers per lane)
constexpr int CM_NW = CM_NT / 64;

__host__ __device__ constexpr int cm_lblk(int i, int j) { return i * (i + 1) / 2 + j; }   // lower block, i >= j
__host__ constexpr size_t cm_lds(int K) {
  const int nb = (K + 15) / 16;
  return (size_t)cm_lblk(nb, 0) * CM_BS * 16;
}

__device__ __forceinline__ v4d mfma_f64(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Intra-wave ordering of LDS accesses (the wave's lanes exchange data through LDS).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Accumulators of one 16 x 16 complex block: P1, P2, P3 of the three-product form.
struct ZAcc {
  v4d p1, p2, p3;
};
__device__ __forceinline__ void zacc_zero(ZAcc& z) { z.p1 = z.p2 = z.p3 = v4d{0, 0, 0, 0}; }

// z += op(A) op(B) over k = 0..15 for blocks A, B in LDS; HA / HB: the
// conjugate transpose of the stored block; NEG: subtract.
template <bool HA, bool HB, bool NEG>
__device__ __forceinline__ void zmma16(ZAcc& z, const double2* __restrict__ A, const double2* __restrict__ B,
                                       int lane) {
  const int i = lane & 15, kk = lane >> 4;
#pragma unroll
  for (int k0 = 0; k0 < 16; k0 += 4) {
    const int k = k0 + kk;
    double2 a = HA ? A[k * CM_P + i] : A[i * CM_P + k];   // A[i][k]
    double2 b = HB ? B[i * CM_P + k] : B[k * CM_P + i];   // B[k][j], j = lane & 15
    if (HA) a.y = -a.y;
    if (HB) b.y = -b.y;
    if (NEG) {
      a.x = -a.x;
      a.y = -a.y;
    }
    z.p1 = mfma_f64(a.x, b.x, z.p1);
    z.p2 = mfma_f64(a.y, b.y, z.p2);
    z.p3 = mfma_f64(a.x + a.y, b.x + b.y, z.p3);
  }
}

// element e of this lane's share of the block: row lane / 16 + 4 e, column lane % 16
__device__ __forceinline__ double2 zacc_get(const ZAcc& z, int e) {
  return make_double2(z.p1[e] - z.p2[e], z.p3[e] - z.p1[e] - z.p2[e]);
}
// a block held as (re, im) is loaded into the accumulators as P1 = re, P2 = 0, P3 = re + im
__device__ __forceinline__ void zacc_load(ZAcc& z, const double2* __restrict__ D, int lane) {
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const double2 v = D[((lane >> 4) + 4 * e) * CM_P + (lane & 15)];
    z.p1[e] = v.x;
    z.p2[e] = 0.0;
    z.p3[e] = v.x + v.y;
  }
}
__device__ __forceinline__ void zacc_store(const ZAcc& z, double2* __restrict__ D, int lane) {
#pragma unroll
  for (int e = 0; e < 4; ++e) D[((lane >> 4) + 4 * e) * CM_P + (lane & 15)] = zacc_get(z, e);
}

// Factorise the 16 x 16 diagonal block D (lower triangle, Hermitian positive
// definite) and replace it by W = L^-1 (lower, zeros above).  One wave.
__device__ __forceinline__ void cm_diag_block(double2* __restrict__ D, int lane, int* __restrict__ breakdown) {
  // Cholesky in four steps of 4 columns
#pragma unroll
  for (int s = 0; s < 16; s += 4) {
    double2 d[4][4];   // factor of the 4 x 4 diagonal piece, every lane alike; .y of d[c][c] = 1 / d_cc
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int c = 0; c < 4; ++c) d[r][c] = make_double2(0.0, 0.0);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      double sd = D[(s + c) * CM_P + s + c].x;
#pragma unroll
      for (int m = 0; m < c; ++m) sd -= d[c][m].x * d[c][m].x + d[c][m].y * d[c][m].y;
      if (!(sd > 0.0) && lane == 0) atomicOr(breakdown, 1);
      const double dc = sqrt(sd), ic = 1.0 / dc;
      d[c][c] = make_double2(dc, ic);
#pragma unroll
      for (int r = c + 1; r < 4; ++r) {
        double2 v = D[(s + r) * CM_P + s + c];
#pragma unroll
        for (int m = 0; m < c; ++m) v = zsub_mulc(v, d[r][m], d[c][m]);
        d[r][c] = make_double2(v.x * ic, v.y * ic);
      }
    }
    // rows below the piece: l_r = a_r D^-H, one lane per row
    const int r = s + 4 + lane;
    double2 l[4];
    if (lane < 12 - s) {
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        double2 v = D[r * CM_P + s + c];
#pragma unroll
        for (int m = 0; m < c; ++m) v = zsub_mulc(v, l[m], d[c][m]);
        l[c] = make_double2(v.x * d[c][c].y, v.y * d[c][c].y);
      }
    }
    wave_sync();   // every lane has read the piece and its row before they are overwritten
    if (lane < 4) {
#pragma unroll
      for (int c = 0; c < 4; ++c)
        if (c <= lane) {
          // the lane's row of the factored piece (compile-time selection of d)
          double2 v = make_double2(0.0, 0.0);
#pragma unroll
          for (int rr = 0; rr < 4; ++rr)
            if (rr == lane) v = (rr == c) ? make_double2(d[rr][rr].x, 0.0) : d[rr][c];
          D[(s + lane) * CM_P + s + c] = v;
        }
    }
    if (lane < 12 - s) {
#pragma unroll
      for (int c = 0; c < 4; ++c) D[r * CM_P + s + c] = l[c];
    }
    wave_sync();
    // trailing lower triangle of rows and columns s + 4 .. 15: A_rc -= sum_m l_rm conj(l_cm)
    const int n = 12 - s;
    for (int e = lane; e < n * n; e += 64) {
      const int rr = s + 4 + e / n, cc = s + 4 + e % n;
      if (cc <= rr) {
        double2 v = D[rr * CM_P + cc];
#pragma unroll
        for (int m = 0; m < 4; ++m) v = zsub_mulc(v, D[rr * CM_P + s + m], D[cc * CM_P + s + m]);
        D[rr * CM_P + cc] = v;
      }
    }
    wave_sync();
  }
  // W = L^-1 by forward substitution, lane c < 16 forming column c in
  // registers (W_rc = (delta_rc - sum_{c <= m < r} L_rm W_mc) / L_rr; the L
  // entries are the same for every lane)
  const int c = lane & 15;
  double2 w[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    double2 v = make_double2(r == c ? 1.0 : 0.0, 0.0);
#pragma unroll
    for (int m = 0; m < r; ++m) v = zsub_mul(v, D[r * CM_P + m], w[m]);   // w[m] = 0 for m < c
    const double ir = 1.0 / D[r * CM_P + r].x;
    w[r] = (r >= c) ? make_double2(v.x * ir, v.y * ir) : make_double2(0.0, 0.0);
  }
  wave_sync();   // every lane has read L
  if (lane < 16) {
#pragma unroll
    for (int r = 0; r < 16; ++r) D[r * CM_P + c] = w[r];
  }
  wave_sync();
}

template <bool FULL>
__global__ __launch_bounds__(CM_NT) void k_chol_inv_mfma(const float* __restrict__ Hm, float* __restrict__ Cm,
                                                         const double2* __restrict__ Ain,
                                                         double2* __restrict__ Cout, int K, int fs, double rho_d,
                                                         int* __restrict__ breakdown) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double2* Lb = reinterpret_cast<double2*>(smem_raw);
  const int NB = (K + 15) / 16;
  const int p = blockIdx.x, tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int ld = K + 1;
  auto blk = [&](int i, int j) { return Lb + (size_t)cm_lblk(i, j) * CM_BS; };
  // 1. A = H + rho_d I into the lower blocks (diagonal blocks: lower triangle)
  const int nel = cm_lblk(NB, 0) * 256;
  for (int t = tid; t < nel; t += CM_NT) {
    const int b = t >> 8, e = t & 255;
    int bi = 0;
    while (cm_lblk(bi + 1, 0) <= b) ++bi;
    const int bj = b - cm_lblk(bi, 0);
    const int r = e >> 4, cc = e & 15;
    const int i = bi * 16 + r, j = bj * 16 + cc;
    double2 v;
    if (i < j) {
      v = make_double2(0.0, 0.0);   // upper part of a diagonal block
    } else if (i >= K || j >= K) {
      v = make_double2(i == j ? 1.0 : 0.0, 0.0);
    } else if constexpr (FULL) {
      v = Ain[(size_t)p * CB_N * CB_N + i * CB_N + j];
    } else {
      const float* R = Hm + (size_t)p * fs;
      v = (i == j) ? make_double2((double)R[i * ld + i] + rho_d, 0.0)
                   : make_double2((double)R[j * ld + i], -(double)R[i * ld + j]);
    }
    Lb[(size_t)b * CM_BS + r * CM_P + cc] = v;
  }
  __syncthreads();
  // 2. blocked Cholesky; W_jj replaces L_jj
  if (wave == 0) cm_diag_block(blk(0, 0), lane, breakdown);
  __syncthreads();
  for (int j = 0; j < NB; ++j) {
    // panel: L_ij = A_ij W_jj^H
    for (int i = j + 1 + wave; i < NB; i += CM_NW) {
      ZAcc z;
      zacc_zero(z);
      zmma16<false, true, false>(z, blk(i, j), blk(j, j), lane);
      zacc_store(z, blk(i, j), lane);
    }
    __syncthreads();
    if (j + 1 < NB) {
      if (wave == 0) {
        // the next diagonal block first, then its factor
        ZAcc z;
        zacc_load(z, blk(j + 1, j + 1), lane);
        zmma16<false, true, true>(z, blk(j + 1, j), blk(j + 1, j), lane);
        zacc_store(z, blk(j + 1, j + 1), lane);
        wave_sync();
        cm_diag_block(blk(j + 1, j + 1), lane, breakdown);
      } else {
        // the rest of the trailing triangle: blocks (i, k), j < k <= i, except (j + 1, j + 1)
        const int n = NB - 1 - j;
        for (int t = 1 + (wave - 1); t < n * (n + 1) / 2; t += CM_NW - 1) {
          int ti = 0;
          while (cm_lblk(ti + 1, 0) <= t) ++ti;
          const int tk = t - cm_lblk(ti, 0);
          const int i = j + 1 + ti, k = j + 1 + tk;
          ZAcc z;
          zacc_load(z, blk(i, k), lane);
          zmma16<false, true, true>(z, blk(i, j), blk(k, j), lane);
          zacc_store(z, blk(i, k), lane);
        }
      }
    }
    __syncthreads();
  }
  // 3. X = L^-1, right-looking per block column k (X_kk = W_kk already)
  for (int k = 0; k < NB; ++k) {
    for (int jj = wave; jj < k; jj += CM_NW) {   // X_kj = W_kk B_kj
      ZAcc z;
      zacc_zero(z);
      zmma16<false, false, false>(z, blk(k, k), blk(k, jj), lane);
      zacc_store(z, blk(k, jj), lane);
    }
    __syncthreads();
    // B_ij -= L_ik X_kj for i > k, j < k (reads block (i, k))
    const int nr = NB - 1 - k;
    for (int t = wave; t < nr * k; t += CM_NW) {
      const int i = k + 1 + t / k, jj = t % k;
      ZAcc z;
      zacc_load(z, blk(i, jj), lane);
      zmma16<false, false, true>(z, blk(i, k), blk(k, jj), lane);
      zacc_store(z, blk(i, jj), lane);
    }
    if (k > 0) __syncthreads();
    // then B_ik = -L_ik W_kk overwrites block (i, k)
    for (int i = k + 1 + wave; i < NB; i += CM_NW) {
      ZAcc z;
      zacc_zero(z);
      zmma16<false, false, true>(z, blk(i, k), blk(k, k), lane);
      wave_sync();   // every lane's reads of L_ik are done before it is overwritten
      zacc_store(z, blk(i, k), lane);
    }
    __syncthreads();
  }
  // 4. C = X^H X, blocks (bi, bj) with bi <= bj
  for (int t = wave; t < NB * (NB + 1) / 2; t += CM_NW) {
    int bj = 0;
    while (cm_lblk(bj + 1, 0) <= t) ++bj;
    const int bi = t - cm_lblk(bj, 0);   // bi <= bj
    ZAcc z;
    zacc_zero(z);
    for (int m = bj; m < NB; ++m) zmma16<true, false, false>(z, blk(m, bi), blk(m, bj), lane);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int i = bi * 16 + (lane >> 4) + 4 * e, jx = bj * 16 + (lane & 15);
      if (i >= K || jx >= K || i > jx) continue;
      const double2 v = zacc_get(z, e);
      if constexpr (FULL) {
        double2* Co = Cout + (size_t)p * CB_N * CB_N;
        Co[i * CB_N + jx] = v;
        Co[jx * CB_N + i] = make_double2(v.x, -v.y);
      } else {
        float* Co = Cm + (size_t)p * fs;
        Co[i * ld + jx] = (float)v.x;
        if (i < jx) Co[jx * ld + i] = (float)v.y;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// K > 128 (up to 256): C_p = A^-1 for A = H_p + rho_d I from the FP64 block
// inverses of two Cholesky factors and a Schur complement.  With the split
// n1 = 128, n2 = K - 128 and every block stored as a full 128 x 128 FP64
// matrix (block 2 padded with the identity, so the padding stays out of the
// top-left K x K result):
//   P = A11^-1;  B = A21 P;  S = A22 - B A21^H;  Q = S^-1;
//   C22 = Q;  C21 = -Q B;  C11 = P - B^H C21.
// S is Hermitian positive definite whenever A is, so both inverses come from
// Cholesky factors.  Frequencies are processed in chunks; the five blocks of
// a frequency live at W + (slot * nfreq + f) * 128 * 128.
// ---------------------------------------------------------------------------

// Blocks A11, A21, A22 (slots 0, 2, 3) of A = H + rho_d I for frequencies
// [f0, f0 + nf), from H in R-form (FP32, rows of pitch K + 1).  Workgroup
// (blockIdx.x = block * 16 + 32 x 32 tile, blockIdx.y = frequency): the tile
// of R and its transpose pass through LDS, so both reads are row reads.
constexpr int SU_T = 32;

__global__ __launch_bounds__(256) void k_schur_unpack(const float* __restrict__ Hm, int fs, int K, double rho_d,
                                                      int f0, int nf, double2* __restrict__ W) {
  __shared__ float t1[SU_T][SU_T + 1], t2[SU_T][SU_T + 1];   // t1[r][c] = R[a][b], t2[c][r] = R[b][a]
  const int f = blockIdx.y, blk = blockIdx.x / 16, tile = blockIdx.x % 16;
  // A11 and A22: rows 0..63 x columns 64..127 are never read (the inverse
  // reads the lower triangle, S = A22 - B A21^H the tiles on and below the
  // diagonal of 64 x 64)
  if (blk != 1 && tile / 4 < 2 && tile % 4 >= 2) return;
  const int slot = blk == 0 ? 0 : (blk == 1 ? 2 : 3);
  const int abase = blk == 0 ? 0 : CB_N, bbase = blk == 2 ? CB_N : 0;
  const int a0 = abase + (tile / 4) * SU_T, b0 = bbase + (tile % 4) * SU_T;
  const float* R = Hm + (size_t)(f0 + f) * fs;
  const int ld = K + 1;
  for (int e = threadIdx.x; e < SU_T * SU_T; e += 256) {
    const int r = e / SU_T, c = e % SU_T;
    t1[r][c] = (a0 + r < K && b0 + c < K) ? R[(size_t)(a0 + r) * ld + b0 + c] : 0.f;
    t2[r][c] = (b0 + r < K && a0 + c < K) ? R[(size_t)(b0 + r) * ld + a0 + c] : 0.f;   // row b0 + r of R
  }
  __syncthreads();
  double2* out = W + ((size_t)slot * nf + f) * CB_N * CB_N;
  for (int e = threadIdx.x; e < SU_T * SU_T; e += 256) {
    const int r = e / SU_T, c = e % SU_T;
    const int a = a0 + r, b = b0 + c;
    double2 v;
    if (a >= K || b >= K) {
      v = make_double2(a == b ? 1.0 : 0.0, 0.0);   // identity padding (block 2 only)
    } else if (a == b) {
      v = make_double2((double)t1[r][c] + rho_d, 0.0);
    } else if (a < b) {
      v = make_double2((double)t1[r][c], (double)t2[c][r]);    // Re at R[a][b], Im at R[b][a]
    } else {
      v = make_double2((double)t2[c][r], -(double)t1[r][c]);   // conj(H_ba)
    }
    out[(size_t)(a - abase) * CB_N + (b - bbase)] = v;
  }
}

// Cout = beta Cin + alpha op(A) op(B) for 128 x 128 complex FP64 blocks, one
// frequency per blockIdx.z, a 64 x 64 output tile per workgroup (blockIdx.x,
// blockIdx.y), 256 threads with 4 x 4 outputs each; op = conjugate transpose
// when HA / HB.  Cin may alias Cout (each output is read, then written, by
// one thread).  LOWER: the result is Hermitian and only its lower triangle is
// used, so the tile above the diagonal is skipped (blockIdx.x = 0, 1, 2 for
// tiles (0, 0), (1, 0), (1, 1)).
constexpr int ZG_T = 64, ZG_K = 16;

template <bool HA, bool HB, bool LOWER = false>
__global__ __launch_bounds__(256) void k_zgemm128(const double2* __restrict__ A, const double2* __restrict__ B,
                                                  const double2* Cin, double2* Cout, double alpha, double beta) {
  __shared__ double2 as[ZG_K][ZG_T + 1];   // as[kk][i] = op(A)[i0 + i][k0 + kk]
  __shared__ double2 bs[ZG_K][ZG_T + 1];   // bs[kk][j] = op(B)[k0 + kk][j0 + j]
  const size_t off = (size_t)blockIdx.z * CB_N * CB_N;
  const double2* a = A + off;
  const double2* b = B + off;
  const int i0 = LOWER ? (blockIdx.x > 0 ? ZG_T : 0) : blockIdx.y * ZG_T;
  const int j0 = LOWER ? (blockIdx.x == 2 ? ZG_T : 0) : blockIdx.x * ZG_T;
  const int tid = threadIdx.x, ti = tid >> 4, tj = tid & 15;
  double2 acc[4][4];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[r][q] = make_double2(0.0, 0.0);
  for (int k0 = 0; k0 < CB_N; k0 += ZG_K) {
    for (int e = tid; e < ZG_K * ZG_T; e += 256) {
      // op(A)[i][k]: A[i][k], or conj(A[k][i]); consecutive threads take consecutive memory
      if (HA) {
        const int i = e % ZG_T, kk = e / ZG_T;
        const double2 v = a[(size_t)(k0 + kk) * CB_N + i0 + i];
        as[kk][i] = make_double2(v.x, -v.y);
      } else {
        const int kk = e % ZG_K, i = e / ZG_K;
        as[kk][i] = a[(size_t)(i0 + i) * CB_N + k0 + kk];
      }
      // op(B)[k][j]: B[k][j], or conj(B[j][k])
      if (HB) {
        const int kk = e % ZG_K, j = e / ZG_K;
        const double2 v = b[(size_t)(j0 + j) * CB_N + k0 + kk];
        bs[kk][j] = make_double2(v.x, -v.y);
      } else {
        const int j = e % ZG_T, kk = e / ZG_T;
        bs[kk][j] = b[(size_t)(k0 + kk) * CB_N + j0 + j];
      }
    }
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < ZG_K; ++kk) {
      double2 av[4], bv[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) av[r] = as[kk][ti + 16 * r];
#pragma unroll
      for (int q = 0; q < 4; ++q) bv[q] = bs[kk][tj + 16 * q];
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          acc[r][q].x = fma(av[r].x, bv[q].x, fma(-av[r].y, bv[q].y, acc[r][q].x));
          acc[r][q].y = fma(av[r].x, bv[q].y, fma(av[r].y, bv[q].x, acc[r][q].y));
        }
    }
    __syncthreads();
  }
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const size_t o = off + (size_t)(i0 + ti + 16 * r) * CB_N + j0 + tj + 16 * q;
      double2 v = make_double2(alpha * acc[r][q].x, alpha * acc[r][q].y);
      if (beta != 0.0) {
        const double2 c = Cin[o];
        v.x = fma(beta, c.x, v.x);
        v.y = fma(beta, c.y, v.y);
      }
      Cout[o] = v;
    }
}

// C_p in R-form (FP32, rows of pitch K + 1) from C11 (slot 1, its lower
// triangle only), C21 (slot 2) and C22 (slot 0) of frequencies [f0, f0 + nf):
// R[i][j] = Re C_ij for j >= i, -Im C_ij for j < i.  Workgroup (blockIdx.x =
// 32 x 32 tile of R, blockIdx.y = frequency).  On and above the diagonal in
// the first 128 rows, C_ij = conj(C21[j-128][i]) or conj(C11[j][i]): those
// tiles are read transposed through LDS.
__global__ __launch_bounds__(256) void k_schur_pack(const double2* __restrict__ W, int f0, int nf, int K, int fs,
                                                    float* __restrict__ Cm) {
  __shared__ double2 tt[SU_T][SU_T + 1];
  const int f = blockIdx.y, kt = (K + SU_T - 1) / SU_T;
  const int i0 = (blockIdx.x / kt) * SU_T, j0 = (blockIdx.x % kt) * SU_T;
  float* Co = Cm + (size_t)(f0 + f) * fs;
  const int ld = K + 1;
  const size_t bs = (size_t)CB_N * CB_N;
  const double2* c11 = W + (1 * (size_t)nf + f) * bs;
  const double2* c21 = W + (2 * (size_t)nf + f) * bs;
  const double2* c22 = W + (0 * (size_t)nf + f) * bs;
  if (i0 < CB_N && j0 >= i0) {
    // tt[r][c] = C[j0 + r][i0 + c]: row j0 + r - 128 of C21, or row j0 + r of C11
    const double2* src = j0 >= CB_N ? c21 + (size_t)(j0 - CB_N) * CB_N : c11 + (size_t)j0 * CB_N;
    for (int e = threadIdx.x; e < SU_T * SU_T; e += 256) {
      const int r = e / SU_T, c = e % SU_T;
      tt[r][c] = (j0 + r < K) ? src[(size_t)r * CB_N + i0 + c] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    for (int e = threadIdx.x; e < SU_T * SU_T; e += 256) {
      const int r = e / SU_T, c = e % SU_T, i = i0 + r, j = j0 + c;
      if (i >= K || j >= K) continue;
      // j >= i: Re C_ij = Re C_ji;  j < i (diagonal tiles, i0 = j0): -Im C_ij, with C_ij = tt[r][c]
      Co[i * ld + j] = (float)(j >= i ? tt[c][r].x : -tt[r][c].y);
    }
    return;
  }
  for (int e = threadIdx.x; e < SU_T * SU_T; e += 256) {
    const int r = e / SU_T, c = e % SU_T, i = i0 + r, j = j0 + c;
    if (i >= K || j >= K) continue;
    double2 v;
    if (i < CB_N && j < CB_N) v = c11[i * CB_N + j];   // j < i here
    else if (i >= CB_N && j >= CB_N) v = c22[(i - CB_N) * CB_N + (j - CB_N)];
    else v = c21[(i - CB_N) * CB_N + j];   // i >= 128 > j
    Co[i * ld + j] = (float)(j >= i ? v.x : -v.y);
  }
}

// ---------------------------------------------------------------------------
// D-step d_p = C_p r_p (eq. sub_d_sol, column form) for K > 128, where C_p
// (R-form, FP32, K (K + 1) reals) does not fit in LDS: one workgroup of 256
// threads per frequency; C_p passes through LDS in strips of 16 rows read
// once from HBM.  Each stored value v = R[a][b] serves two outputs:
//   a < b (v = Re C_ab = Re C_ba):  d_a += v r_b,      d_b += v r_a;
//   a > b (v = Im C_ba = -Im C_ab): d_a += -i v r_b,   d_b += i v r_a;
//   a = b:                          d_a += v r_a.
// The column role (output b) is one thread's running sum; the row role
// (output a) is summed by 16 lanes and reduced by shuffles.  rhs and d are
// complex [K][Pf].
// ---------------------------------------------------------------------------
constexpr int DS_ROWS = 16, DS_PITCH = 260;
constexpr int DS_V = (DS_ROWS * DS_PITCH / 4 + 255) / 256;   // 16-byte vectors per thread and strip

// A strip of rows [a0, a0 + nr) of C_p is one contiguous, 16-byte aligned
// run of nr (K + 1) reals (C_p starts at a multiple of 4 reals and 16 rows
// of pitch K + 1 are 64 (K + 1) bytes); it is copied as 16-byte vectors and
// keeps the pitch K + 1 in LDS (odd, so a column walk spreads over the banks).
__device__ __forceinline__ void ds_fetch(v4f (&pf)[DS_V], const float* __restrict__ R, int a0, int nr, int ld,
                                         int t) {
  const int nv = (nr * ld + 3) / 4;
  const v4f* src = reinterpret_cast<const v4f*>(R + (size_t)a0 * ld);
#pragma unroll
  for (int m = 0; m < DS_V; ++m) {
    const int v = t + m * 256;
    if (v < nv) pf[m] = src[v];
  }
}
__device__ __forceinline__ void ds_stage(const v4f (&pf)[DS_V], float* strip, int nr, int ld, int t) {
  const int nv = (nr * ld + 3) / 4;
#pragma unroll
  for (int m = 0; m < DS_V; ++m) {
    const int v = t + m * 256;
    if (v < nv) reinterpret_cast<v4f*>(strip)[v] = pf[m];
  }
}

__global__ __launch_bounds__(256) void k_dstep_stream(const float* __restrict__ Cm, int fs, int K, int Pf,
                                                      const float2* __restrict__ rhs, float2* __restrict__ dout) {
  __shared__ __align__(16) float strip[DS_ROWS * DS_PITCH];
  __shared__ float2 rv[256], drow[256];
  const int p = blockIdx.x, t = threadIdx.x;
  const int ld = K + 1;
  const float* R = Cm + (size_t)p * fs;
  if (t < K) {
    rv[t] = rhs[(size_t)t * Pf + p];
    drow[t] = make_float2(0.f, 0.f);
  }
  float2 dc = make_float2(0.f, 0.f);
  const int rr = t >> 4, q = t & 15;
  // the next strip is fetched into registers while the current one is used
  v4f pf[DS_V];
  ds_fetch(pf, R, 0, min(DS_ROWS, K), ld, t);
  __syncthreads();
  for (int a0 = 0; a0 < K; a0 += DS_ROWS) {
    const int nr = min(DS_ROWS, K - a0);
    ds_stage(pf, strip, nr, ld, t);
    __syncthreads();
    if (a0 + DS_ROWS < K) ds_fetch(pf, R, a0 + DS_ROWS, min(DS_ROWS, K - a0 - DS_ROWS), ld, t);
    if (t < K) {   // column role: output t
      for (int r = 0; r < nr; ++r) {
        const int a = a0 + r;
        const float v = strip[r * ld + t];
        const float2 ra = rv[a];
        if (a <= t) {
          dc.x = fma(v, ra.x, dc.x);
          dc.y = fma(v, ra.y, dc.y);
        } else {
          dc.x = fma(-v, ra.y, dc.x);
          dc.y = fma(v, ra.x, dc.y);
        }
      }
    }
    float2 sum = make_float2(0.f, 0.f);   // row role: output a0 + rr, columns q, q + 16, ...
    if (rr < nr) {
      const int a = a0 + rr;
      for (int b = q; b < K; b += 16) {
        if (b == a) continue;
        const float v = strip[rr * ld + b];
        const float2 rb = rv[b];
        if (a < b) {
          sum.x = fma(v, rb.x, sum.x);
          sum.y = fma(v, rb.y, sum.y);
        } else {
          sum.x = fma(v, rb.y, sum.x);
          sum.y = fma(-v, rb.x, sum.y);
        }
      }
    }
#pragma unroll
    for (int off = 8; off > 0; off >>= 1) {
      sum.x += __shfl_xor(sum.x, off, 16);
      sum.y += __shfl_xor(sum.y, off, 16);
    }
    if (rr < nr && q == 0) {
      float2 d = drow[a0 + rr];
      d.x += sum.x;
      d.y += sum.y;
      drow[a0 + rr] = d;
    }
    __syncthreads();   // the strip is overwritten next
  }
  if (t < K) dout[(size_t)t * Pf + p] = make_float2(dc.x + drow[t].x, dc.y + drow[t].y);
}

// ---------------------------------------------------------------------------
// One step of iterative refinement of the D-step solve (eq. sub_d_sol) in the
// precision form, against the history H_p the context keeps:
//   r_p = rhs_p - (H_p + rho_d I) d_p      (products of FP32 values, summed in FP64),
//   d_p <- d_p + C_p r_p                   (FP64 sums, rounded once to FP32).
// The FP64 Cholesky factors solve the stored H to ~1e-15; what the refinement
// removes is the error of using the FP32 rounding of C_p = (H_p + rho_d I)^-1.
// One workgroup of 256 threads per frequency; H_p and then C_p pass through
// LDS in strips of 16 rows, each stored real serving a row and a column
// output as in k_dstep_stream.  K <= 256; d is updated in place.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_dstep_refine(const float* __restrict__ Hm, const float* __restrict__ Cm,
                                                      int fs, int K, int Pf, double rho_d,
                                                      const float2* __restrict__ rhs, float2* __restrict__ d) {
  __shared__ __align__(16) float strip[DS_ROWS * DS_PITCH];
  __shared__ double2 xv[256], acc[256];
  const int p = blockIdx.x, t = threadIdx.x;
  const int ld = K + 1;
  const int rr = t >> 4, q = t & 15;
  float2 d0 = make_float2(0.f, 0.f);
  if (t < K) {
    d0 = d[(size_t)t * Pf + p];
    xv[t] = make_double2((double)d0.x, (double)d0.y);
  }
  // y = M x for the Hermitian M stored in the R-form at R (FP64 sums);
  // returns output t (t < K) to the thread that owns it
  auto matvec = [&](const float* __restrict__ R) -> double2 {
    v4f pf[DS_V];
    if (t < K) acc[t] = make_double2(0.0, 0.0);
    double2 dc = make_double2(0.0, 0.0);
    ds_fetch(pf, R, 0, min(DS_ROWS, K), ld, t);
    __syncthreads();
    for (int a0 = 0; a0 < K; a0 += DS_ROWS) {
      const int nr = min(DS_ROWS, K - a0);
      ds_stage(pf, strip, nr, ld, t);
      __syncthreads();
      if (a0 + DS_ROWS < K) ds_fetch(pf, R, a0 + DS_ROWS, min(DS_ROWS, K - a0 - DS_ROWS), ld, t);
      if (t < K) {   // column role: output t
        for (int r = 0; r < nr; ++r) {
          const int a = a0 + r;
          const double v = (double)strip[r * ld + t];
          const double2 xa = xv[a];
          if (a <= t) {
            dc.x = fma(v, xa.x, dc.x);
            dc.y = fma(v, xa.y, dc.y);
          } else {
            dc.x = fma(-v, xa.y, dc.x);
            dc.y = fma(v, xa.x, dc.y);
          }
        }
      }
      double2 sum = make_double2(0.0, 0.0);   // row role: output a0 + rr, columns q, q + 16, ...
      if (rr < nr) {
        const int a = a0 + rr;
        for (int b = q; b < K; b += 16) {
          if (b == a) continue;
          const double v = (double)strip[rr * ld + b];
          const double2 xb = xv[b];
          if (a < b) {
            sum.x = fma(v, xb.x, sum.x);
            sum.y = fma(v, xb.y, sum.y);
          } else {
            sum.x = fma(v, xb.y, sum.x);
            sum.y = fma(-v, xb.x, sum.y);
          }
        }
      }
#pragma unroll
      for (int off = 8; off > 0; off >>= 1) {
        sum.x += __shfl_xor(sum.x, off, 16);
        sum.y += __shfl_xor(sum.y, off, 16);
      }
      if (rr < nr && q == 0) {
        double2 s = acc[a0 + rr];
        s.x += sum.x;
        s.y += sum.y;
        acc[a0 + rr] = s;
      }
      __syncthreads();   // the strip is overwritten next
    }
    double2 y = make_double2(0.0, 0.0);
    if (t < K) y = make_double2(dc.x + acc[t].x, dc.y + acc[t].y);
    __syncthreads();   // acc and xv are reused by the caller
    return y;
  };
  // r = rhs - H d - rho_d d
  const double2 hd = matvec(Hm + (size_t)p * fs);
  if (t < K) {
    const float2 b = rhs[(size_t)t * Pf + p];
    xv[t] = make_double2((double)b.x - hd.x - rho_d * (double)d0.x, (double)b.y - hd.y - rho_d * (double)d0.y);
  }
  __syncthreads();
  // d += C r
  const double2 cr = matvec(Cm + (size_t)p * fs);
  if (t < K)
    d[(size_t)t * Pf + p] = make_float2((float)((double)d0.x + cr.x), (float)((double)d0.y + cr.y));
}

}  // namespace ocsc
