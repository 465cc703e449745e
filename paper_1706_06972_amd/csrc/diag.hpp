// diag.hpp -- kept history, online surrogate and diagnostics (gfx950).
//
// None of these kernels is on the per-sample path unless the learner keeps
// its history (H, the sums of ||x_i||^2 and ||U_i||_1); all reductions are
// accumulated in double, in a fixed order (partials per block, then one
// workgroup), so repeated runs give identical bits.
#pragma once
#include "kernels.hpp"

namespace ocsc {

constexpr int DIAG_BLOCKS = 256;   // partial sums of the grid-stride reductions

__device__ __forceinline__ double block_sum256(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

// Parseval weight of stored frequency p of the half spectrum: the columns
// v = 0 and v = PW/2 are their own mirror images, every other column stands
// for itself and its conjugate.
__device__ __forceinline__ double parseval_w(int p, int PW) {
  const int WC = PW / 2 + 1;
  const int v = p % WC;
  return (v == 0 || 2 * v == PW) ? 1.0 : 2.0;
}

// History (Proposition 1, unnormalised): H_p += sum_b conj(z_bp) z_bp^T for
// every frequency, stored like C (R-form, rows of pitch K + 1, stride fs).
// One workgroup per frequency; samples are taken in chunks of HB.
template <typename T>
__global__ __launch_bounds__(256) void k_hist_herk(T* __restrict__ Hm, const cx<T>* __restrict__ Zh, int B, int K,
                                                   int Pf, int fs) {
  constexpr int HB = 8;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* zs = reinterpret_cast<cx<T>*>(smem_raw);   // [HB][K]
  const int p = blockIdx.x;
  const int ld = K + 1;
  T* R = Hm + (size_t)p * fs;
  for (int b0 = 0; b0 < B; b0 += HB) {
    const int nb = min(HB, B - b0);
    __syncthreads();
    for (int i = threadIdx.x; i < nb * K; i += blockDim.x) {
      const int b = i / K, k = i % K;
      zs[i] = Zh[((size_t)(b0 + b) * K + k) * Pf + p];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < K * ld; e += blockDim.x) {
      const int r = e / ld, c = e % ld;
      if (c >= K) continue;
      T acc = R[e];
      for (int b = 0; b < nb; ++b) {
        // H_ij = conj(z_i) z_j; (r, c) holds Re H_rc for c >= r and Im H_cr for c < r
        const cx<T> zi = zs[b * K + (c >= r ? r : c)];
        const cx<T> zj = zs[b * K + (c >= r ? c : r)];
        acc += c >= r ? zi.x * zj.x + zi.y * zj.y : zi.x * zj.y - zi.y * zj.x;
      }
      R[e] = acc;
    }
  }
}

// Partial sums over n = planes * Pf spectrum entries of the Parseval-weighted
// squared modulus of A - Bsp (Bsp may be null).  gridDim.y selects a group of
// `planes` planes (a sample), part[y * gridDim.x + x].
template <typename T>
__global__ __launch_bounds__(256) void k_wsq(const cx<T>* __restrict__ A, const cx<T>* __restrict__ Bsp,
                                             double* __restrict__ part, int planes, int Pf, int PW) {
  __shared__ double red[256];
  const size_t n = (size_t)planes * Pf;
  const size_t off = (size_t)blockIdx.y * n;
  double acc = 0;
  for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (size_t)gridDim.x * 256) {
    cx<T> a = A[off + e];
    if (Bsp) a = csub<T>(a, Bsp[off + e]);
    acc += parseval_w((int)(e % Pf), PW) * ((double)a.x * a.x + (double)a.y * a.y);
  }
  const double s = block_sum256(acc, red);
  if (threadIdx.x == 0) part[(size_t)blockIdx.y * gridDim.x + blockIdx.x] = s;
}

// Euclidean norm of each of gridDim.x real planes of n entries.
template <typename T>
__global__ __launch_bounds__(256) void k_plane_norm(const T* __restrict__ X, int n, double* __restrict__ out) {
  __shared__ double red[256];
  const T* x = X + (size_t)blockIdx.x * n;
  double acc = 0;
  for (int i = threadIdx.x; i < n; i += 256) acc += (double)x[i] * (double)x[i];
  const double s = block_sum256(acc, red);
  if (threadIdx.x == 0) out[blockIdx.x] = sqrt(s);
}

// out[slot] = sqrt?(scale * sum(part[0..n))), one workgroup.
__global__ __launch_bounds__(256) void k_sum_parts(const double* __restrict__ part, int n, double* __restrict__ out,
                                                   double scale, int take_sqrt) {
  __shared__ double red[256];
  double acc = 0;
  for (int i = threadIdx.x; i < n; i += 256) acc += part[i];
  const double s = scale * block_sum256(acc, red);
  if (threadIdx.x == 0) out[0] = take_sqrt ? sqrt(s) : s;
}

// Running sums of the history: acc[0] += sum(xpart) * invP (= sum_b ||x_b||^2
// by Parseval), acc[1] += sum(upart) (= sum_b ||U_b||_1).
__global__ __launch_bounds__(256) void k_hist_sums(const double* __restrict__ xpart, int nx,
                                                   const double* __restrict__ upart, int nu,
                                                   double* __restrict__ acc, double invP) {
  __shared__ double red[256];
  double a = 0, b = 0;
  for (int i = threadIdx.x; i < nx; i += 256) a += xpart[i];
  for (int i = threadIdx.x; i < nu; i += 256) b += upart[i];
  a = block_sum256(a, red);
  b = block_sum256(b, red);
  if (threadIdx.x == 0) {
    acc[0] += a * invP;
    acc[1] += b;
  }
}

// Surrogate, per frequency p (one workgroup each):
//   part[p] = c_p (d^H H_p d - 2 Re d^H G_p),  d = Dsp[:, p],
// with H_p in R-form; products and sums in double.
template <typename T>
__global__ __launch_bounds__(256) void k_surr_quad(const T* __restrict__ Hm, const cx<T>* __restrict__ G,
                                                   const cx<T>* __restrict__ Dsp, double* __restrict__ part,
                                                   int K, int Pf, int PW, int fs) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* dr = reinterpret_cast<double*>(smem_raw);   // [K] real parts
  double* di = dr + K;                                // [K] imaginary parts
  __shared__ double red[256];
  const int p = blockIdx.x;
  const int ld = K + 1;
  const T* R = Hm + (size_t)p * fs;
  double acc = 0;
  for (int k = threadIdx.x; k < K; k += 256) {
    const cx<T> d = Dsp[(size_t)k * Pf + p];
    const cx<T> g = G[(size_t)k * Pf + p];
    dr[k] = d.x;
    di[k] = d.y;
    acc -= 2.0 * ((double)d.x * g.x + (double)d.y * g.y);
  }
  __syncthreads();
  for (int e = threadIdx.x; e < K * ld; e += 256) {
    const int r = e / ld, c = e % ld;
    if (c >= K) continue;
    const double h = (double)R[e];
    if (c == r) {
      acc += h * (dr[r] * dr[r] + di[r] * di[r]);
    } else if (c > r) {   // Re H_rc: 2 Re H_rc Re(conj(d_r) d_c)
      acc += 2.0 * h * (dr[r] * dr[c] + di[r] * di[c]);
    } else {              // Im H_cr: -2 Im H_cr Im(conj(d_c) d_r)
      acc -= 2.0 * h * (dr[c] * di[r] - di[c] * dr[r]);
    }
  }
  const double s = block_sum256(acc, red);
  if (threadIdx.x == 0) part[p] = parseval_w(p, PW) * s;
}

// F_t = sum(part) / (2P) + acc[0] / 2 + lam * acc[1], one workgroup.
__global__ __launch_bounds__(256) void k_surr_final(const double* __restrict__ part, int n,
                                                    const double* __restrict__ acc, double* __restrict__ out,
                                                    double invP, double lam) {
  __shared__ double red[256];
  double a = 0;
  for (int i = threadIdx.x; i < n; i += 256) a += part[i];
  a = block_sum256(a, red);
  if (threadIdx.x == 0) out[0] = 0.5 * a * invP + 0.5 * acc[0] + lam * acc[1];
}

}  // namespace ocsc
