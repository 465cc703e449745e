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
  __shared__ cx<T> buf[PH * G::LDW];
  __shared__ cx<T> sH[PH], sW[PW];
  const int tid = threadIdx.x;
  const long q = blockIdx.x;
  load_tables<PH, PW, T>(sH, sW, twH, twW, tid, NT);
  const T* s = src + q * sstride;
  for (int e = tid; e < PH * G::M; e += NT) {
    const int r = e / G::M, n = e % G::M, c = 2 * n;
    T a = 0, b = 0;
    if (r < sh) {
      if (c < sw) a = s[r * sw + c];
      if (c + 1 < sw) b = s[r * sw + c + 1];
    }
    buf[r * G::LDW + n] = mk<T>(a, b);
  }
  __syncthreads();
  rfft2_lds<PH, PW, NT, T>(buf, sH, sW, tid);
  cx<T>* d = dst + q * dstride;
  for (int e = tid; e < G::PF; e += NT) d[e] = buf[e];
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
  __shared__ cx<T> buf[PH * G::LDW];
  __shared__ cx<T> sH[PH], sW[PW];
  const int tid = threadIdx.x;
  const long q = blockIdx.x;
  load_tables<PH, PW, T>(sH, sW, twH, twW, tid, NT);
  const cx<T>* s = src + q * sstride;
  for (int e = tid; e < G::PF; e += NT) buf[e] = s[e];
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
  __shared__ cx<T> buf[PH * G::LDW];
  __shared__ cx<T> sH[PH], sW[PW];
  const int tid = threadIdx.x;
  const long q = blockIdx.x;
  load_tables<PH, PW, T>(sH, sW, twH, twW, tid, NT);
  const cx<T>* z = Zh + q * G::PF;
  for (int e = tid; e < G::PF; e += NT) buf[e] = z[e];
  __syncthreads();
  irfft2_lds<PH, PW, NT, T>(buf, sH, sW, tid);
  const T scale = (T)1 / (T)G::P;
  cx<T>* wp = reinterpret_cast<cx<T>*>(W + q * G::P);   // pixel pairs (2n, 2n+1)
  cx<T>* up = Uout ? reinterpret_cast<cx<T>*>(Uout + q * G::P) : nullptr;
  for (int e = tid; e < PH * G::M; e += NT) {
    const int r = e / G::M, n = e % G::M;
    const cx<T> y = buf[r * G::LDW + n];
    const cx<T> w = first ? mk<T>(0, 0) : wp[e];
    const T v0 = y.x * scale + w.x, v1 = y.y * scale + w.y;
    const T u0 = copysign(fmax(fabs(v0) - kappa, (T)0), v0);
    const T u1 = copysign(fmax(fabs(v1) - kappa, (T)0), v1);
    if (last) {
      if (up) up[e] = mk<T>(u0, u1);
    } else {
      const T w0 = v0 - u0, w1 = v1 - u1;
      wp[e] = mk<T>(w0, w1);
      buf[r * G::LDW + n] = mk<T>(u0 - w0, u1 - w1);
    }
  }
  if (last) return;
  __syncthreads();
  rfft2_lds<PH, PW, NT, T>(buf, sH, sW, tid);
  cx<T>* s = S + q * G::PF;
  for (int e = tid; e < G::PF; e += NT) s[e] = buf[e];
}

// ---------------------------------------------------------------------------
// Code update, frequency half of one ADMM iteration (the Z-step).  At each
// frequency p with a = Dh[:, p], s = S[:, p]:
//   z = s + conj(a) * gam_p * (x_p - a^T s),   gam_p = 1 / (rho + ||a||^2),
// which is the Sherman-Morrison solution of (conj(a) a^T + rho I) z =
// conj(a) x_p + rho s.  A workgroup of NW waves serves 64 frequencies of one
// sample; wave w holds filters k = w, w + NW, ... (at most KPW) in registers.
// first: s = 0.
// ---------------------------------------------------------------------------
template <typename T, int NW, int KPW>
__global__ __launch_bounds__(64 * NW) void k_code_zstep(const cx<T>* __restrict__ Dh,
                                                        const T* __restrict__ gam,
                                                        const cx<T>* __restrict__ xh,
                                                        const cx<T>* __restrict__ S,
                                                        cx<T>* __restrict__ Zh, int K, int Pf,
                                                        int first) {
  __shared__ cx<T> red[NW][64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int b = blockIdx.y;
  const int p = blockIdx.x * 64 + lane;
  const bool ok = p < Pf;
  cx<T> a[KPW], s[KPW];
  cx<T> acc = mk<T>(0, 0);
#pragma unroll
  for (int j = 0; j < KPW; ++j) {
    const int k = wv + j * NW;
    a[j] = mk<T>(0, 0);
    s[j] = mk<T>(0, 0);
    if (ok && k < K) {
      a[j] = Dh[(long)k * Pf + p];
      if (!first) s[j] = S[((long)b * K + k) * Pf + p];
      acc = cadd<T>(acc, cmul<T>(a[j], s[j]));
    }
  }
  red[wv][lane] = acc;
  __syncthreads();
  if (wv == 0) {
    cx<T> tot = red[0][lane];
#pragma unroll
    for (int i = 1; i < NW; ++i) tot = cadd<T>(tot, red[i][lane]);
    cx<T> qv = mk<T>(0, 0);
    if (ok) qv = cscale<T>(csub<T>(xh[(long)b * Pf + p], tot), gam[p]);
    red[0][lane] = qv;
  }
  __syncthreads();
  const cx<T> qv = red[0][lane];
#pragma unroll
  for (int j = 0; j < KPW; ++j) {
    const int k = wv + j * NW;
    if (ok && k < K) Zh[((long)b * K + k) * Pf + p] = cadd<T>(s[j], cmulc<T>(qv, a[j]));
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
// Per-frequency Hermitian algebra on the R-form of C held in LDS.
// ---------------------------------------------------------------------------
template <typename T>
struct HermLds {
  T* R;      // [K][K+1]
  int K, ld;
  __device__ __forceinline__ cx<T> elem(int i, int j) const {   // C_ij
    const int lo = i < j ? i : j, hi = i < j ? j : i;
    const T a = R[lo * ld + hi];
    const T braw = R[hi * ld + lo];
    const T b = j > i ? braw : (j < i ? -braw : (T)0);
    return mk<T>(a, b);
  }
};

// y = C x for one frequency, by the lt-th of tpg threads of its group.  Rows are
// split over up to 4 column chunks when the group has spare threads; partial
// sums go through part[4][K].
template <typename T>
__device__ __forceinline__ void herm_matvec(const HermLds<T>& C, const cx<T>* x, cx<T>* y, cx<T>* part,
                                            int lt, int tpg) {
  const int K = C.K;
  int ns = tpg / K;
  ns = ns < 1 ? 1 : (ns > 4 ? 4 : ns);
  const int chunk = (K + ns - 1) / ns;
  for (int task = lt; task < K * ns; task += tpg) {
    const int i = task % K, h = task / K;
    const int j0 = h * chunk, j1 = min(K, j0 + chunk);
    T ar = 0, ai = 0;
    for (int j = j0; j < j1; ++j) {
      const cx<T> c = C.elem(i, j);
      const cx<T> xv = x[j];
      ar += c.x * xv.x - c.y * xv.y;
      ai += c.x * xv.y + c.y * xv.x;
    }
    part[h * K + i] = mk<T>(ar, ai);
  }
  __syncthreads();
  for (int i = lt; i < K; i += tpg) {
    cx<T> s = part[i];
    for (int h = 1; h < ns; ++h) s = cadd<T>(s, part[h * K + i]);
    y[i] = s;
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// One D-step sweep over all frequencies (eq. sub_d_sol, column form):
//   d_p = C_p rhs_p,
// FPB frequencies per workgroup, C_p staged in LDS.  When nfold > 0 the
// history of nfold samples is folded first, in sample order (eqs. B_update
// and C_update):  u = conj(z_p);  G_p += u x_p;  v = C_p u;
// C_p <- C_p - v v^H / (1 + u^H v);  the updated C_p is written back and the
// right-hand side is the updated G_p (the first DictOCSC iterate, V = Theta = 0).
// With nfold = 0 and dout == nullptr the kernel only folds (stand-alone history
// update).  gam_out (optional): 1 / (rho + ||d_p||^2) for the next code update.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_dict_sweep(T* __restrict__ Cm, cx<T>* __restrict__ G,
                                                    const cx<T>* __restrict__ rhs,
                                                    const cx<T>* __restrict__ Zh,
                                                    const cx<T>* __restrict__ xh, int nfold,
                                                    cx<T>* __restrict__ dout, T* __restrict__ gam_out,
                                                    T rho, int K, int Pf, int fpb, int reverse) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int ld = K + 1;
  const int tpg = 256 / fpb;
  const int g = threadIdx.x / tpg, lt = threadIdx.x % tpg;
  // carve LDS: R blocks, then per-group vectors
  T* Rall = reinterpret_cast<T*>(smem_raw);
  const size_t rbytes = ((size_t)fpb * K * ld * sizeof(T) + 15) & ~(size_t)15;
  cx<T>* vecs = reinterpret_cast<cx<T>*>(smem_raw + rbytes);
  cx<T>* xv = vecs + (size_t)g * 7 * K;   // rhs / u
  cx<T>* yv = xv + K;                     // result
  cx<T>* vv = yv + K;                     // C u
  cx<T>* part = vv + K;                   // [4][K]
  __shared__ T sred[16];

  const int nb = (Pf + fpb - 1) / fpb;
  int fb = xcd_block(blockIdx.x, nb);
  if (reverse) fb = nb - 1 - fb;
  const int p = fb * fpb + g;
  const bool ok = p < Pf;
  HermLds<T> C{Rall + (size_t)g * K * ld, K, ld};
  const size_t kk = (size_t)K * K;

  // stage C_p into LDS
  if (ok) {
    const T* src = Cm + (size_t)p * kk;
    for (int e = lt; e < (int)kk; e += tpg) C.R[(e / K) * ld + (e % K)] = src[e];
  }
  __syncthreads();

  for (int b = 0; b < nfold; ++b) {
    if (ok) {
      const cx<T> xp = xh[(size_t)b * Pf + p];
      for (int k = lt; k < K; k += tpg) {
        const cx<T> z = Zh[((size_t)b * K + k) * Pf + p];
        const cx<T> u = cconj<T>(z);
        xv[k] = u;
        G[(size_t)k * Pf + p] = cadd<T>(G[(size_t)k * Pf + p], cmul<T>(u, xp));
      }
    }
    __syncthreads();
    herm_matvec<T>(C, xv, vv, part, lt, tpg);
    if (lt == 0) {
      T s = 0;
      for (int i = 0; i < K; ++i) s += xv[i].x * vv[i].x + xv[i].y * vv[i].y;   // Re(u^H v)
      sred[g] = (T)1 / ((T)1 + s);
    }
    __syncthreads();
    const T beta = sred[g];
    for (int e = lt; e < (int)kk; e += tpg) {
      const int i = e / K, j = e % K;
      const cx<T> vi = vv[i], vj = vv[j];
      if (j >= i) C.R[i * ld + j] -= beta * (vi.x * vj.x + vi.y * vj.y);   // Re(v_i conj v_j)
      else C.R[i * ld + j] -= beta * (vj.y * vi.x - vj.x * vi.y);          // Im(v_j conj v_i)
    }
    __syncthreads();
  }
  if (nfold > 0 && ok) {
    T* dst = Cm + (size_t)p * kk;
    for (int e = lt; e < (int)kk; e += tpg) dst[e] = C.R[(e / K) * ld + (e % K)];
  }
  if (!dout) return;

  // right-hand side
  const cx<T>* r = nfold > 0 ? G : rhs;
  if (ok)
    for (int k = lt; k < K; k += tpg) xv[k] = r[(size_t)k * Pf + p];
  __syncthreads();
  herm_matvec<T>(C, xv, yv, part, lt, tpg);
  if (ok)
    for (int k = lt; k < K; k += tpg) dout[(size_t)k * Pf + p] = yv[k];
  if (gam_out && lt == 0 && ok) {
    T s = 0;
    for (int i = 0; i < K; ++i) s += yv[i].x * yv[i].x + yv[i].y * yv[i].y;
    gam_out[p] = (T)1 / (rho + s);
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
constexpr int VB = 8;
constexpr int MAXF = 128;   // filter extent bound (filt <= pad <= 128)

template <typename T>
__global__ __launch_bounds__(256) void k_vstep_alpha(const cx<T>* __restrict__ d,
                                                     const cx<T>* __restrict__ Th, T* __restrict__ apart,
                                                     const cx<T>* __restrict__ twH,
                                                     const cx<T>* __restrict__ twW, int PH, int PW,
                                                     int Mh, int Mw, int first) {
  __shared__ cx<T> X[MAXF * VB];
  __shared__ cx<T> t[MAXF * VB];
  const int WC = PW / 2 + 1, Pf = PH * WC;
  const int vb = blockIdx.x, k = blockIdx.y, nvb = gridDim.x;
  const int v0 = vb * VB, nv = min(VB, WC - v0);
  const int tid = threadIdx.x;
  const cx<T>* dk = d + (size_t)k * Pf;
  const cx<T>* tk = Th + (size_t)k * Pf;
  for (int e = tid; e < PH * VB; e += 256) {
    const int u = e / VB, c = e % VB;
    cx<T> x = mk<T>(0, 0);
    if (c < nv) {
      x = dk[u * WC + v0 + c];
      if (!first) x = cadd<T>(x, tk[u * WC + v0 + c]);
    }
    X[e] = x;
  }
  __syncthreads();
  for (int e = tid; e < Mh * VB; e += 256) {
    const int m = e / VB, c = e % VB;
    T ar = 0, ai = 0;
    for (int u = 0; u < PH; ++u) {
      const cx<T> w = twH[(u * m) & (PH - 1)];   // e^{-2 pi i um/PH}; use its conjugate
      const cx<T> x = X[u * VB + c];
      ar += x.x * w.x + x.y * w.y;
      ai += x.y * w.x - x.x * w.y;
    }
    t[e] = mk<T>(ar, ai);
  }
  __syncthreads();
  const T invP = (T)1 / (T)(PH * PW);
  T* out = apart + ((size_t)k * nvb + vb) * Mh * Mw;
  for (int e = tid; e < Mh * Mw; e += 256) {
    const int m = e / Mw, n = e % Mw;
    T acc = 0;
    for (int c = 0; c < nv; ++c) {
      const int v = v0 + c;
      const T cv = (v == 0 || 2 * v == PW) ? (T)1 : (T)2;
      const cx<T> w = twW[(v * n) & (PW - 1)];
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
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* alpha = reinterpret_cast<T*>(smem_raw);                        // [Mh*Mw]
  cx<T>* rr = reinterpret_cast<cx<T>*>(smem_raw + (((size_t)Mh * Mw * sizeof(T) + 15) & ~(size_t)15));
  __shared__ T red[256];
  const int WC = PW / 2 + 1, Pf = PH * WC;
  const int vb = blockIdx.x, k = blockIdx.y, nvb = gridDim.x;
  const int v0 = vb * VB, nv = min(VB, WC - v0);
  const int tid = threadIdx.x;
  const int MM = Mh * Mw;
  const T* ap = apart + (size_t)k * nvb * MM;
  T ss = 0;
  for (int e = tid; e < MM; e += 256) {
    T a = 0;
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
        const cx<T> w = twW[(v * n) & (PW - 1)];
        const T x = alpha[m * Mw + n];
        ar += x * w.x;
        ai += x * w.y;
      }
    }
    rr[e] = mk<T>(ar, ai);
  }
  __syncthreads();
  const size_t base = (size_t)k * Pf;
  for (int e = tid; e < PH * VB; e += 256) {
    const int u = e / VB, c = e % VB;
    if (c >= nv) continue;
    T ar = 0, ai = 0;
    for (int m = 0; m < Mh; ++m) {
      const cx<T> w = twH[(u * m) & (PH - 1)];
      const cx<T> x = rr[m * VB + c];
      ar += x.x * w.x - x.y * w.y;
      ai += x.x * w.y + x.y * w.x;
    }
    const size_t idx = base + (size_t)u * WC + v0 + c;
    const cx<T> dv = d[idx];
    cx<T> th = first ? mk<T>(0, 0) : Th[idx];
    th = mk<T>(th.x + dv.x - ar, th.y + dv.y - ai);
    Th[idx] = th;
    const cx<T> gv = G[idx];
    rhs[idx] = mk<T>(gv.x + rho_d * (ar - th.x), gv.y + rho_d * (ai - th.y));
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
                            double* __restrict__ out, double invP, double lam) {
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
  if (threadIdx.x == 0) out[b] = 0.5 * a[0] * invP + lam * c[0];
}

// C_p = I / rho_d in R-form for every frequency.
template <typename T>
__global__ void k_c_init(T* __restrict__ Cm, int K, int Pf, T inv_rho_d) {
  const size_t kk = (size_t)K * K;
  const size_t n = kk * Pf;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
    const size_t r = e % kk;
    Cm[e] = (r / K == r % K) ? inv_rho_d : (T)0;
  }
}

template <typename T>
__global__ void k_fill_zero(T* __restrict__ x, size_t n) {
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) x[e] = (T)0;
}

}  // namespace ocsc
