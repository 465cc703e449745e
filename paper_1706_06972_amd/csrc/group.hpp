// group.hpp -- one persistent launch that runs every code-ADMM iteration
// (eq. fcsc_code) of sample batches on several grids of different sizes.
//
// The launch is cooperative: a fixed grid of workgroups, all resident, walks
// each phase's work items (grouped by grid, i.e. by FFT size) with a
// grid-stride loop and meets at a grid-wide barrier between phases.  Per
// iteration:
//   Z      Z-steps of every grid (frequency blocks x samples);
//   P      one-pass grids: the fused plane step; two-pass grids: the inverse
//          column pass (column blocks x planes);
//   R      two-pass grids: the row pass (U-step, dual, forward rows);
//   F      two-pass grids: the forward column pass (not on the last iteration).
// Each item runs the same device body as the separate kernels, so the values
// are those of per-grid launches bit for bit.  Every workgroup executes every
// barrier: the item loops depend on blockIdx only and the barriers sit
// outside them.
#pragma once
#include <hip/hip_cooperative_groups.h>

#include "bigplane.hpp"
#include "kernels.hpp"

namespace ocsc {

constexpr int CG_MAX = 8;             // grids per launch
constexpr int CG_NT = 512;            // threads per workgroup (every phase)
constexpr int CG_ZF = CG_NT / 16;     // Z-step frequencies per item

template <typename T>
struct CodeGroupArgs {
  int n, Jz, any_big;
  int ph[CG_MAX], pw[CG_MAX], K[CG_MAX], B[CG_MAX], Pf[CG_MAX], big[CG_MAX], ldt[CG_MAX];
  const cx<T>* Dh[CG_MAX];
  const T* gam[CG_MAX];
  const cx<T>* xh[CG_MAX];
  cx<T>* S[CG_MAX];
  cx<T>* Zh[CG_MAX];
  T* W[CG_MAX];
  cx<T>* Yb[CG_MAX];
  T* U[CG_MAX];
  cx<T>* Zt[CG_MAX];   // frequency-major copy of the last iterate, or null
  const cx<T>* twH[CG_MAX];
  const cx<T>* twW[CG_MAX];
  T kappa[CG_MAX];
  // first item of each grid in each phase; entry n is the phase's total
  int z0[CG_MAX + 1], p0[CG_MAX + 1], r0[CG_MAX + 1], f0[CG_MAX + 1];
};

__device__ __forceinline__ int cg_grid_of(const int* first, int n, int item) {
  int s = 0;
  while (s + 1 < n && item >= first[s + 1]) ++s;
  return s;
}

// Work items per phase of one grid (host and device agree on these).
template <typename T>
__host__ __device__ inline int cg_col_blocks(int pw) {
  return (pw / 2 + 1 + big_cb<T>() - 1) / big_cb<T>();
}

template <typename T, int PH, int PW>
__device__ __attribute__((noinline)) void cg_plane(unsigned char* smem, const CodeGroupArgs<T>& g, int s, int local, int first,
                                         int last) {
  if constexpr (PH > 128 || PW > 128) {
    // inverse column pass of two-pass grids: column block x plane
    cx<T>* buf = reinterpret_cast<cx<T>*>(smem);
    const int ncb = cg_col_blocks<T>(PW);
    big_cols_body<T, PH, PW, true, big_cb<T>(), CG_NT>(buf, buf + PH * big_cb<T>(), local % ncb, local / ncb,
                                                       g.Zh[s], g.Yb[s], g.twH[s]);
  } else {
    cx<T>* buf = reinterpret_cast<cx<T>*>(smem);
    cx<T>* sH = buf + PH * PlaneGeom<PH, PW>::LDW;
    code_plane_body<T, PH, PW, CG_NT>(buf, sH, sH + PH, local, g.Zh[s], g.W[s], g.S[s], g.U[s], g.twH[s],
                                      g.twW[s], g.kappa[s], first, last);
  }
}

template <typename T, int PH, int PW>
__device__ __attribute__((noinline)) void cg_rows(unsigned char* smem, const CodeGroupArgs<T>& g, int s, int local, int first,
                                        int last) {
  if constexpr (PH > 128 || PW > 128) {
    cx<T>* buf = reinterpret_cast<cx<T>*>(smem);
    constexpr int NRB = PH / BIG_RB;
    big_code_rows_body<T, PH, PW, BIG_RB, CG_NT>(buf, buf + BIG_RB * (PW / 2 + 1), local % NRB, local / NRB,
                                                 g.Yb[s], g.W[s], g.S[s], g.U[s], g.twW[s], g.kappa[s], first,
                                                 last);
  }
}

template <typename T, int PH, int PW>
__device__ __attribute__((noinline)) void cg_cols_fwd(unsigned char* smem, const CodeGroupArgs<T>& g, int s, int local) {
  if constexpr (PH > 128 || PW > 128) {
    cx<T>* buf = reinterpret_cast<cx<T>*>(smem);
    const int ncb = cg_col_blocks<T>(PW);
    big_cols_body<T, PH, PW, false, big_cb<T>(), CG_NT>(buf, buf + PH * big_cb<T>(), local % ncb, local / ncb,
                                                        g.S[s], g.S[s], g.twH[s]);
  }
}

#define OCSC_GROUP_SIZES(X)                                                                                  \
  X(32, 32) X(32, 64) X(32, 128) X(64, 32) X(64, 64) X(64, 128) X(128, 32) X(128, 64) X(128, 128) X(256, 256) \
  X(256, 512) X(512, 256) X(512, 512)

template <typename T, int KPT>
__device__ __attribute__((noinline)) void cg_zstep(unsigned char* smem, const CodeGroupArgs<T>& g, int s, int local,
                                                   int first, int last) {
  const int nzb = (g.Pf[s] + CG_ZF - 1) / CG_ZF;
  zstep_body<T, KPT, CG_ZF, 1>(reinterpret_cast<cx<T>(*)[CG_ZF + 1]>(smem), local % nzb, local / nzb, g.Dh[s],
                               g.gam[s], g.xh[s], g.S[s], g.Zh[s], g.K[s], g.Pf[s], g.B[s], first,
                               last ? g.Zt[s] : nullptr, g.ldt[s], 0);
}

// At most 128 registers per lane (four waves per SIMD), so that two
// workgroups share a CU when the largest plane's LDS allows it.
// The arguments are copied once into LDS: indexed by a grid number only known
// at run time, the by-value parameter would otherwise be copied into every
// lane's private memory (1.2-1.9 KB of scratch per lane).
template <typename T, int KPT>
__global__ __launch_bounds__(CG_NT, 4) void k_code_group(CodeGroupArgs<T> ga) {
  extern __shared__ __align__(16) unsigned char cg_smem[];
  __shared__ CodeGroupArgs<T> g;
  if (threadIdx.x == 0) g = ga;
  __syncthreads();
  cooperative_groups::grid_group grid = cooperative_groups::this_grid();
  for (int j = 0; j < g.Jz; ++j) {
    const int first = j == 0, last = j == g.Jz - 1;
    // Z: every grid's Z-step
    for (int it = blockIdx.x; it < g.z0[g.n]; it += gridDim.x) {
      const int s = cg_grid_of(g.z0, g.n, it);
      cg_zstep<T, KPT>(cg_smem, g, s, it - g.z0[s], first, last);
      __syncthreads();
    }
    grid.sync();
    // P: plane steps / inverse column passes
    for (int it = blockIdx.x; it < g.p0[g.n]; it += gridDim.x) {
      const int s = cg_grid_of(g.p0, g.n, it), local = it - g.p0[s];
      switch (g.ph[s] * 1000 + g.pw[s]) {
#define X(A, B)                                                 \
  case A * 1000 + B:                                            \
    cg_plane<T, A, B>(cg_smem, g, s, local, first, last);       \
    break;
        OCSC_GROUP_SIZES(X)
#undef X
        default:
          break;
      }
      __syncthreads();
    }
    grid.sync();
    if (g.any_big) {
      // R: row passes of the two-pass grids
      for (int it = blockIdx.x; it < g.r0[g.n]; it += gridDim.x) {
        const int s = cg_grid_of(g.r0, g.n, it), local = it - g.r0[s];
        switch (g.ph[s] * 1000 + g.pw[s]) {
#define X(A, B)                                              \
  case A * 1000 + B:                                         \
    cg_rows<T, A, B>(cg_smem, g, s, local, first, last);     \
    break;
          OCSC_GROUP_SIZES(X)
#undef X
          default:
            break;
        }
        __syncthreads();
      }
      grid.sync();
      if (!last) {
        // F: forward column passes of the two-pass grids
        for (int it = blockIdx.x; it < g.f0[g.n]; it += gridDim.x) {
          const int s = cg_grid_of(g.f0, g.n, it), local = it - g.f0[s];
          switch (g.ph[s] * 1000 + g.pw[s]) {
#define X(A, B)                                        \
  case A * 1000 + B:                                   \
    cg_cols_fwd<T, A, B>(cg_smem, g, s, local);        \
    break;
            OCSC_GROUP_SIZES(X)
#undef X
            default:
              break;
          }
          __syncthreads();
        }
        grid.sync();
      }
    }
  }
}

}  // namespace ocsc
