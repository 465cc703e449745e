// group.hpp -- one persistent launch that runs every code-ADMM iteration
// (eq. fcsc_code) of sample batches on several grids of different sizes.
//
// The launch is cooperative: a fixed grid of workgroups, all resident, walks
// each phase's work items (grouped by grid, i.e. by FFT size) with a
// grid-stride loop and meets at a grid-wide barrier between phases.  Per
// iteration:
//   Z      Z-steps of every grid (frequency blocks x groups of CG_ZS samples);
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
constexpr int CG_ZS = 4;              // Z-step samples per item

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

// Work items per phase of one grid (host and device agree on these).
template <typename T>
__host__ __device__ inline int cg_col_blocks(int pw) {
  return (pw / 2 + 1 + big_cb<T>() - 1) / big_cb<T>();
}

// Each phase's items are dealt out grid-stride over the workgroups (item it
// to workgroup it mod gridDim.x).  A workgroup runs its items grid by grid:
// local items i0, i0 + step, ... below n of grid s.  The small items (Z-step
// blocks, column and row blocks of two-pass grids) run in one call of a
// non-inlined body loop per grid, instead of one call (a call frame saved and
// restored) per item; a one-pass plane step is one call per item, since the
// loop around it spilled inside the transforms.
template <typename T, int PH, int PW>
__device__ __attribute__((noinline)) void cg_plane1(unsigned char* smem, const CodeGroupArgs<T>& g, int s,
                                                    int local, int first, int last) {
  cx<T>* buf = reinterpret_cast<cx<T>*>(smem);
  cx<T>* sH = buf + PH * PlaneGeom<PH, PW>::LDW;
  code_plane_body<T, PH, PW, CG_NT>(buf, sH, sH + PH, local, g.Zh[s], g.W[s], g.S[s], g.U[s], g.twH[s], g.twW[s],
                                    g.kappa[s], first, last);
}

// inverse column pass of two-pass grids: column block x plane
template <typename T, int PH, int PW>
__device__ __attribute__((noinline)) void cg_cols_inv(unsigned char* smem, const CodeGroupArgs<T>& g, int s, int i0,
                                                      int n, int step) {
  cx<T>* buf = reinterpret_cast<cx<T>*>(smem);
  const int ncb = cg_col_blocks<T>(PW);
  for (int local = i0; local < n; local += step) {
    big_cols_body<T, PH, PW, true, big_cb<T>(), CG_NT>(buf, buf + PH * big_cb<T>(), local % ncb, local / ncb,
                                                       g.Zh[s], g.Yb[s], g.twH[s]);
    __syncthreads();
  }
}

// P phase of grid s: plane steps (one-pass grids) or inverse column passes
template <typename T, int PH, int PW>
__device__ __forceinline__ void cg_plane(unsigned char* smem, const CodeGroupArgs<T>& g, int s, int i0, int n,
                                         int step, int first, int last) {
  if constexpr (PH > 128 || PW > 128) {
    cg_cols_inv<T, PH, PW>(smem, g, s, i0, n, step);
  } else {
    for (int local = i0; local < n; local += step) {
      cg_plane1<T, PH, PW>(smem, g, s, local, first, last);
      __syncthreads();
    }
  }
}

template <typename T, int PH, int PW>
__device__ __attribute__((noinline)) void cg_rows(unsigned char* smem, const CodeGroupArgs<T>& g, int s, int i0,
                                                  int n, int step, int first, int last) {
  if constexpr (PH > 128 || PW > 128) {
    cx<T>* buf = reinterpret_cast<cx<T>*>(smem);
    constexpr int NRB = PH / BIG_RB;
    for (int local = i0; local < n; local += step) {
      big_code_rows_body<T, PH, PW, BIG_RB, CG_NT>(buf, buf + BIG_RB * (PW / 2 + 1), local % NRB, local / NRB,
                                                   g.Yb[s], g.W[s], g.S[s], g.U[s], g.twW[s], g.kappa[s], first,
                                                   last);
      __syncthreads();
    }
  }
}

template <typename T, int PH, int PW>
__device__ __attribute__((noinline)) void cg_cols_fwd(unsigned char* smem, const CodeGroupArgs<T>& g, int s, int i0,
                                                      int n, int step) {
  if constexpr (PH > 128 || PW > 128) {
    cx<T>* buf = reinterpret_cast<cx<T>*>(smem);
    const int ncb = cg_col_blocks<T>(PW);
    for (int local = i0; local < n; local += step) {
      big_cols_body<T, PH, PW, false, big_cb<T>(), CG_NT>(buf, buf + PH * big_cb<T>(), local % ncb, local / ncb,
                                                          g.S[s], g.S[s], g.twH[s]);
      __syncthreads();
    }
  }
}

#define OCSC_GROUP_SIZES(X)                                                                                  \
  X(32, 32) X(32, 64) X(32, 128) X(64, 32) X(64, 64) X(64, 128) X(128, 32) X(128, 64) X(128, 128) X(256, 256) \
  X(256, 512) X(512, 256) X(512, 512)

// Z-step items: a block of CG_ZF frequencies for CG_ZS samples, so that the
// dictionary spectrum is read once per CG_ZS samples
template <typename T, int KPT>
__device__ __attribute__((noinline)) void cg_zstep(unsigned char* smem, const CodeGroupArgs<T>& g, int s, int i0,
                                                   int n, int step, int first, int last) {
  const int nzb = (g.Pf[s] + CG_ZF - 1) / CG_ZF;
  for (int local = i0; local < n; local += step) {
    zstep_body<T, KPT, CG_ZF, CG_ZS>(reinterpret_cast<cx<T>(*)[CG_ZF + 1]>(smem), local % nzb, local / nzb,
                                     g.Dh[s], g.gam[s], g.xh[s], g.S[s], g.Zh[s], g.K[s], g.Pf[s], g.B[s], first,
                                     last ? g.Zt[s] : nullptr, g.ldt[s], 0);
    __syncthreads();
  }
}

// The first item of grid s's range [first[s], first[s + 1]) that falls to
// this workgroup, as a local index (>= the range's length if none does).
__device__ __forceinline__ int cg_first_local(const int* first, int s) {
  const int lo = first[s], G = (int)gridDim.x;
  return ((int)blockIdx.x - lo % G + G) % G;
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
  const int G = (int)gridDim.x;
  for (int j = 0; j < g.Jz; ++j) {
    const int first = j == 0, last = j == g.Jz - 1;
    // Z: every grid's Z-step
    for (int s = 0; s < g.n; ++s)
      cg_zstep<T, KPT>(cg_smem, g, s, cg_first_local(g.z0, s), g.z0[s + 1] - g.z0[s], G, first, last);
    grid.sync();
    // P: plane steps / inverse column passes
    for (int s = 0; s < g.n; ++s) {
      const int i0 = cg_first_local(g.p0, s), n = g.p0[s + 1] - g.p0[s];
      switch (g.ph[s] * 1000 + g.pw[s]) {
#define X(A, B)                                                 \
  case A * 1000 + B:                                            \
    cg_plane<T, A, B>(cg_smem, g, s, i0, n, G, first, last);    \
    break;
        OCSC_GROUP_SIZES(X)
#undef X
        default:
          break;
      }
    }
    grid.sync();
    if (g.any_big) {
      // R: row passes of the two-pass grids
      for (int s = 0; s < g.n; ++s) {
        const int i0 = cg_first_local(g.r0, s), n = g.r0[s + 1] - g.r0[s];
        switch (g.ph[s] * 1000 + g.pw[s]) {
#define X(A, B)                                              \
  case A * 1000 + B:                                         \
    cg_rows<T, A, B>(cg_smem, g, s, i0, n, G, first, last);  \
    break;
          OCSC_GROUP_SIZES(X)
#undef X
          default:
            break;
        }
      }
      grid.sync();
      if (!last) {
        // F: forward column passes of the two-pass grids
        for (int s = 0; s < g.n; ++s) {
          const int i0 = cg_first_local(g.f0, s), n = g.f0[s + 1] - g.f0[s];
          switch (g.ph[s] * 1000 + g.pw[s]) {
#define X(A, B)                                        \
  case A * 1000 + B:                                   \
    cg_cols_fwd<T, A, B>(cg_smem, g, s, i0, n, G);     \
    break;
            OCSC_GROUP_SIZES(X)
#undef X
            default:
              break;
          }
        }
        grid.sync();
      }
    }
  }
}

}  // namespace ocsc
