// common.hpp -- helpers shared by the gfx950 kernels of the OCSC hot path.
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

typedef float v4f __attribute__((ext_vector_type(4)));

}  // namespace ocsc
