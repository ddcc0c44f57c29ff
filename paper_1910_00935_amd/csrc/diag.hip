// Measurement support (not part of the method): the cost of adding
// overlapping workgroup boxes of grid nodes into a global grid with different
// lane layouts, the pattern of the step kernels' scatter-tile flush
// (include/mpm.h, mpm_diag_box_atomics).

#include <hip/hip_runtime.h>

#include "mpm.h"

namespace {

// 128 workgroups, each a 7 x 7 x 5 box of nodes (a 4 x 4 x 2 block of cells
// and its quadratic stencil), blocks tiling a 16 x 16 x 16 cell region from
// cell 16 on, so neighbouring boxes overlap by three nodes along each axis as
// the boxes of the 3D lattice workload do. Node index z fastest.
constexpr int kBX = 7, kBY = 7, kBZ = 5, kNB = kBX * kBY * kBZ, kWG = 128;

__device__ __forceinline__ long box_node(int w, int q, int n) {
  const int bx = w & 3, by = (w >> 2) & 3, bz = w >> 4;
  const int x = 15 + 4 * bx + q / (kBZ * kBY), y = 15 + 4 * by + (q / kBZ) % kBY, z = 15 + 2 * bz + q % kBZ;
  return (long(x) * n + y) * n + z;
}

// layout 0: one node per lane, one atomic instruction per component;
// 1: lanes over (node, component), component fastest; 2: as 1 with plain
// stores; 3: no memory operation.
template <int L>
__global__ void __launch_bounds__(256) k_box_atomics(float* g, int n) {
  const int w = blockIdx.x;
  if (L == 0) {
    for (int q = threadIdx.x; q < kNB; q += blockDim.x) {
      float* dst = g + 4 * box_node(w, q, n);
#pragma unroll
      for (int c = 0; c < 4; ++c) unsafeAtomicAdd(dst + c, 1.0f);
    }
  } else if (L == 1 || L == 2) {
    for (int j = threadIdx.x; j < 4 * kNB; j += blockDim.x) {
      float* dst = g + 4 * box_node(w, j >> 2, n) + (j & 3);
      if (L == 1)
        unsafeAtomicAdd(dst, 1.0f);
      else
        *dst = 1.0f;
    }
  }
}

}  // namespace

extern "C" {

mpm_status mpm_diag_box_atomics(int32_t layout, float* grid, int32_t n, int32_t launches, void* stream) {
  // The boxes reach node 15 + 12 + 6 = 33 along x and y, 15 + 14 + 4 = 33 along z.
  if (!grid || n < 34 || n > 1024 || launches < 0 || layout < 0 || layout > 3) return MPM_E_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  for (int i = 0; i < launches; ++i) {
    switch (layout) {
      case 0: hipLaunchKernelGGL(k_box_atomics<0>, dim3(kWG), dim3(256), 0, s, grid, n); break;
      case 1: hipLaunchKernelGGL(k_box_atomics<1>, dim3(kWG), dim3(256), 0, s, grid, n); break;
      case 2: hipLaunchKernelGGL(k_box_atomics<2>, dim3(kWG), dim3(256), 0, s, grid, n); break;
      default: hipLaunchKernelGGL(k_box_atomics<3>, dim3(kWG), dim3(256), 0, s, grid, n); break;
    }
    if (hipGetLastError() != hipSuccess) return MPM_E_HIP;
  }
  return MPM_OK;
}

}  // extern "C"
