// Launch of the stencil kernel for a given radius; the instantiations for each
// radius are compiled in their own translation unit (stencil_inst.hip).
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.h"

namespace alofdft {

struct LaunchCfg {
  hipStream_t stream;
  int variant;        // tile shape (order 12 only; other orders use variant 0)
  int target_blocks;  // workgroups per launch to aim for (sets the z chunk length); 0: one round
  hipEvent_t ev_start = nullptr;  // optional: set to the start and end of the kernel itself
  hipEvent_t ev_stop = nullptr;
};

// Kernel launch on lc.stream; with events set, the runtime stamps them with the
// kernel's own start and end (not the surrounding queue packets).
template <typename K, typename... A>
inline hipError_t launch_kernel(const LaunchCfg& lc, K kernel, dim3 grid, dim3 block, A... args) {
  if (lc.ev_start)
    hipExtLaunchKernelGGL(kernel, grid, block, 0, lc.stream, lc.ev_start, lc.ev_stop, 0, args...);
  else
    hipLaunchKernelGGL(kernel, grid, block, 0, lc.stream, args...);
  return hipGetLastError();
}

// Largest number of workgroups any stencil launch can use on geometry g (sizes the
// block-partial buffers).
inline int max_stencil_blocks(const Geom& g, int target) {
  // a launch uses tiles * chunks <= target + 8 * tiles workgroups, with tiles no
  // more than this count of 32 x 4 tiles; target 0 (one round of resident
  // workgroups) stays below 8192 on any part with up to 512 compute units
  const int tiles = ((g.nx + 31) / 32) * ((g.ny + 3) / 4);
  return (target > 0 ? target : 8192) + 8 * tiles + 64;
}

template <int R, typename T, class Op>
hipError_t launch_stencil_r(const LaunchCfg& lc, const Geom& g, const StencilW<T>& W, const Op& op, int* nblocks);

}  // namespace alofdft
