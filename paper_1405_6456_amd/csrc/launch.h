// Launch of the stencil kernel for a given radius; the instantiations for each
// radius are compiled in their own translation unit (stencil_inst.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.h"

namespace alofdft {

struct LaunchCfg {
  hipStream_t stream;
  int variant;        // tile shape (order 12 only; other orders use variant 0)
  int target_blocks;  // workgroups per launch to aim for (sets the z chunk length)
};

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
