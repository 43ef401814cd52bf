// Stencil launches for one radius (compiled once per radius with -DALOFDFT_RADIUS=n).
#include <type_traits>

#include "launch.h"

#ifndef ALOFDFT_RADIUS
#error "compile with -DALOFDFT_RADIUS=n"
#endif

namespace alofdft {

// Launch shapes.  Large grids: one contiguous z slab per XCD -- the chunk count is a
// multiple of 8 and the XCD swizzle of the kernel hands XCD x the chunks
// [x k, (x+1) k), so the x-y tiles of a slab and their halos meet in that XCD's L2;
// more chunks per XCD (k > 1) only while the launch is below the target workgroup
// count and chunks stay at least 4 planes long.  Small grids (fewer tiles x planes
// than the target) are latency bound: chunks of 2 planes for the most workgroups.
template <typename T, int R, int BX, int BY, int VY, bool DEEP, class Op>
static hipError_t launch_cfg(const LaunchCfg& lc, const Geom& g, const StencilW<T>& W, const Op& op, int* nblocks) {
  const int tiles_x = (g.nx + BX - 1) / BX;
  const int tiles_y = (g.ny + BY * VY - 1) / (BY * VY);
  const int tiles = tiles_x * tiles_y;
  int nchunks;
  if ((long long)tiles * g.nz <= lc.target_blocks) {
    nchunks = (g.nz + 1) / 2;
  } else {
    const int kmax = std::max(1, g.nz / (8 * 4));
    const int k = std::max(1, std::min(kmax, (lc.target_blocks + 8 * tiles - 1) / (8 * tiles)));
    nchunks = std::min(8 * k, g.nz);
  }
  const int zc = (g.nz + nchunks - 1) / nchunks;
  nchunks = (g.nz + zc - 1) / zc;
  const int nb = tiles * nchunks;
  hipLaunchKernelGGL((k_stencil<T, R, BX, BY, VY, DEEP, Op>), dim3(nb), dim3(BX * BY), 0, lc.stream, g, W, zc,
                     tiles_x, tiles_y, op);
  *nblocks = nb;
  return hipGetLastError();
}

template <int R, typename T, class Op>
hipError_t launch_stencil_r(const LaunchCfg& lc, const Geom& g, const StencilW<T>& W, const Op& op, int* nblocks) {
  // the residual pass carries the XC arithmetic: one node per thread keeps it in registers
  if constexpr (std::is_same_v<Op, GradOp>) {
    return launch_cfg<T, R, 64, 4, 1, false, Op>(lc, g, W, op, nblocks);
  } else {
    // automatic shape: small grids 64x4 with deep prefetch, large grids 64x8, two rows per thread
    if (lc.variant < 0) {
      const long long tiles = (long long)((g.nx + 63) / 64) * ((g.ny + 7) / 8);
      if (tiles * g.nz <= lc.target_blocks) return launch_cfg<T, R, 64, 4, 1, true, Op>(lc, g, W, op, nblocks);
      return launch_cfg<T, R, 64, 4, 2, false, Op>(lc, g, W, op, nblocks);
    }
    if constexpr (R == 6) {
      switch (lc.variant) {
        case 1: return launch_cfg<T, R, 64, 4, 1, true, Op>(lc, g, W, op, nblocks);
        case 2: return launch_cfg<T, R, 64, 8, 1, false, Op>(lc, g, W, op, nblocks);
        case 3: return launch_cfg<T, R, 64, 8, 1, true, Op>(lc, g, W, op, nblocks);
        case 4: return launch_cfg<T, R, 64, 4, 1, false, Op>(lc, g, W, op, nblocks);
        default: break;
      }
    }
    return launch_cfg<T, R, 64, 4, 2, false, Op>(lc, g, W, op, nblocks);
  }
}

#define ALOFDFT_INST(T, OP)                                                                                     \
  template hipError_t launch_stencil_r<ALOFDFT_RADIUS, T, OP>(const LaunchCfg&, const Geom&, const StencilW<T>&, \
                                                               const OP&, int*);
ALOFDFT_INST(double, LapOp<double>)
ALOFDFT_INST(float, LapOp<float>)
ALOFDFT_INST(double, CGInitOp<double>)
ALOFDFT_INST(float, CGInitOp<float>)
ALOFDFT_INST(double, CGP1Op<double>)
ALOFDFT_INST(float, CGP1Op<float>)
ALOFDFT_INST(double, GradOp)
#undef ALOFDFT_INST

}  // namespace alofdft
