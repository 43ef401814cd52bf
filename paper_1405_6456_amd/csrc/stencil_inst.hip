// Stencil launches for one radius (compiled once per radius with -DALOFDFT_RADIUS=n).
#include <atomic>
#include <type_traits>

#include "launch.h"

#ifndef ALOFDFT_RADIUS
#error "compile with -DALOFDFT_RADIUS=n"
#endif

namespace alofdft {

// Compute units of the current device (every device the library drives is the same
// part, so the first answer is kept).
static int cu_count() {
  static std::atomic<int> n{-1};
  int v = n.load(std::memory_order_relaxed);
  if (v < 0) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) !=
                                                  hipSuccess || v < 1)
      v = 256;
    n.store(v, std::memory_order_relaxed);
  }
  return v;
}

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
  *nblocks = nb;
  return launch_kernel(lc, k_stencil<T, R, BX, BY, VY, DEEP, Op>, dim3(nb), dim3(BX * BY), g, W, zc, tiles_x, tiles_y,
                       op);
}

// Streaming kernel k_stencil2: 64 x (BY*VY) tiles, the z extent split into about
// target / tiles chunks (target 0: as many as one round of resident workgroups
// holds), odd chunks swept downwards when alt is set.
template <typename T, int R, int BY, int VY, int PD, class Op>
static hipError_t launch_cfg2(const LaunchCfg& lc, const Geom& g, const StencilW<T>& W, const Op& op, int* nblocks,
                              int alt) {
  constexpr int TY = BY * VY;
  const int tiles_x = (g.nx + 63) / 64;
  const int tiles_y = (g.ny + TY - 1) / TY;
  const int tiles = tiles_x * tiles_y;
  int nchunks;
  if (lc.target_blocks > 0) {
    nchunks = std::max(1, std::min(g.nz, (lc.target_blocks + tiles - 1) / tiles));
  } else {
    // one full round of resident workgroups
    static std::atomic<int> per_cu{-1};
    int occ = per_cu.load(std::memory_order_relaxed);
    if (occ < 0) {
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, (const void*)k_stencil2<T, R, BY, VY, PD, Op>, 64 * BY, 0) !=
              hipSuccess ||
          occ < 1)
        occ = 1;
      per_cu.store(occ, std::memory_order_relaxed);
    }
    nchunks = std::max(1, std::min(g.nz, occ * cu_count() / tiles));
  }
  const int zc = (g.nz + nchunks - 1) / nchunks;
  nchunks = (g.nz + zc - 1) / zc;
  const int nb = tiles * nchunks;
  *nblocks = nb;
  return launch_kernel(lc, k_stencil2<T, R, BY, VY, PD, Op>, dim3(nb), dim3(64 * BY), g, W, zc, tiles_x, tiles_y, alt,
                       op);
}

// Forward-accumulating kernel k_stencil3, same tiles and chunks as k_stencil2.
template <typename T, int R, int BY, int VY, int PD, class Op>
static hipError_t launch_cfg3(const LaunchCfg& lc, const Geom& g, const StencilW<T>& W, const Op& op, int* nblocks,
                              int alt) {
  constexpr int TY = BY * VY;
  const int tiles_x = (g.nx + 63) / 64;
  const int tiles_y = (g.ny + TY - 1) / TY;
  const int tiles = tiles_x * tiles_y;
  int nchunks;
  if (lc.target_blocks > 0) {
    nchunks = std::max(1, std::min(g.nz, (lc.target_blocks + tiles - 1) / tiles));
  } else {
    // one full round of resident workgroups
    static std::atomic<int> per_cu{-1};
    int occ = per_cu.load(std::memory_order_relaxed);
    if (occ < 0) {
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, (const void*)k_stencil3<T, R, BY, VY, PD, Op>, 64 * BY, 0) !=
              hipSuccess ||
          occ < 1)
        occ = 1;
      per_cu.store(occ, std::memory_order_relaxed);
    }
    nchunks = std::max(1, std::min(g.nz, occ * cu_count() / tiles));
  }
  const int zc = (g.nz + nchunks - 1) / nchunks;
  nchunks = (g.nz + zc - 1) / zc;
  const int nb = tiles * nchunks;
  *nblocks = nb;
  return launch_kernel(lc, k_stencil3<T, R, BY, VY, PD, Op>, dim3(nb), dim3(64 * BY), g, W, zc, tiles_x, tiles_y, alt,
                       op);
}

template <int R, typename T, class Op>
hipError_t launch_stencil_plain(const LaunchCfg& lc, const Geom& g, const StencilW<T>& W, const Op& op, int* nblocks);

template <class Op>
struct is_cg_linear : std::false_type {};
template <typename T>
struct is_cg_linear<CGP1LOp<T>> : std::true_type {};
template <>
struct is_cg_linear<CGP1LIOp> : std::true_type {};
template <typename T>
struct is_cg_linear<CGPipeOp<T>> : std::true_type {};
template <class Op>
struct is_cg_pipe : std::false_type {};
template <typename T>
struct is_cg_pipe<CGPipeOp<T>> : std::true_type {};

template <int R, typename T, class Op>
hipError_t launch_stencil_r(const LaunchCfg& lc, const Geom& g, const StencilW<T>& W, const Op& op, int* nblocks) {
  // the CG first half by linearity and the pipelined CG iteration: streaming kernel
  // over 64x8 tiles (forward accumulation for variants 11..16)
  if constexpr (is_cg_linear<Op>::value) {
    const int var = lc.variant >= 100 ? lc.variant - 100 : lc.variant;
    const int alt = lc.variant >= 100 ? 0 : 1;
    if (var >= 11 && var <= 16) return launch_cfg3<T, R, 4, 2, 1, Op>(lc, g, W, op, nblocks, alt);
    if constexpr (R == 6) {
      switch (var) {
        case 5: return launch_cfg2<T, R, 4, 2, 1, Op>(lc, g, W, op, nblocks, alt);
        case 6: return launch_cfg2<T, R, 4, 4, 1, Op>(lc, g, W, op, nblocks, alt);
        case 7: return launch_cfg2<T, R, 4, 2, 3, Op>(lc, g, W, op, nblocks, alt);
        case 9: return launch_cfg2<T, R, 8, 2, 1, Op>(lc, g, W, op, nblocks, alt);
        case 10: return launch_cfg2<T, R, 2, 8, 1, Op>(lc, g, W, op, nblocks, alt);
        case 17: return launch_cfg2<T, R, 8, 1, 1, Op>(lc, g, W, op, nblocks, alt);
        case 18: return launch_cfg2<T, R, 16, 1, 1, Op>(lc, g, W, op, nblocks, alt);
        case 19: return launch_cfg2<T, R, 16, 2, 1, Op>(lc, g, W, op, nblocks, alt);
        default: break;
      }
    }
    // automatic: the pipelined iteration over 64x16 tiles of 8 waves (measured 3-4 %
    // faster at 63^3, 1 % at 109^3); the first half of schedule 1 over 64x8 tiles of 8 waves
    // of one row each (FP32 at 185^3: 31.2 us against 34.1 us for 4 waves of two rows, 11.6
    // against 12.7 at 109^3; FP64 53.7-58.4 against 61.5 at 185^3, 15.5 against 17.9 at
    // 109^3; 16-wave tiles were slower for both)
    if constexpr (is_cg_pipe<Op>::value) return launch_cfg2<T, R, 8, 2, 1, Op>(lc, g, W, op, nblocks, alt);
    // the FP32 first half (pairs of p and A p) from 250^3 over 64 x 32 tiles of 16 waves of
    // two rows: 474^3 452 us against 495 us (185^3: 34.0 against 28.5-29.0 us)
    if constexpr (std::is_same_v<Op, CGP1LIOp>) {
      if ((long long)g.nx * g.ny * g.nz >= 250ll * 250 * 250)
        return launch_cfg2<T, R, 16, 2, 1, Op>(lc, g, W, op, nblocks, alt);
    }
    if constexpr (std::is_same_v<Op, CGP1LOp<double>> || std::is_same_v<Op, CGP1LIOp>)
      return launch_cfg2<T, R, 8, 1, 1, Op>(lc, g, W, op, nblocks, alt);
    return launch_cfg2<T, R, 4, 2, 1, Op>(lc, g, W, op, nblocks, alt);
  } else {
    return launch_stencil_plain<R, T, Op>(lc, g, W, op, nblocks);
  }
}

template <int R, typename T, class Op>
hipError_t launch_stencil_plain(const LaunchCfg& lc, const Geom& g, const StencilW<T>& W, const Op& op, int* nblocks) {
  // the residual pass carries the XC arithmetic: one node per thread keeps it in registers
  if constexpr (std::is_same_v<Op, GradOp>) {
    return launch_cfg<T, R, 64, 4, 1, false, Op>(lc, g, W, op, nblocks);
  } else {
    // buffer-addressed streaming kernel (arrays below 4 GiB); variants >= 100 sweep
    // every chunk upwards
    const int var = lc.variant >= 100 ? lc.variant - 100 : lc.variant;
    const int alt = lc.variant >= 100 ? 0 : 1;
    if ((var < 0 || var >= 5) && g.total * (long long)sizeof(T) < (1ll << 32)) {
      if constexpr (R == 6) {
        switch (var) {
          case 5: return launch_cfg2<T, R, 4, 2, 1, Op>(lc, g, W, op, nblocks, alt);
          case 6: return launch_cfg2<T, R, 4, 4, 1, Op>(lc, g, W, op, nblocks, alt);
          case 7: return launch_cfg2<T, R, 4, 2, 3, Op>(lc, g, W, op, nblocks, alt);
          case 8: return launch_cfg2<T, R, 4, 4, 3, Op>(lc, g, W, op, nblocks, alt);
          case 9: return launch_cfg2<T, R, 8, 2, 1, Op>(lc, g, W, op, nblocks, alt);
          case 10: return launch_cfg2<T, R, 2, 8, 1, Op>(lc, g, W, op, nblocks, alt);
          case 11: return launch_cfg3<T, R, 4, 2, 1, Op>(lc, g, W, op, nblocks, alt);
          case 12: return launch_cfg3<T, R, 4, 4, 1, Op>(lc, g, W, op, nblocks, alt);
          case 13: return launch_cfg3<T, R, 4, 2, 2, Op>(lc, g, W, op, nblocks, alt);
          case 14: return launch_cfg3<T, R, 8, 2, 1, Op>(lc, g, W, op, nblocks, alt);
          case 15: return launch_cfg3<T, R, 4, 4, 2, Op>(lc, g, W, op, nblocks, alt);
          case 16: return launch_cfg3<T, R, 8, 4, 1, Op>(lc, g, W, op, nblocks, alt);
          case 17: return launch_cfg2<T, R, 8, 1, 1, Op>(lc, g, W, op, nblocks, alt);
          case 18: return launch_cfg2<T, R, 16, 1, 1, Op>(lc, g, W, op, nblocks, alt);
          case 19: return launch_cfg2<T, R, 16, 2, 1, Op>(lc, g, W, op, nblocks, alt);
          default: break;
        }
      }
      // automatic: 64 x 8 tiles of 4 waves; the plain Laplacian of large grids with more
      // waves per tile (measured, unconditional plane loop): FP64 64 x 16 tiles of 16 waves
      // up to 250^3 (185^3: 34.2-36.5 us against 38-39 for forward accumulation), forward
      // accumulation over 64 x 16 tiles above (equal to the best streaming shape at 300^3
      // and 474^3); FP32 from 250^3 on 64 x 32 tiles of 16 waves of two rows (300^3: 82
      // against 91 us; 474^3: 294 against 331; at 185^3 no shape beat 64 x 8 beyond the
      // run-to-run spread)
      const long long n3 = (long long)g.nx * g.ny * g.nz;
      if constexpr (std::is_same_v<Op, LapOp<double>>) {
        if (n3 >= 250ll * 250 * 250) return launch_cfg3<T, R, 4, 4, 2, Op>(lc, g, W, op, nblocks, alt);
        if (n3 >= 150ll * 150 * 150) return launch_cfg2<T, R, 16, 1, 1, Op>(lc, g, W, op, nblocks, alt);
      }
      if constexpr (std::is_same_v<Op, LapOp<float>>) {
        if (n3 >= 250ll * 250 * 250) return launch_cfg2<T, R, 16, 2, 1, Op>(lc, g, W, op, nblocks, alt);
      }
      return launch_cfg2<T, R, 4, 2, 1, Op>(lc, g, W, op, nblocks, alt);
    }
    // automatic shape: small grids 64x4 with deep prefetch, large grids 64x8, two rows per thread
    if (var < 0) {
      const long long tiles = (long long)((g.nx + 63) / 64) * ((g.ny + 7) / 8);
      if (tiles * g.nz <= lc.target_blocks) return launch_cfg<T, R, 64, 4, 1, true, Op>(lc, g, W, op, nblocks);
      return launch_cfg<T, R, 64, 4, 2, false, Op>(lc, g, W, op, nblocks);
    }
    if constexpr (R == 6) {
      switch (var) {
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
ALOFDFT_INST(double, CGP1LOp<double>)
ALOFDFT_INST(float, CGP1LIOp)
ALOFDFT_INST(double, CGWInitOp<double>)
ALOFDFT_INST(float, CGWInitOp<float>)
ALOFDFT_INST(double, CGPipeOp<double>)
ALOFDFT_INST(float, CGPipeOp<float>)
#undef ALOFDFT_INST

}  // namespace alofdft
