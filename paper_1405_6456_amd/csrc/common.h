// Shared declarations of the gfx950 kernels and the host engine.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace alofdft {

constexpr int kMaxRadius = 8;       // fd half width n <= 8
constexpr int kPointwiseThreads = 256;
constexpr int kPointwiseBlocks = 2048;  // grid-stride blocks of the pointwise kernels
constexpr int kMaxRed = 12;         // reductions per kernel

// Padded storage of one grid array: the interior n = (nx, ny, nz) is surrounded
// by a zero halo of width >= R (the zero ghosts of Sec. 4), x fastest.  Extra
// x and y padding lets the stencil tiles run past the interior without bounds
// checks on loads.  Element (i,j,k) of the interior sits at base + k*plane + j*px + i.
struct Geom {
  int nx, ny, nz;
  int R;           // halo width = fd half width
  int px, py, pz;  // padded extents
  long long plane; // px*py
  long long base;  // offset of interior (0,0,0)
  long long total; // px*py*pz
  // active domain (Sec. 5.1): nullptr for the whole box, else for every interior row
  // (j, k) the x range dom[2(j + ny k)] .. dom[2(j + ny k) + 1] of its free nodes (empty
  // when the first exceeds the second); every other node is a Dirichlet node (zero)
  const int* dom;
};

// Whether interior node (i, j, k) is a free node of the active domain.
__host__ __device__ inline bool in_domain(const Geom& g, int i, int j, int k) {
  if (!g.dom) return true;
  const long long r = 2ll * ((long long)k * g.ny + j);
  return i >= g.dom[r] && i <= g.dom[r + 1];
}

// Stencil coefficients scaled by a factor: c0 = 6 w_0 * scale, w[p] = w_p * scale.
template <typename T>
struct StencilW {
  T c0;
  T w[kMaxRadius + 1];
};

// Per-solve scalars kept on the device by the conjugate-gradient kernels.
struct CGState {
  double rrh[2];   // r.r at the start of iteration k, indexed by k & 1
  double rhs2;     // ||rhs||^2
  double thresh;   // tol^2 ||rhs||^2
  double rr_last;  // r.r when the solve stopped
  double ah[2];    // alpha of iteration k, indexed by k & 1 (one-reduction schedule)
  long long iter;  // iterations completed
  int done;        // 0 running, 1 converged, 2 non-finite, 3 zero rhs, 4 rounding breakdown
  int pad;
  long long done_iter;  // iteration whose prologue set done (iter must still equal it at the end)
  long long halt;       // 1 + done_iter, written atomically with done (0 while running)
  double xa[2];         // alpha of iteration k, indexed by k & 1: two-launch CG applies it to x
                        // in the first half of iteration k + 1
};

// Multipole moments of u^2 + b about the box centre and the constraint sum,
// as produced by the update kernels: [sum u^2, Q, Px, Py, Pz, Txx, Tyy, Tzz, Txy, Txz, Tyz]
// (all multiplied by h^3 after the final reduction).
constexpr int kUpdRed = 11;

// Reductions of the residual pass (see GradOp).
enum GradRed {
  G_GG = 0,     // sum g^2
  G_SLOPE,      // sum g sign(v) d   (derivative along the projected path)
  G_GD,         // sum g d
  G_GS_NEW,     // sum g s_new   (= -delta_new)
  G_GS_OLD,     // sum g s_old   (= -delta_mid)
  G_TF,         // sum |u|^(10/3)
  G_VW,         // sum u Delta_h u
  G_XC,         // sum eps_xc u^2
  G_ES,         // sum (u^2 + b) phi
  G_U2,         // sum u^2
  G_UG,         // sum u g   (Rayleigh quotient of the Lagrange-multiplier method)
  G_NRED
};

}  // namespace alofdft
