// gfx950 kernels of the AL orbital-free DFT solve (Suryanarayana & Phanish,
// arXiv:1405.6456).  Every grid array lives in the padded layout of Geom (common.h).
//
//  * k_stencil: the order-2n star stencil of Eq. FD:Laplacian (Sec. 4).  A block
//    owns a BX x (BY*VY) tile in x-y and streams a chunk of z planes.  The current
//    plane, with its x/y halo, is staged in LDS (double buffered, one barrier per
//    plane); the 2R+1 planes of the z taps stay in registers as a queue of 2R+4
//    slots that rotates by renaming (the z loop is unrolled over the queue length),
//    with the z column prefetched three planes ahead and the halo two.  The epilogue is an Op
//    functor, so the CG update, the residual/energy evaluation and the plain
//    Laplacian all share one load/stage/compute skeleton.
//  * k_pointwise: wave-per-row sweeps of the interior for the vector updates, with
//    deterministic block reductions (wavefront shuffles, then LDS) whose per-block
//    partials are summed in a fixed order by the consumer.
//  * per-atom kernels for the pseudocharge ball, self energy and forces.
#pragma once

#include <cmath>

#include "common.h"

namespace alofdft {

// ----------------------------------------------------------------- reductions
__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// Reduces acc[0..NRED) over the block; thread r < NRED writes component r to out[r].
template <int NRED, int NT>
__device__ inline void block_reduce_store(const double* acc, double* out) {
  constexpr int NW = NT / 64;
  __shared__ double sh[NRED > 0 ? NRED : 1][NW];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int r = 0; r < NRED; ++r) {
    double v = wave_sum(acc[r]);
    if (lane == 0) sh[r][wid] = v;
  }
  __syncthreads();
  if ((int)threadIdx.x < NRED) {
    double s = 0.0;
    for (int w = 0; w < NW; ++w) s += sh[threadIdx.x][w];
    out[threadIdx.x] = s;
  }
}

// Sum over n block partials (stride values apart) of component comp, in a fixed
// order; every thread of the block returns the same value.
template <int NT>
__device__ inline double block_sum_parts(const double* parts, int n, int stride, int comp) {
  __shared__ double sh[NT / 64];
  double s = 0.0;
  for (int b = threadIdx.x; b < n; b += NT) s += parts[(long long)b * stride + comp];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  double tot = 0.0;
#pragma unroll
  for (int w = 0; w < NT / 64; ++w) tot += sh[w];
  __syncthreads();
  return tot;
}

__device__ inline bool is_block0_thread0() { return blockIdx.x == 0 && threadIdx.x == 0; }

// Logical block index such that the blocks the hardware places on one XCD
// (physical index b = x mod 8) form one contiguous range of logical indices.
__device__ inline int xcd_swizzle(int b, int nb) {
  const int q = nb / 8, r = nb % 8, x = b % 8;
  return x * q + min(x, r) + b / 8;
}

// ----------------------------------------------------------------- stencil
// Software pipeline per z plane (one barrier each).  Own z-columns stream through a
// register queue of K = 2R+1+PD slots (2R+1 taps in use, PD planes in flight), the
// x/y halo through HS register sets (HS planes ahead), then the plane is staged in
// one of two LDS buffers.  DEEP = false: PD = 1, HS = 1; DEEP = true: PD = 3, HS = 2.
// The y taps that fall on this thread's own rows come from the queue, the rest from
// LDS.  Every global load is limited to planes zbeg-R .. zend-1+R of the chunk, which
// the padded layout holds.
template <typename T, int R, int BX, int BY, int VY, bool DEEP, class Op>
__global__ void __launch_bounds__(BX* BY) k_stencil(Geom g, StencilW<T> W, int zc, int tiles_x, int tiles_y, Op op) {
  constexpr int NT = BX * BY;
  constexpr int TY = BY * VY;
  constexpr int LX = BX + 2 * R;
  constexpr int LY = TY + 2 * R;
  constexpr int PD = DEEP ? 3 : 1;   // own-column planes in flight
  constexpr int HS = DEEP ? 2 : 1;   // halo register sets (planes ahead)
  constexpr int K = 2 * R + 1 + PD;  // even for both choices
  constexpr int NHALO = 2 * R * (TY + BX);
  constexpr int NH = (NHALO + NT - 1) / NT;
  constexpr int NRED = Op::NRED;
  static_assert(K % 2 == 0, "queue length must be even (LDS and halo parity)");
  __shared__ T lds[2][LY * LX];

  Op o = op;
  if (!o.template begin<NT>()) return;

  const int ntile = tiles_x * tiles_y;
  const int lb = xcd_swizzle(blockIdx.x, gridDim.x);
  const int tile = lb % ntile, chunk = lb / ntile;
  const int x0 = (tile % tiles_x) * BX, y0 = (tile / tiles_x) * TY;
  const int zbeg = chunk * zc, zend = min(zbeg + zc, g.nz);
  const int zlast = zend - 1 + R;  // last plane any output of this chunk reads
  const int tx = threadIdx.x % BX, ty = threadIdx.x / BX;
  const int gx = x0 + tx, gy0 = y0 + ty * VY;
  const long long colofs = (long long)gy0 * g.px + gx;

  // halo elements owned by this thread: LDS offset and in-plane offset
  int hl[NH];
  int hg[NH];
  bool hv[NH];
#pragma unroll
  for (int m = 0; m < NH; ++m) {
    const int e = threadIdx.x + m * NT;
    hv[m] = e < NHALO;
    int lx = 0, ly = 0;
    if (e < 2 * R * BX) {  // rows above and below the tile
      const int r = e / BX, c = e % BX;
      ly = (r < R) ? r : TY + r;
      lx = R + c;
    } else if (hv[m]) {  // columns left and right of the tile
      const int e2 = e - 2 * R * BX;
      const int r = e2 / (2 * R), c = e2 % (2 * R);
      lx = (c < R) ? c : BX + c;
      ly = R + r;
    }
    hl[m] = ly * LX + lx;
    hg[m] = (y0 - R + ly) * g.px + (x0 - R + lx);
  }

  T q[K][VY];
  T hreg[HS][NH];
  double red[NRED > 0 ? NRED : 1];
#pragma unroll
  for (int r = 0; r < (NRED > 0 ? NRED : 1); ++r) red[r] = 0.0;

  // queue: planes zbeg-R .. zbeg+R+PD-1 into slots 0 .. K-2 (slot of plane z+d at
  // unrolled step s is (s + R + d) mod K); the last slot is filled by the first prefetch
#pragma unroll
  for (int m = 0; m < K - 1; ++m) {
    const int pz = zbeg - R + m;
    const long long pb = g.base + (long long)pz * g.plane + colofs;
#pragma unroll
    for (int v = 0; v < VY; ++v) q[m][v] = (pz <= zlast) ? o.load(pb + (long long)v * g.px) : T(0);
  }
#pragma unroll
  for (int v = 0; v < VY; ++v) q[K - 1][v] = T(0);
  // halo of planes zbeg .. zbeg+HS-1 into sets 0 .. HS-1
#pragma unroll
  for (int h = 0; h < HS; ++h) {
    const bool ok = zbeg + h < zend;
    const long long hb = g.base + (long long)(zbeg + h) * g.plane;
#pragma unroll
    for (int m = 0; m < NH; ++m) hreg[h][m] = (ok && hv[m]) ? o.load(hb + hg[m]) : T(0);
  }

  for (int z0 = zbeg; z0 < zend; z0 += K) {
#pragma unroll
    for (int s = 0; s < K; ++s) {
      const int z = z0 + s;
      if (z < zend) {
        T* L = lds[s & 1];
        const int hs = (HS == 2) ? (s & 1) : 0;
        // stage plane z: own rows from the queue, halo from its register set
#pragma unroll
        for (int v = 0; v < VY; ++v) L[(R + ty * VY + v) * LX + R + tx] = q[(s + R) % K][v];
#pragma unroll
        for (int m = 0; m < NH; ++m)
          if (hv[m]) L[hl[m]] = hreg[hs][m];
        // prefetch: own column of plane z+R+PD, halo of plane z+HS (into the set just staged)
        if (z + R + PD <= zlast) {
          const long long pb = g.base + (long long)(z + R + PD) * g.plane + colofs;
#pragma unroll
          for (int v = 0; v < VY; ++v) q[(s + 2 * R + PD) % K][v] = o.load(pb + (long long)v * g.px);
        }
        if (z + HS < zend) {
          const long long hb = g.base + (long long)(z + HS) * g.plane;
#pragma unroll
          for (int m = 0; m < NH; ++m)
            if (hv[m]) hreg[hs][m] = o.load(hb + hg[m]);
        }
        __syncthreads();
        // y taps beyond this thread's rows: R rows above and R below, from LDS
        T up[R], dn[R];
#pragma unroll
        for (int m = 0; m < R; ++m) {
          up[m] = L[(ty * VY + m) * LX + R + tx];           // row offset m - R from the first own row
          dn[m] = L[(R + ty * VY + VY + m) * LX + R + tx];  // row offset VY + m
        }
#pragma unroll
        for (int v = 0; v < VY; ++v) {
          const T* row = L + (R + ty * VY + v) * LX + R + tx;
          const T c = q[(s + R) % K][v];
          T acc = W.c0 * c;
#pragma unroll
          for (int p = 1; p <= R; ++p) {
            const int a = v - p, b = v + p;  // own-row index of the y neighbours
            const T ya = (a >= 0) ? q[(s + R) % K][a >= 0 ? a : 0] : up[a + R >= 0 ? a + R : 0];
            const T yb = (b < VY) ? q[(s + R) % K][b < VY ? b : 0] : dn[b - VY < R ? b - VY : 0];
            acc += W.w[p] * (((q[(s + R - p) % K][v] + q[(s + R + p) % K][v]) + (row[-p] + row[p])) + (ya + yb));
          }
          const int gy = gy0 + v;
          if (gx < g.nx && gy < g.ny)
            o.store(g.base + (long long)z * g.plane + (long long)gy * g.px + gx, gx, gy, z, c, acc, red);
        }
      }
    }
  }
  if constexpr (NRED > 0) block_reduce_store<NRED, NT>(red, o.parts_out + (long long)blockIdx.x * NRED);
}

// ----------------------------------------------------------------- pointwise sweep
template <class Op, int NT>
__global__ void __launch_bounds__(NT) k_pointwise(Geom g, Op op) {
  constexpr int NRED = Op::NRED;
  Op o = op;
  if (!o.template begin<NT>()) return;
  double red[NRED > 0 ? NRED : 1];
#pragma unroll
  for (int r = 0; r < (NRED > 0 ? NRED : 1); ++r) red[r] = 0.0;
  const int lane = threadIdx.x & 63;
  const int nwaves = gridDim.x * (NT / 64);
  const int nrows = g.ny * g.nz;
  for (int row = blockIdx.x * (NT / 64) + (threadIdx.x >> 6); row < nrows; row += nwaves) {
    const int j = row % g.ny, k = row / g.ny;
    const long long rb = g.base + (long long)k * g.plane + (long long)j * g.px;
    for (int i = lane; i < g.nx; i += 64) o.apply(rb + i, i, j, k, red);
  }
  if constexpr (NRED > 0) block_reduce_store<NRED, NT>(red, o.parts_out + (long long)blockIdx.x * NRED);
}

// Single-block sum of block partials: out[c] = scale * sum_b parts[b*nred + c].
template <int NT>
__global__ void __launch_bounds__(NT) k_finalize(const double* parts, int nparts, int nred, double scale, double* out) {
  for (int c = 0; c < nred; ++c) {
    double v = block_sum_parts<NT>(parts, nparts, nred, c);
    if (threadIdx.x == 0) out[c] = scale * v;
  }
}

// ----------------------------------------------------------------- ops: plain Laplacian
template <typename T>
struct LapOp {
  static constexpr int NRED = 0;
  const T* x;
  T* y;
  double* parts_out;
  template <int NT>
  __device__ bool begin() { return true; }
  __device__ T load(long long i) const { return x[i]; }
  __device__ void store(long long i, int, int, int, T, T lap, double*) const { y[i] = lap; }
};

// ----------------------------------------------------------------- ops: conjugate gradients
// A = -(1/4 pi) Delta_h with zero ghosts; the stencil weights carry the -1/4pi.
// Initial residual r = rhs - A x and, when p is not null, p = r; reduces r.r and rhs.rhs.
template <typename T>
struct CGInitOp {
  static constexpr int NRED = 2;
  const T* x;
  const T* rhs;
  T* r;
  T* p;
  double* parts_out;
  template <int NT>
  __device__ bool begin() { return true; }
  __device__ T load(long long i) const { return x[i]; }
  __device__ void store(long long i, int, int, int, T, T ax, double* red) const {
    const T b = rhs[i];
    const T ri = b - ax;
    r[i] = ri;
    if (p) p[i] = ri;  // the refined solve forms only the FP64 residual
    red[0] += (double)ri * (double)ri;
    red[1] += (double)b * (double)b;
  }
};

// Iteration k, first half: reduce r.r from the previous kernel's partials, stop
// at r.r <= tol^2 ||rhs||^2, else p_new = r + beta p_old staged on load, Ap = A p_new,
// reduce p.Ap.  Block 0 keeps the scalars in CGState (indexed by k parity so no
// block reads a value written by the same launch).
template <typename T>
struct CGP1Op {
  static constexpr int NRED = 1;
  const T* r;
  const T* pold;
  T* pnew;
  T* Ap;
  CGState* st;
  const double* parts_in;
  int nparts_in, nred_in, k;
  double tol2;
  double* parts_out;
  T beta;
  template <int NT>
  __device__ bool begin() {
    if (st->done) return false;
    const double rr = block_sum_parts<NT>(parts_in, nparts_in, nred_in, 0);
    double thresh;
    if (k == 0) {
      const double rhs2 = block_sum_parts<NT>(parts_in, nparts_in, nred_in, 1);
      thresh = tol2 * rhs2;
      if (is_block0_thread0()) {
        st->rhs2 = rhs2;
        st->thresh = thresh;
      }
      if (rhs2 == 0.0) {
        if (is_block0_thread0()) { st->done = 3; st->rr_last = rr; st->iter = 0; }
        return false;
      }
    } else {
      thresh = st->thresh;
    }
    const bool bad = !isfinite(rr);
    if (bad || rr <= thresh) {
      if (is_block0_thread0()) {
        st->done = bad ? 2 : 1;
        st->rr_last = rr;
        st->iter = k;
      }
      return false;
    }
    beta = (k == 0) ? T(0) : (T)(rr / st->rrh[(k - 1) & 1]);
    if (is_block0_thread0()) {
      st->rrh[k & 1] = rr;
      st->iter = k;
    }
    return true;
  }
  __device__ T load(long long i) const { return r[i] + beta * pold[i]; }
  __device__ void store(long long i, int, int, int, T c, T ap, double* red) const {
    pnew[i] = c;
    Ap[i] = ap;
    red[0] += (double)c * (double)ap;
  }
};

// Iteration k, second half: alpha = r.r / p.Ap; x += alpha p; r -= alpha Ap; reduce r.r.
template <typename T>
struct CGP2Op {
  static constexpr int NRED = 1;
  T* x;
  T* r;
  const T* p;
  const T* Ap;
  CGState* st;
  const double* parts_in;
  int nparts_in, k;
  double* parts_out;
  T alpha;
  template <int NT>
  __device__ bool begin() {
    if (st->done) return false;
    const double pap = block_sum_parts<NT>(parts_in, nparts_in, 1, 0);
    const double a = st->rrh[k & 1] / pap;
    if (!isfinite(a) || pap <= 0.0) {
      if (is_block0_thread0()) { st->done = 2; st->iter = k; }
      return false;
    }
    alpha = (T)a;
    return true;
  }
  __device__ void apply(long long i, int, int, int, double* red) const {
    x[i] += alpha * p[i];
    const T ri = r[i] - alpha * Ap[i];
    r[i] = ri;
    red[0] += (double)ri * (double)ri;
  }
};

// ----------------------------------------------------------------- ops: density updates
// Position of node (i,j,k) relative to the box centre.
struct BoxFrame {
  double h, hx, hy, hz;  // h and half extents (n-1)/2 in index units
  __device__ void rel(int i, int j, int k, double& dx, double& dy, double& dz) const {
    dx = (i - hx) * h;
    dy = (j - hy) * h;
    dz = (k - hz) * h;
  }
};

__device__ inline void add_moments(double* red, double u2, double q, double dx, double dy, double dz) {
  const double r2 = dx * dx + dy * dy + dz * dz;
  red[0] += u2;
  red[1] += q;
  red[2] += q * dx;
  red[3] += q * dy;
  red[4] += q * dz;
  red[5] += q * (3.0 * dx * dx - r2);
  red[6] += q * (3.0 * dy * dy - r2);
  red[7] += q * (3.0 * dz * dz - r2);
  red[8] += q * 3.0 * dx * dy;
  red[9] += q * 3.0 * dx * dz;
  red[10] += q * 3.0 * dy * dz;
}

// Trial point v = u_start + t d (sign kept; every reader uses |v|); reduces
// sum v^2 and the moments of v^2 + b.
struct TrialOp {
  static constexpr int NRED = kUpdRed;
  const double* us;
  const double* d;
  const double* b;
  double* v;
  double t;
  BoxFrame f;
  double* parts_out;
  template <int NT>
  __device__ bool begin() { return true; }
  __device__ void apply(long long i, int ii, int jj, int kk, double* red) const {
    const double vi = us[i] + t * d[i];
    v[i] = vi;
    double dx, dy, dz;
    f.rel(ii, jj, kk, dx, dy, dz);
    add_moments(red, vi * vi, vi * vi + b[i], dx, dy, dz);
  }
};

// New line search: u_start = |v| (the projection u <- |u|), d = s + beta d, and the
// probe v = u_start + t d; same reductions as TrialOp.
struct DirOp {
  static constexpr int NRED = kUpdRed;
  double* us;
  double* d;
  const double* s;
  double* v;
  const double* b;
  double beta, t;
  BoxFrame f;
  double* parts_out;
  template <int NT>
  __device__ bool begin() { return true; }
  __device__ void apply(long long i, int ii, int jj, int kk, double* red) const {
    const double u = fabs(v[i]);
    us[i] = u;
    const double dn = s[i] + beta * d[i];
    d[i] = dn;
    const double vi = u + t * dn;
    v[i] = vi;
    double dx, dy, dz;
    f.rel(ii, jj, kk, dx, dy, dz);
    add_moments(red, vi * vi, vi * vi + b[i], dx, dy, dz);
  }
};

// Multipole potential of the moments mom = [.., Q, Px, Py, Pz, Txx, Tyy, Tzz,
// Txy, Txz, Tyz] (h^3 included) at offset (dx,dy,dz) from the box centre.
__device__ inline double phi_multipole(const double* mom, double dx, double dy, double dz) {
  const double r2 = dx * dx + dy * dy + dz * dz;
  const double ir = 1.0 / sqrt(r2);
  const double ir2 = ir * ir, ir3 = ir2 * ir, ir5 = ir3 * ir2;
  const double dip = mom[2] * dx + mom[3] * dy + mom[4] * dz;
  const double quad = mom[5] * dx * dx + mom[6] * dy * dy + mom[7] * dz * dz +
                      2.0 * (mom[8] * dx * dy + mom[9] * dx * dz + mom[10] * dy * dz);
  return mom[1] * ir + dip * ir3 + 0.5 * quad * ir5;
}

// Poisson right-hand side rhs = v^2 + b, plus for the multipole boundary the ghost
// values moved to the right: (1/4 pi) sum over taps leaving the grid of w_p phi_mp.
template <typename T>
struct RhsOp {
  static constexpr int NRED = 0;
  const double* v;
  const double* b;
  T* rhs;
  const double* mom;  // finalized moments (h^3 included), nullptr for zero ghosts
  StencilW<double> W;  // unscaled weights (w[1..R])
  int R, nx, ny, nz;
  BoxFrame f;
  double* parts_out;
  template <int NT>
  __device__ bool begin() { return true; }
  __device__ void apply(long long i, int ii, int jj, int kk, double*) const {
    double val = v[i] * v[i] + b[i];
    if (mom && (ii < R || jj < R || kk < R || ii >= nx - R || jj >= ny - R || kk >= nz - R)) {
      double dx, dy, dz;
      f.rel(ii, jj, kk, dx, dy, dz);
      const double h = f.h;
      double add = 0.0;
      for (int p = 1; p <= R; ++p) {
        if (ii - p < 0) add += W.w[p] * phi_multipole(mom, dx - p * h, dy, dz);
        if (ii + p >= nx) add += W.w[p] * phi_multipole(mom, dx + p * h, dy, dz);
        if (jj - p < 0) add += W.w[p] * phi_multipole(mom, dx, dy - p * h, dz);
        if (jj + p >= ny) add += W.w[p] * phi_multipole(mom, dx, dy + p * h, dz);
        if (kk - p < 0) add += W.w[p] * phi_multipole(mom, dx, dy, dz - p * h);
        if (kk + p >= nz) add += W.w[p] * phi_multipole(mom, dx, dy, dz + p * h);
      }
      val += add * (0.25 / M_PI);
    }
    rhs[i] = (T)val;
  }
};

// ----------------------------------------------------------------- ops: residual and energy
// LDA exchange + Ceperley-Alder correlation (Perdew-Zunger form) of Sec. 2/3 at
// u >= 0: energy per particle and potential; zero below rho = 1e-30.
__device__ inline void lda_xc(double u, double u13, double& eps, double& vxc) {
  if (u * u < 1e-30) {
    eps = 0.0;
    vxc = 0.0;
    return;
  }
  const double g1 = -0.1423, b1 = 1.0529, b2 = 0.3334;
  const double A1 = 0.0311, B1 = -0.048, C1 = 0.002, D1 = -0.0116;
  const double c3pi = 0.98474502184269641;       // (3/pi)^(1/3)
  const double c34pi = 0.62035049089940001;      // (3/(4 pi))^(1/3)
  const double u23 = u13 * u13;
  const double ex = -0.75 * c3pi * u23;
  const double vx = -c3pi * u23;
  const double rs = c34pi / u23;
  double ec, vc;
  if (rs >= 1.0) {
    const double sq = sqrt(rs);
    const double den = 1.0 + b1 * sq + b2 * rs;
    ec = g1 / den;
    vc = (g1 + (7.0 / 6.0) * g1 * b1 * sq + (4.0 / 3.0) * g1 * b2 * rs) / (den * den);
  } else {
    const double lr = log(rs);
    ec = A1 * lr + B1 + C1 * rs * lr + D1 * rs;
    vc = (A1 + (2.0 / 3.0) * C1 * rs) * lr + (B1 - A1 / 3.0) + (1.0 / 3.0) * (2.0 * D1 - C1) * rs;
  }
  eps = ex + ec;
  vxc = vx + vc;
}

// Residual of Eq. EulerLagrangeDiscretized at u = |v| fused with the energy sums:
//   g = -(lambda/2) Delta_h u + (V_K + V_xc + phi) u + (-eta + C_h/mu) u
// writes s_new = -g/M with the Jacobi diagonal M = -3 lambda w_0 +
// max(0, (4/3)V_K + V_K + V_xc + phi - eta + C_h/mu), optionally g, and reduces
// the GradRed sums.
struct GradOp {
  static constexpr int NRED = G_NRED;
  const double* v;
  const double* phi;
  const double* b;
  const double* d;      // nullable
  const double* s_old;  // nullable
  double* s_new;        // nullable
  double* gout;         // nullable
  const double* Cptr;   // device h^3 sum u^2 - N
  double lam_half, eta, inv_mu, vw_diag, CF;
  int xc;
  double* parts_out;
  double shift;
  template <int NT>
  __device__ bool begin() {
    shift = -eta + (*Cptr) * inv_mu;
    return true;
  }
  __device__ double load(long long i) const { return fabs(v[i]); }
  __device__ void store(long long i, int, int, int, double u, double lap, double* red) const {
    const double u13 = cbrt(u);
    const double vk = (5.0 / 3.0) * CF * u * u13;
    double eps = 0.0, vxc = 0.0;
    if (xc) lda_xc(u, u13, eps, vxc);
    const double ph = phi[i];
    const double veff = vk + vxc + ph;
    const double g = -lam_half * lap + (veff + shift) * u;
    const double M = vw_diag + fmax(0.0, (4.0 / 3.0) * vk + veff + shift);
    const double sn = -g / M;
    if (s_new) s_new[i] = sn;
    if (gout) gout[i] = g;
    const double u2 = u * u;
    red[G_GG] += g * g;
    if (d) {
      const double di = d[i];
      red[G_SLOPE] += (v[i] < 0.0) ? -g * di : g * di;
      red[G_GD] += g * di;
    }
    red[G_GS_NEW] += g * sn;
    if (s_old) red[G_GS_OLD] += g * s_old[i];
    red[G_TF] += u2 * u * u13;
    red[G_VW] += u * lap;
    red[G_XC] += eps * u2;
    red[G_ES] += (u2 + b[i]) * ph;
    red[G_U2] += u2;
  }
};

}  // namespace alofdft
