// Per-atom and layout kernels (pseudocharge, self energy and force sums, packing).
#pragma once

#include "kernels.h"

namespace alofdft {

// ----------------------------------------------------------------- nuclei
__device__ inline double bJ_val(double Z, double s, double rc, double r2) {
  if (r2 > rc * rc) return 0.0;
  const double is = 1.0 / s;
  return -Z * 0.17958712212516656 * is * is * is * exp(-r2 * is * is);  // pi^-3/2
}
__device__ inline double VJ_val(double Z, double s, double r) {
  if (r == 0.0) return -2.0 * Z / (s * 1.7724538509055159);
  return -Z * erf(r / s) / r;
}

// Pseudocharge of one nucleus: mode 0 the Gaussian charge b_J above, mode 1 the
// construction of Sec. 4, b_J = -(1/4 pi) Delta_h V_J on the nodes, with the order-2n
// stencil applied to the nucleus' potential V_J; both are zero beyond r_cut.
struct PseudoDev {
  int mode;
  int R;                      // stencil half width (mode 1)
  double s, rc, h;
  double w[kMaxRadius + 1];   // unscaled Laplacian weights w_0 .. w_R (mode 1)
};
__device__ inline double bJ_at(const PseudoDev& P, double Z, double dx, double dy, double dz) {
  const double r2 = dx * dx + dy * dy + dz * dz;
  if (P.mode == 0) return bJ_val(Z, P.s, P.rc, r2);
  if (r2 > P.rc * P.rc) return 0.0;
  auto V = [&](double x, double y, double z) { return VJ_val(Z, P.s, sqrt(x * x + y * y + z * z)); };
  double lap = 6.0 * P.w[0] * V(dx, dy, dz);
  for (int p = 1; p <= P.R; ++p) {
    const double ph = p * P.h;
    lap += P.w[p] * ((V(dx + ph, dy, dz) + V(dx - ph, dy, dz)) + (V(dx, dy + ph, dz) + V(dx, dy - ph, dz)) +
                     (V(dx, dy, dz + ph) + V(dx, dy, dz - ph)));
  }
  return -lap * (0.25 / M_PI);
}

struct AtomsDev {
  const double* R;      // 3M
  const double* Z;      // M
  const int* cell_start;  // ncell+1
  const int* cell_atoms;  // M, atom ids sorted by cell
  int M;
  int cdim[3];
  double clo[3];
  double csize;
};

// b at every interior node: sum over atoms of the 27 neighbouring cells.
__global__ void __launch_bounds__(256) k_pseudocharge(Geom g, double h, double ox, double oy, double oz, AtomsDev A,
                                                       PseudoDev P, double* b) {
  const long long n = (long long)g.nx * g.ny * g.nz;
  for (long long t = blockIdx.x * 256ll + threadIdx.x; t < n; t += (long long)gridDim.x * 256) {
    const int i = (int)(t % g.nx);
    const int j = (int)((t / g.nx) % g.ny);
    const int k = (int)(t / ((long long)g.nx * g.ny));
    const double x = ox + i * h, y = oy + j * h, z = oz + k * h;
    const int ci = (int)floor((x - A.clo[0]) / A.csize);
    const int cj = (int)floor((y - A.clo[1]) / A.csize);
    const int ck = (int)floor((z - A.clo[2]) / A.csize);
    double acc = 0.0;
    for (int c2 = max(ck - 1, 0); c2 <= min(ck + 1, A.cdim[2] - 1); ++c2)
      for (int c1 = max(cj - 1, 0); c1 <= min(cj + 1, A.cdim[1] - 1); ++c1)
        for (int c0 = max(ci - 1, 0); c0 <= min(ci + 1, A.cdim[0] - 1); ++c0) {
          const int c = (c2 * A.cdim[1] + c1) * A.cdim[0] + c0;
          for (int a = A.cell_start[c]; a < A.cell_start[c + 1]; ++a) {
            const int J = A.cell_atoms[a];
            const double dx = x - A.R[3 * J], dy = y - A.R[3 * J + 1], dz = z - A.R[3 * J + 2];
            acc += bJ_at(P, A.Z[J], dx, dy, dz);
          }
        }
    b[g.base + (long long)k * g.plane + (long long)j * g.px + i] = acc;
  }
}

// Node index box of atom J's ball.
__device__ inline void ball_box(const Geom& g, double h, const double* o, const double* RJ, double rc, int lo[3],
                                int hi[3]) {
  const int n[3] = {g.nx, g.ny, g.nz};
  for (int a = 0; a < 3; ++a) {
    lo[a] = max((int)floor((RJ[a] - rc - o[a]) / h) - 1, 0);
    hi[a] = min((int)ceil((RJ[a] + rc - o[a]) / h) + 1, n[a] - 1);
  }
}

// Per atom: self-energy sum_i b_J V_J over the ball (out[J]) and, if phi is
// given, the force sum_i (grad_h b_J)_i (phi_i - V_J(x_i)) (out3[3J..3J+2]).
template <int NT>
__global__ void __launch_bounds__(NT) k_atom_sums(Geom g, double h, double ox, double oy, double oz, AtomsDev A,
                                                  PseudoDev P, StencilW<double> wt, int R,
                                                  const double* phi, double* out_self, double* out_force) {
  const double s = P.s, rc = P.rc;
  const int J = blockIdx.x;
  const double o[3] = {ox, oy, oz};
  const double RJ[3] = {ld_dev(A.R + 3 * J), ld_dev(A.R + 3 * J + 1), ld_dev(A.R + 3 * J + 2)};
  const double ZJ = ld_dev(A.Z + J);
  int lo[3], hi[3];
  ball_box(g, h, o, RJ, rc, lo, hi);
  const int ex = hi[0] - lo[0] + 1, ey = hi[1] - lo[1] + 1, ez = hi[2] - lo[2] + 1;
  const long long nbox = (long long)ex * ey * ez;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (long long t = threadIdx.x; t < nbox; t += NT) {
    const int i = lo[0] + (int)(t % ex);
    const int j = lo[1] + (int)((t / ex) % ey);
    const int k = lo[2] + (int)(t / ((long long)ex * ey));
    const double dx = ox + i * h - RJ[0], dy = oy + j * h - RJ[1], dz = oz + k * h - RJ[2];
    const double r2 = dx * dx + dy * dy + dz * dz;
    if (r2 > rc * rc) continue;
    const double r = sqrt(r2);
    const double vj = VJ_val(ZJ, s, r);
    if (out_self) acc[3] += bJ_at(P, ZJ, dx, dy, dz) * vj;
    if (phi) {
      double gr[3] = {0.0, 0.0, 0.0};
      for (int p = 1; p <= R; ++p) {
        const double ph = p * h;
        gr[0] += wt.w[p] * (bJ_at(P, ZJ, dx + ph, dy, dz) - bJ_at(P, ZJ, dx - ph, dy, dz));
        gr[1] += wt.w[p] * (bJ_at(P, ZJ, dx, dy + ph, dz) - bJ_at(P, ZJ, dx, dy - ph, dz));
        gr[2] += wt.w[p] * (bJ_at(P, ZJ, dx, dy, dz + ph) - bJ_at(P, ZJ, dx, dy, dz - ph));
      }
      const double pot = phi[g.base + (long long)k * g.plane + (long long)j * g.px + i] - vj;
      acc[0] += gr[0] * pot;
      acc[1] += gr[1] * pot;
      acc[2] += gr[2] * pot;
    }
  }
  __shared__ double res[4];
  block_reduce_store<4, NT>(acc, res);
  __syncthreads();
  if (threadIdx.x == 0) {
    if (out_self) out_self[J] = res[3];
    if (out_force) {
      out_force[3 * J] = res[0];
      out_force[3 * J + 1] = res[1];
      out_force[3 * J + 2] = res[2];
    }
  }
}

// Superposition of atomic densities (Sec. 4 initial guess): rho = sum_J Z_J (pi w^2)^(-3/2)
// exp(-r^2/w^2) over the atoms within 5w (cell list of cells >= 5w) plus the floor, at
// every interior node; block partials of sum rho.
template <int NT>
__global__ void __launch_bounds__(NT) k_atomic_density(Geom g, double h, double ox, double oy, double oz, AtomsDev A,
                                                       double w, double floor_rho, double* rho, double* parts) {
  const long long n = (long long)g.nx * g.ny * g.nz;
  const double rc2 = 25.0 * w * w, iw2 = 1.0 / (w * w);
  const double norm = 1.0 / (w * w * w) * 0.17958712212516656;  // (pi w^2)^(-3/2)
  double acc[1] = {0.0};
  for (long long t = blockIdx.x * (long long)NT + threadIdx.x; t < n; t += (long long)gridDim.x * NT) {
    const int i = (int)(t % g.nx);
    const int j = (int)((t / g.nx) % g.ny);
    const int k = (int)(t / ((long long)g.nx * g.ny));
    const double x = ox + i * h, y = oy + j * h, z = oz + k * h;
    const int ci = (int)floor((x - A.clo[0]) / A.csize);
    const int cj = (int)floor((y - A.clo[1]) / A.csize);
    const int ck = (int)floor((z - A.clo[2]) / A.csize);
    double r = 0.0;
    for (int c2 = max(ck - 1, 0); c2 <= min(ck + 1, A.cdim[2] - 1); ++c2)
      for (int c1 = max(cj - 1, 0); c1 <= min(cj + 1, A.cdim[1] - 1); ++c1)
        for (int c0 = max(ci - 1, 0); c0 <= min(ci + 1, A.cdim[0] - 1); ++c0) {
          const int c = (c2 * A.cdim[1] + c1) * A.cdim[0] + c0;
          for (int a = A.cell_start[c]; a < A.cell_start[c + 1]; ++a) {
            const int J = A.cell_atoms[a];
            const double dx = x - A.R[3 * J], dy = y - A.R[3 * J + 1], dz = z - A.R[3 * J + 2];
            const double r2 = dx * dx + dy * dy + dz * dz;
            if (r2 <= rc2) r += A.Z[J] * norm * exp(-r2 * iw2);
          }
        }
    r += floor_rho;
    rho[g.base + (long long)k * g.plane + (long long)j * g.px + i] = r;
    acc[0] += r;
  }
  block_reduce_store<1, NT>(acc, parts + blockIdx.x);
}

// u = sqrt(rho * scale) over the interior, into a dense array (x fastest).
__global__ void __launch_bounds__(256) k_density_to_u(Geom g, const double* rho, const double* sum_rho, double N,
                                                      double h3, double* u_dense) {
  const long long n = (long long)g.nx * g.ny * g.nz;
  const double scale = N / (h3 * ld_dev(sum_rho));
  for (long long t = blockIdx.x * 256ll + threadIdx.x; t < n; t += (long long)gridDim.x * 256) {
    const long long i = t % g.nx, j = (t / g.nx) % g.ny, k = t / ((long long)g.nx * g.ny);
    u_dense[t] = sqrt(rho[g.base + k * g.plane + j * g.px + i] * scale);
  }
}

// Order-independent checksum of the interior of a padded FP64 array, added to *out: the
// wrapping sum over nodes of the SplitMix64 finalizer of (value bits XOR index times the
// generator's increment).  Integer sums do not depend on the order of the blocks, so equal
// arrays give equal checksums whatever the schedule (a diagnostic of the solve trace).
__device__ inline unsigned long long mix64(unsigned long long z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
__global__ void __launch_bounds__(256) k_checksum(Geom g, const double* a, unsigned long long* out) {
  const long long n = (long long)g.nx * g.ny * g.nz;
  unsigned long long acc = 0;
  for (long long t = blockIdx.x * 256ll + threadIdx.x; t < n; t += (long long)gridDim.x * 256) {
    const long long i = t % g.nx, j = (t / g.nx) % g.ny, k = t / ((long long)g.nx * g.ny);
    const unsigned long long bits = __builtin_bit_cast(unsigned long long, a[g.base + k * g.plane + j * g.px + i]);
    acc += mix64(bits ^ ((unsigned long long)t * 0x9E3779B97F4A7C15ull));
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  if ((threadIdx.x & 63) == 0) atomicAdd(out, acc);
}

// ----------------------------------------------------------------- layout conversion
template <typename TS, typename TD>
__global__ void __launch_bounds__(256) k_pack(Geom g, const TS* dense, TD* padded, int absval) {
  const long long n = (long long)g.nx * g.ny * g.nz;
  for (long long t = blockIdx.x * 256ll + threadIdx.x; t < n; t += (long long)gridDim.x * 256) {
    const long long i = t % g.nx, j = (t / g.nx) % g.ny, k = t / ((long long)g.nx * g.ny);
    TS v = dense[t];
    if (absval) v = v < TS(0) ? -v : v;
    if (!in_domain(g, (int)i, (int)j, (int)k)) v = TS(0);  // a Dirichlet node of the active domain
    padded[g.base + k * g.plane + j * g.px + i] = (TD)v;
  }
}
template <typename TS, typename TD>
__global__ void __launch_bounds__(256) k_unpack(Geom g, const TS* padded, TD* dense, int absval) {
  const long long n = (long long)g.nx * g.ny * g.nz;
  for (long long t = blockIdx.x * 256ll + threadIdx.x; t < n; t += (long long)gridDim.x * 256) {
    const long long i = t % g.nx, j = (t / g.nx) % g.ny, k = t / ((long long)g.nx * g.ny);
    TS v = padded[g.base + k * g.plane + j * g.px + i];
    if (absval) v = v < TS(0) ? -v : v;
    dense[t] = (TD)v;
  }
}

// Fill of a padded array (halo included) with a value.
template <typename T>
__global__ void __launch_bounds__(256) k_fill(T* a, long long n, T val) {
  for (long long t = blockIdx.x * 256ll + threadIdx.x; t < n; t += (long long)gridDim.x * 256) a[t] = val;
}

}  // namespace alofdft
