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

#include <type_traits>

#include "common.h"

namespace alofdft {

// ----------------------------------------------------------------- values written by other blocks
// The CG scalars, finalized sums and block partials are written by one block (of this
// launch, for the verdict flag, or of an earlier one) and read by all: they are read with
// an agent-scope atomic load, a vector load that is coherent with other blocks' writes and
// well defined while another block of the same launch writes the value (a plain load at a
// wave-uniform address would go through the scalar data cache).
template <typename T>
__device__ inline T ld_dev(const T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ----------------------------------------------------------------- reductions
__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// Ops whose stencil input does not depend on the scalars their prologue computes
// declare LATE_BEGIN = true.
template <class Op, class = void>
struct late_begin : std::false_type {};
template <class Op>
struct late_begin<Op, std::void_t<decltype(Op::LATE_BEGIN)>> : std::bool_constant<Op::LATE_BEGIN> {};

// Node operands an op's epilogue reads at the node itself (NPRE of them): the streaming
// kernel loads them one plane ahead through op.prefetch and hands them to op.storep, so
// the wait for them does not also wait for that step's plane prefetches.  Ops without
// NPRE read nothing at the node (or do it inside storeb).
template <class Op, class = void>
struct op_npre : std::integral_constant<int, 0> {};
template <class Op>
struct op_npre<Op, std::void_t<decltype(Op::NPRE)>> : std::integral_constant<int, Op::NPRE> {};

// Ops with XPASS = true may leave their prologue in a mode (op.xonly) in which the
// launch only runs op.xpass(g) over the grid instead of the stencil.
template <class Op, class = void>
struct op_xpass : std::false_type {};
template <class Op>
struct op_xpass<Op, std::void_t<decltype(Op::XPASS)>> : std::bool_constant<Op::XPASS> {};

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
// order; every thread of the block returns the same value.  Loads go out in
// batches of 8 per thread, so the sum costs one memory latency per 8 x NT partials.
template <int NT>
__device__ inline double block_sum_parts(const double* parts, int n, int stride, int comp) {
  __shared__ double sh[NT / 64];
  double s = 0.0;
  for (int b0 = threadIdx.x; b0 < n; b0 += 8 * NT) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int b = b0 + u * NT;
      v[u] = b < n ? ld_dev(parts + (long long)b * stride + comp) : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) s += v[u];
  }
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

// The CG verdict flag is written by block 0 of a launch while the other blocks of the same
// launch run.  A block reads it once and shares it through LDS, so all its waves take the
// same branch: a wave that returned on a fresh flag while its siblings, which read the old
// one, waited at the next barrier of the prologue's reduction would release that barrier
// early and the siblings would sum per-wave partials that were never written.
__device__ inline int block_read_done(const CGState* st) {
  __shared__ int flag;
  if (threadIdx.x == 0) flag = ld_dev(&st->done);
  __syncthreads();
  return flag;
}

// The verdict with the iteration that reached it, as one word (1 + that iteration, 0
// while running), so a block of iteration k can tell a verdict of an earlier launch
// (halt <= k: stop) from one its own launch's block 0 has just written (halt = k + 1:
// the block reaches the same verdict from the same sums itself).  Read like done.
__device__ inline long long block_read_halt(const CGState* st) {
  __shared__ long long flag;
  if (threadIdx.x == 0) flag = ld_dev(&st->halt);
  __syncthreads();
  return flag;
}
__device__ inline void set_halt(CGState* st, long long k) {
  __hip_atomic_store(&st->halt, k + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

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
  if constexpr (op_xpass<Op>::value) {
    if (o.xonly) {
      o.xpass(g);
      return;
    }
  }

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
          if (gx < g.nx && gy < g.ny)  // Dirichlet nodes of an active domain: zero stencil value
            o.store(g.base + (long long)z * g.plane + (long long)gy * g.px + gx, gx, gy, z, c,
                    in_domain(g, gx, gy, z) ? acc : T(0), red);
        }
      }
    }
  }
  if constexpr (NRED > 0) {
    block_reduce_store<NRED, NT>(red, o.parts_out + (long long)blockIdx.x * NRED);
  }
}

// ----------------------------------------------------------------- streaming stencil, buffer addressed
// Raw buffer access to one grid array: the address is the array base + a per-lane
// byte offset (VGPR) + a wave-uniform byte offset (SGPR), so the streaming loop
// needs no per-load address arithmetic.  Arrays must stay below 4 GiB.
__device__ inline __amdgpu_buffer_rsrc_t brsrc(const void* p, uint32_t nbytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)nbytes, 0x00020000);
}
template <typename T>
__device__ inline T bld(const T* p, uint32_t nb, uint32_t vo, uint32_t so);
template <>
__device__ inline float bld<float>(const float* p, uint32_t nb, uint32_t vo, uint32_t so) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(brsrc(p, nb), (int)vo, (int)so, 0));
}
template <>
__device__ inline double bld<double>(const double* p, uint32_t nb, uint32_t vo, uint32_t so) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(brsrc(p, nb), (int)vo, (int)so, 0));
}
// Stores of the streaming kernel are non-temporal (cache policy nt): the outputs are
// not read again by the launch, so they should not displace the input planes that
// neighbouring tiles still read from L2.
#ifndef ALOFDFT_STORE_POLICY
#define ALOFDFT_STORE_POLICY 2
#endif
template <typename T>
__device__ inline void bst(T* p, uint32_t nb, uint32_t vo, uint32_t so, T v);
template <>
__device__ inline void bst<float>(float* p, uint32_t nb, uint32_t vo, uint32_t so, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), brsrc(p, nb), (int)vo, (int)so,
                                        ALOFDFT_STORE_POLICY);
}
template <>
__device__ inline void bst<double>(double* p, uint32_t nb, uint32_t vo, uint32_t so, double v) {
  using u2 = uint32_t __attribute__((ext_vector_type(2)));
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, v), brsrc(p, nb), (int)vo, (int)so,
                                        ALOFDFT_STORE_POLICY);
}
// p and A p of one node side by side (the interleaved FP32 CG layout), moved by one
// 8-byte access; the byte offsets are those of the pair array
struct PApair {
  float p, ap;
};
__device__ inline PApair bldpair(const float* pa, uint32_t nb, uint32_t vo, uint32_t so) {
  return __builtin_bit_cast(PApair, __builtin_amdgcn_raw_buffer_load_b64(brsrc(pa, nb), (int)vo, (int)so, 0));
}
__device__ inline void bstpair(float* pa, uint32_t nb, uint32_t vo, uint32_t so, PApair v) {
  using u2 = uint32_t __attribute__((ext_vector_type(2)));
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, v), brsrc(pa, nb), (int)vo, (int)so,
                                        ALOFDFT_STORE_POLICY);
}

// Same computation as k_stencil with a different schedule for large planes.  The
// block is BY waves; wave w owns VY consecutive rows of a 64 x (BY*VY) tile and lane
// l the column x0 + l, so the row part of every address is wave-uniform and only
// the lane term is per thread.  The z column of each own node streams through a
// register queue of K = 2R+1+PD slots (PD planes prefetched ahead); the 2R halo
// rows of the tile are loaded one row per wave instruction and the 2R*BY*VY x-halo
// nodes by the first threads, HS planes ahead in HS register sets, all staged in LDS
// (double buffered, one barrier per plane).  With alt set, odd z chunks are swept downwards, so the planes two
// neighbouring chunks share are read by both at about the same time.
template <typename T, int R, int BY, int VY, int PD, class Op, int HS = 1>
__global__ void __launch_bounds__(64 * BY) k_stencil2(Geom g, StencilW<T> W, int zc, int tiles_x, int tiles_y,
                                                      int alt, Op op) {
  constexpr int BX = 64;
  constexpr int NT = BX * BY;
  constexpr int TY = BY * VY;
  constexpr int LX = BX + 2 * R;
  constexpr int LY = TY + 2 * R;
  constexpr int K = 2 * R + 1 + PD;
  constexpr int HR = (2 * R + BY - 1) / BY;  // halo rows per wave
  constexpr int NXH = 2 * R * TY;            // x-halo nodes per plane
  constexpr int XH = (NXH + NT - 1) / NT;    // x-halo nodes per thread
  constexpr int NRED = Op::NRED;
  constexpr uint32_t ES = sizeof(T);
  static_assert(K % 2 == 0, "queue length must be even (LDS parity)");
  static_assert(K % HS == 0, "halo register sets must divide the queue");
  __shared__ T lds[2][LY * LX];

  Op o = op;
  // an op whose loads do not depend on its prologue's scalars starts the queue
  // loads first, so the prologue's reduction overlaps them
  constexpr bool LATE = late_begin<Op>::value;
  if constexpr (!LATE) {
    if (!o.template begin<NT>()) return;
    if constexpr (op_xpass<Op>::value) {
      if (o.xonly) {
        o.xpass(g);
        return;
      }
    }
  }

  const uint32_t nb = (uint32_t)(g.total * (long long)ES);
  const int ntile = tiles_x * tiles_y;
  const int nchunks = gridDim.x / ntile;
  const int lb = xcd_swizzle(blockIdx.x, gridDim.x);
  // mode bit 1 clear: chunk-fastest order within each XCD's contiguous range, so an XCD
  // owns whole tile columns and the chunks of one column meet in its L2; set:
  // tile-fastest, so an XCD owns whole chunks (a z slab when the chunk count is a
  // multiple of 8) and the x-y halos of neighbouring tiles meet in its L2.
  // Bit 0: odd chunks sweep downwards.
  const bool slab = (alt & 2) != 0;
  const int tile = slab ? lb % ntile : lb / nchunks, chunk = slab ? lb / ntile : lb % nchunks;
  const int x0 = (tile % tiles_x) * BX, y0 = (tile / tiles_x) * TY;
  const int zbeg = chunk * zc, zend = min(zbeg + zc, g.nz), len = zend - zbeg;
  const bool down = (alt & 1) && (chunk & 1);
  const int zfirst = down ? zend - 1 : zbeg;
  const long long pstep = down ? -g.plane : g.plane;
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint32_t rowb = (uint32_t)g.px * ES;
  const uint32_t vl = (uint32_t)lane * ES;
  // byte offset of node (x0, y0) of logical plane t (plane zfirst + t * direction)
  const long long org = g.base + (long long)zfirst * g.plane + (long long)y0 * g.px + x0;
  auto plane_off = [&](int t) -> uint32_t { return (uint32_t)((org + (long long)t * pstep) * ES); };
  const uint32_t own_row = (uint32_t)(wv * VY) * rowb;

  // halo rows handled by this wave: LDS row and byte offset from row y0 - R
  int hly[HR];
  uint32_t hro[HR];
  bool hok[HR];
#pragma unroll
  for (int i = 0; i < HR; ++i) {
    const int hr = wv + BY * i;
    hok[i] = hr < 2 * R;
    const int ly = hr < R ? hr : TY + hr;
    hly[i] = ly;
    hro[i] = (uint32_t)ly * rowb;  // row y0 - R + ly, biased by +R rows
  }
  // x-halo nodes of this thread: LDS index and byte offset from (x0 - R, y0)
  int xl[XH];
  uint32_t xo[XH];
  bool xok[XH];
#pragma unroll
  for (int m = 0; m < XH; ++m) {
    const int e = threadIdx.x + m * NT;
    xok[m] = e < NXH;
    const int r = xok[m] ? e / (2 * R) : 0, c = xok[m] ? e % (2 * R) : 0;
    const int lx = c < R ? c : BX + c;
    xl[m] = (R + r) * LX + lx;
    xo[m] = (uint32_t)((r * g.px + lx) * ES);
  }
  const uint32_t rbias = (uint32_t)R * rowb;       // halo rows: offsets carry +R rows
  const uint32_t xbias = (uint32_t)R * ES;         // x halo: offsets carry +R columns

  T q[K][VY];
  T hrg[HS][HR];
  T xrg[HS][XH];
  constexpr int NPRE = op_npre<Op>::value;
  T pre[2][VY][NPRE > 0 ? NPRE : 1];  // node operands of the epilogue, plane t in set t & 1
  double red[NRED > 0 ? NRED : 1];
#pragma unroll
  for (int r = 0; r < (NRED > 0 ? NRED : 1); ++r) red[r] = 0.0;

  // Every global load and store of the streaming loop is issued unconditionally (planes
  // past the chunk are clamped to its last plane and their values never used; lanes
  // outside the interior store zeros into the zero padding), so the number of memory
  // operations in flight is the same on every path and the waits for a prefetched
  // plane do not also wait for the loads issued after it.
  constexpr bool HALL = (2 * R) % BY == 0;  // every wave loads all its HR halo rows
  const int tlast = len - 1;

  // queue: logical planes -R .. R+PD-1 into slots 0 .. K-2 (slot of plane t+d at
  // unrolled step s is (s + R + d) mod K); the last slot is filled by the first prefetch
#pragma unroll
  for (int m = 0; m < K - 1; ++m) {
    const uint32_t so = plane_off(min(m - R, tlast + R)) + own_row;
#pragma unroll
    for (int v = 0; v < VY; ++v) q[m][v] = o.loadb(nb, vl, so + v * rowb);
  }
#pragma unroll
  for (int v = 0; v < VY; ++v) q[K - 1][v] = T(0);
  // x-y halo of planes 0 .. HS-1 into sets 0 .. HS-1 (plane t is staged from set t mod HS)
  auto load_halo = [&](int t, int set) __attribute__((always_inline)) {
    const uint32_t so = plane_off(min(t, tlast));
#pragma unroll
    for (int i = 0; i < HR; ++i)
      if (HALL || hok[i]) hrg[set][i] = o.loadb(nb, vl, so + hro[i] - rbias);
#pragma unroll
    for (int m = 0; m < XH; ++m) xrg[set][m] = o.loadb(nb, xok[m] ? xo[m] : 0u, so - xbias);
  };
#pragma unroll
  for (int d = 0; d < HS; ++d) load_halo(d, d);
  auto load_pre = [&](int t, int set) __attribute__((always_inline)) {
    if constexpr (NPRE > 0) {
      const uint32_t so = plane_off(min(t, tlast)) + own_row;
#pragma unroll
      for (int v = 0; v < VY; ++v) o.prefetch(nb, vl, so + v * rowb, pre[set][v]);
    }
  };
  load_pre(0, 0);
  if constexpr (LATE) {
    if (!o.template begin<NT>()) return;
    if constexpr (op_xpass<Op>::value) {
      if (o.xonly) {
        o.xpass(g);
        return;
      }
    }
  }

  auto step = [&](int s, int t) __attribute__((always_inline)) {
    T* L = lds[s & 1];
    const int hs = s % HS;
#pragma unroll
    for (int v = 0; v < VY; ++v) L[(R + wv * VY + v) * LX + R + lane] = q[(s + R) % K][v];
#pragma unroll
    for (int i = 0; i < HR; ++i)
      if (HALL || hok[i]) L[hly[i] * LX + R + lane] = hrg[hs][i];
#pragma unroll
    for (int m = 0; m < XH; ++m)
      if (xok[m]) L[xl[m]] = xrg[hs][m];
    load_pre(t + 1, (s + 1) & 1);
    {
      const uint32_t so = plane_off(min(t + R + PD, tlast + R)) + own_row;
#pragma unroll
      for (int v = 0; v < VY; ++v) q[(s + 2 * R + PD) % K][v] = o.loadb(nb, vl, so + v * rowb);
    }
    load_halo(t + HS, hs);
    __syncthreads();
    const uint32_t so = plane_off(t) + own_row;
    const int z = zfirst + (down ? -t : t);
#pragma unroll
    for (int v = 0; v < VY; ++v) {
      const T* row = L + (R + wv * VY + v) * LX + R + lane;
      const T c = q[(s + R) % K][v];
      T acc = W.c0 * c;
#pragma unroll
      for (int p = 1; p <= R; ++p) {
        const int a = v - p, b = v + p;  // own-row index of the y neighbours
        const T ya = (a >= 0) ? q[(s + R) % K][a >= 0 ? a : 0] : row[-p * LX];
        const T yb = (b < VY) ? q[(s + R) % K][b < VY ? b : 0] : row[p * LX];
        acc += W.w[p] * (((q[(s + R - p) % K][v] + q[(s + R + p) % K][v]) + (row[-p] + row[p])) + (ya + yb));
      }
      const int gx = x0 + lane, gy = y0 + wv * VY + v;
      // a lane outside the interior sits in the zero padding, where every input of the
      // op is zero: with the stencil value zeroed too, the op stores zeros there and
      // adds nothing to its sums.  The Dirichlet nodes of an active domain are treated
      // alike (every array is zero there too).
      const bool in = gy < g.ny && gx < g.nx && in_domain(g, gx, min(gy, g.ny - 1), z);
      if constexpr (NPRE > 0)
        o.storep(nb, vl, so + v * rowb, c, in ? acc : T(0), pre[s & 1][v], red);
      else
        o.storeb(nb, vl, so + v * rowb, gx, gy, z, c, in ? acc : T(0), red);
    }
  };

  int t0 = 0;
  for (; t0 + K <= len; t0 += K) {
#pragma unroll
    for (int s = 0; s < K; ++s) step(s, t0 + s);
  }
  if (t0 < len) {
#pragma unroll
    for (int s = 0; s < K; ++s)
      if (t0 + s < len) step(s, t0 + s);
  }
  if constexpr (NRED > 0) {
    block_reduce_store<NRED, NT>(red, o.parts_out + (long long)blockIdx.x * NRED);
  }
}

// Forward-accumulating variant of k_stencil2.  Every plane t' of the chunk and its
// 2R z neighbours is loaded once, PD planes ahead, together with its x/y halo, so a
// plane and the halo copies of it that the neighbouring tiles read are fetched at
// about the same time (and meet in L2).  Its z taps are scattered forward into a
// ring of 2R+2 accumulators -- slot (t + R) mod K holds output plane t, which
// receives w_|d| u(t + d) from each plane as it arrives -- and its x/y taps are
// added from LDS when the plane itself is staged; output t is complete, and
// stored, when plane t + R has arrived.  Same arithmetic per node as k_stencil.
template <typename T, int R, int BY, int VY, int PD, class Op>
__global__ void __launch_bounds__(64 * BY) k_stencil3(Geom g, StencilW<T> W, int zc, int tiles_x, int tiles_y,
                                                      int alt, Op op) {
  constexpr int BX = 64;
  constexpr int NT = BX * BY;
  constexpr int TY = BY * VY;
  constexpr int LX = BX + 2 * R;
  constexpr int LY = TY + 2 * R;
  constexpr int K = 2 * R + 2;               // accumulator ring (even: LDS parity)
  constexpr int HR = (2 * R + BY - 1) / BY;  // halo rows per wave
  constexpr int NXH = 2 * R * TY;            // x-halo nodes per plane
  constexpr int XH = (NXH + NT - 1) / NT;    // x-halo nodes per thread
  constexpr int NRED = Op::NRED;
  constexpr uint32_t ES = sizeof(T);
  static_assert(K % PD == 0, "prefetch sets must divide the ring");
  __shared__ T lds[2][LY * LX];

  Op o = op;
  if (!o.template begin<NT>()) return;
  if constexpr (op_xpass<Op>::value) {
    if (o.xonly) {
      o.xpass(g);
      return;
    }
  }

  const uint32_t nb = (uint32_t)(g.total * (long long)ES);
  const int ntile = tiles_x * tiles_y;
  const int nchunks = gridDim.x / ntile;
  const int lb = xcd_swizzle(blockIdx.x, gridDim.x);
  // mode bit 1 clear: chunk-fastest order within each XCD's contiguous range, so an XCD
  // owns whole tile columns and the chunks of one column meet in its L2; set:
  // tile-fastest, so an XCD owns whole chunks (a z slab when the chunk count is a
  // multiple of 8) and the x-y halos of neighbouring tiles meet in its L2.
  // Bit 0: odd chunks sweep downwards.
  const bool slab = (alt & 2) != 0;
  const int tile = slab ? lb % ntile : lb / nchunks, chunk = slab ? lb / ntile : lb % nchunks;
  const int x0 = (tile % tiles_x) * BX, y0 = (tile / tiles_x) * TY;
  const int zbeg = chunk * zc, zend = min(zbeg + zc, g.nz), len = zend - zbeg;
  const bool down = (alt & 1) && (chunk & 1);
  const int zfirst = down ? zend - 1 : zbeg;
  const long long pstep = down ? -g.plane : g.plane;
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint32_t rowb = (uint32_t)g.px * ES;
  const uint32_t vl = (uint32_t)lane * ES;
  const long long org = g.base + (long long)zfirst * g.plane + (long long)y0 * g.px + x0;
  // byte offset of node (x0, y0) of chunk plane t (t = -R .. len-1+R)
  auto plane_off = [&](int t) -> uint32_t { return (uint32_t)((org + (long long)t * pstep) * ES); };
  const uint32_t own_row = (uint32_t)(wv * VY) * rowb;

  int hly[HR];
  uint32_t hro[HR];
  bool hok[HR];
#pragma unroll
  for (int i = 0; i < HR; ++i) {
    const int hr = wv + BY * i;
    hok[i] = hr < 2 * R;
    const int ly = hr < R ? hr : TY + hr;
    hly[i] = ly;
    hro[i] = (uint32_t)ly * rowb;  // row y0 - R + ly, biased by +R rows
  }
  int xl[XH];
  uint32_t xo[XH];
  bool xok[XH];
#pragma unroll
  for (int m = 0; m < XH; ++m) {
    const int e = threadIdx.x + m * NT;
    xok[m] = e < NXH;
    const int r = xok[m] ? e / (2 * R) : 0, c = xok[m] ? e % (2 * R) : 0;
    const int lx = c < R ? c : BX + c;
    xl[m] = (R + r) * LX + lx;
    xo[m] = (uint32_t)((r * g.px + lx) * ES);
  }
  const uint32_t rbias = (uint32_t)R * rowb;
  const uint32_t xbias = (uint32_t)R * ES;

  constexpr bool NEEDC = Op::NEEDC;  // the epilogue uses the centre value (kept R planes)
  T acc[K][VY];
  T cen[NEEDC ? K : 1][VY];
  T own[PD][VY];
  T hrg[PD][HR];
  T xrg[PD][XH];
  double red[NRED > 0 ? NRED : 1];
#pragma unroll
  for (int r = 0; r < (NRED > 0 ? NRED : 1); ++r) red[r] = 0.0;
#pragma unroll
  for (int k = 0; k < K; ++k)
#pragma unroll
    for (int v = 0; v < VY; ++v) acc[k][v] = T(0);

  const int nsteps = len + 2 * R;  // chunk planes t = i - R, i = 0 .. nsteps-1
  auto fetch = [&](int i, int set) {
    const int t = i - R;
    const uint32_t so = plane_off(t);
#pragma unroll
    for (int v = 0; v < VY; ++v) own[set][v] = o.loadb(nb, vl, so + own_row + v * rowb);
    if (t >= 0 && t < len) {
#pragma unroll
      for (int h = 0; h < HR; ++h)
        if (hok[h]) hrg[set][h] = o.loadb(nb, vl, so + hro[h] - rbias);
#pragma unroll
      for (int m = 0; m < XH; ++m)
        if (xok[m]) xrg[set][m] = o.loadb(nb, xo[m], so - xbias);
    }
  };
#pragma unroll
  for (int d = 0; d < PD; ++d)
    if (d < nsteps) fetch(d, d);

  for (int i0 = 0; i0 < nsteps; i0 += K) {
#pragma unroll
    for (int s = 0; s < K; ++s) {
      const int i = i0 + s;
      if (i < nsteps) {
        const int t = i - R;
        const int set = s % PD;
        T u[VY];
#pragma unroll
        for (int v = 0; v < VY; ++v) u[v] = own[set][v];
        if constexpr (NEEDC) {
#pragma unroll
          for (int v = 0; v < VY; ++v) cen[s][v] = u[v];
        }
        const bool staged = t >= 0 && t < len;
        T* L = lds[s & 1];
        if (staged) {
#pragma unroll
          for (int v = 0; v < VY; ++v) L[(R + wv * VY + v) * LX + R + lane] = u[v];
#pragma unroll
          for (int h = 0; h < HR; ++h)
            if (hok[h]) L[hly[h] * LX + R + lane] = hrg[set][h];
#pragma unroll
          for (int m = 0; m < XH; ++m)
            if (xok[m]) L[xl[m]] = xrg[set][m];
        }
        if (i + PD < nsteps) fetch(i + PD, set);
        // z taps of plane t into outputs t-R .. t+R (slot of output t+d is (s+d) mod K)
#pragma unroll
        for (int v = 0; v < VY; ++v) {
          acc[(s + R) % K][v] = W.w[R] * u[v];
#pragma unroll
          for (int d = -R; d < R; ++d) {
            const T wd = d == 0 ? W.c0 : W.w[d < 0 ? -d : d];
            acc[(s + d + K) % K][v] += wd * u[v];
          }
        }
        if (staged) {
          __syncthreads();
#pragma unroll
          for (int v = 0; v < VY; ++v) {
            const T* row = L + (R + wv * VY + v) * LX + R + lane;
            T xy = T(0);
#pragma unroll
            for (int p = 1; p <= R; ++p) {
              const int a = v - p, b = v + p;
              const T ya = (a >= 0) ? u[a >= 0 ? a : 0] : row[-p * LX];
              const T yb = (b < VY) ? u[b < VY ? b : 0] : row[p * LX];
              xy += W.w[p] * ((row[-p] + row[p]) + (ya + yb));
            }
            acc[s % K][v] += xy;
          }
        }
        // output t - R is complete
        const int to = t - R;
        if (to >= 0) {
          const uint32_t so = plane_off(to) + own_row;
          const int z = zfirst + (down ? -to : to);
#pragma unroll
          for (int v = 0; v < VY; ++v) {
            const int gx = x0 + lane, gy = y0 + wv * VY + v;
            if (gy < g.ny && gx < g.nx) {
              const T c = NEEDC ? cen[NEEDC ? (s - R + K) % K : 0][v] : T(0);
              // Dirichlet nodes of an active domain store a zero stencil value (see k_stencil2)
              const T a = in_domain(g, gx, gy, z) ? acc[(s - R + K) % K][v] : T(0);
              o.storeb(nb, vl, so + v * rowb, gx, gy, z, c, a, red);
            }
          }
        }
      }
    }
  }
  if constexpr (NRED > 0) {
    block_reduce_store<NRED, NT>(red, o.parts_out + (long long)blockIdx.x * NRED);
  }
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
  if constexpr (NRED > 0) {
    block_reduce_store<NRED, NT>(red, o.parts_out + (long long)blockIdx.x * NRED);
  }
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
  static constexpr bool NEEDC = false;
  const T* x;
  T* y;
  double* parts_out;
  template <int NT>
  __device__ bool begin() { return true; }
  __device__ T load(long long i) const { return x[i]; }
  __device__ void store(long long i, int, int, int, T, T lap, double*) const { y[i] = lap; }
  __device__ T loadb(uint32_t nb, uint32_t vo, uint32_t so) const { return bld(x, nb, vo, so); }
  __device__ void storeb(uint32_t nb, uint32_t vo, uint32_t so, int, int, int, T, T lap, double*) const {
    bst(y, nb, vo, so, lap);
  }
};

// ----------------------------------------------------------------- ops: conjugate gradients
// Initial residual r = rhs - A x and, when p is not null, p = r; reduces r.r and rhs.rhs.
template <typename T>
struct CGInitOp {
  static constexpr int NRED = 2;
  static constexpr bool NEEDC = false;
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
  __device__ T loadb(uint32_t nb, uint32_t vo, uint32_t so) const { return bld(x, nb, vo, so); }
  __device__ void storeb(uint32_t nb, uint32_t vo, uint32_t so, int, int, int, T, T ax, double* red) const {
    const T b = bld(rhs, nb, vo, so);
    const T ri = b - ax;
    bst(r, nb, vo, so, ri);
    if (p) bst(p, nb, vo, so, ri);
    red[0] += (double)ri * (double)ri;
    red[1] += (double)b * (double)b;
  }
};

// Iteration k, first half: reduce r.r from the previous kernel's partials, stop
// at r.r <= tol^2 ||rhs||^2, else p_new = r + beta p_old formed on load, Ap = A p_new,
// reduce p.Ap.  Block 0 keeps the scalars in CGState (indexed by k parity so no
// block reads a value written by the same launch).  verdict(): 0 stop (a verdict of an
// earlier launch, a zero right-hand side or a non-finite r.r), 1 iterate, 2 converged
// in this launch.
template <typename T>
struct CGP1Op {
  static constexpr int NRED = 1;
  static constexpr bool NEEDC = true;
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
  __device__ int verdict() {
    const long long h = block_read_halt(st);
    if (h != 0 && h <= k) return 0;
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
        if (is_block0_thread0()) {
          st->done = 3; st->rr_last = rr; st->iter = 0; st->done_iter = 0;
          set_halt(st, 0);
        }
        return 0;
      }
    } else {
      thresh = ld_dev(&st->thresh);
    }
    const bool bad = !isfinite(rr);
    if (bad || rr <= thresh) {
      if (is_block0_thread0()) {
        st->done = bad ? 2 : 1;
        st->rr_last = rr;
        st->iter = k;
        st->done_iter = k;
        set_halt(st, k);
      }
      return bad ? 0 : 2;
    }
    beta = (k == 0) ? T(0) : (T)(rr / ld_dev(&st->rrh[(k - 1) & 1]));
    if (is_block0_thread0()) {
      st->rrh[k & 1] = rr;
      st->iter = k;
    }
    return 1;
  }
  template <int NT>
  __device__ bool begin() { return verdict<NT>() == 1; }
  __device__ T load(long long i) const { return r[i] + beta * pold[i]; }
  __device__ void store(long long i, int, int, int, T c, T ap, double* red) const {
    pnew[i] = c;
    Ap[i] = ap;
    red[0] += (double)c * (double)ap;
  }
  __device__ T loadb(uint32_t nb, uint32_t vo, uint32_t so) const {
    return bld(r, nb, vo, so) + beta * bld(pold, nb, vo, so);
  }
  __device__ void storeb(uint32_t nb, uint32_t vo, uint32_t so, int, int, int, T c, T ap, double* red) const {
    bst(pnew, nb, vo, so, c);
    bst(Ap, nb, vo, so, ap);
    red[0] += (double)c * (double)ap;
  }
};

// Iteration k, first half by linearity: the stencil is applied to r alone and
// A p_new = A r + beta A p_old (p_new = r + beta p_old), so the stencil input is
// one array and p and A p are read and written only at the node itself (in
// place).  Same scalars and verdicts as CGP1Op, whose prologue it shares.  A p is
// then a recurrence; its rounding is damped by beta < 1 and the solve's stopping
// test uses the residual r itself.
//
// XD (FP64): the update x += alpha p of iteration k - 1 is made here too, where p_old is
// loaded anyway, and the second half only updates r (10 array passes per iteration
// instead of 11); alpha of iteration k - 1 comes from CGState::xa.  The launch in which
// the solve converges has no p to form, so it only makes that last update of x (xonly,
// op.xpass); launches queued after it stop in their prologue.  The solves launch this op
// in FP64 only; the FP32 first half is CGP1LIOp, which leaves x to the second half (there
// the two extra node operands cost the first half more than they save the second).
template <typename T>
struct CGP1LOp : CGP1Op<T> {
  static constexpr bool NEEDC = true;
  static constexpr bool LATE_BEGIN = true;  // the stencil input r needs no scalar
  static constexpr bool XD = sizeof(T) == 8;
  static constexpr bool XPASS = XD;
  using CGP1Op<T>::r;
  using CGP1Op<T>::pnew;
  using CGP1Op<T>::Ap;
  using CGP1Op<T>::k;
  using CGP1Op<T>::beta;
  using CGP1Op<T>::st;
  T* x;             // XD: the iterate (updated with alpha of iteration k - 1)
  T xalpha;         // XD: alpha of iteration k - 1 (0 at k = 0)
  bool xonly;       // XD: converged in this launch, only x += alpha p remains
  template <int NT>
  __device__ bool begin() {
    const int v = this->template verdict<NT>();
    if constexpr (!XD) {
      return v == 1;
    } else {
      if (v == 0 || (v == 2 && k == 0)) return false;
      xalpha = k == 0 ? T(0) : (T)ld_dev(&st->xa[(k - 1) & 1]);
      xonly = v == 2;
      return true;
    }
  }
  // x += alpha p over the interior nodes, rows spread over all waves of the launch
  __device__ void xpass(const Geom& g) const {
    const int nw = gridDim.x * (blockDim.x >> 6);
    const int nrows = g.ny * g.nz;
    for (int row = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); row < nrows; row += nw) {
      const int j = row % g.ny, kz = row / g.ny;
      const long long rb = g.base + (long long)kz * g.plane + (long long)j * g.px;
      for (int i = threadIdx.x & 63; i < g.nx; i += 64) x[rb + i] = x[rb + i] + xalpha * pnew[rb + i];
    }
  }
  __device__ T load(long long i) const { return r[i]; }
  __device__ void store(long long i, int, int, int, T c, T ar, double* red) const {
    const T po = pnew[i];
    const T pn = k == 0 ? c : c + beta * po;
    const T apn = k == 0 ? ar : ar + beta * Ap[i];
    if constexpr (XD) {
      if (k != 0) x[i] = x[i] + xalpha * po;
    }
    pnew[i] = pn;
    Ap[i] = apn;
    red[0] += (double)pn * (double)apn;
  }
  __device__ T loadb(uint32_t nb, uint32_t vo, uint32_t so) const { return bld(r, nb, vo, so); }
  __device__ void storeb(uint32_t nb, uint32_t vo, uint32_t so, int, int, int, T c, T ar, double* red) const {
    T pn = c, apn = ar;
    if (k != 0) {
      const T po = bld((const T*)pnew, nb, vo, so);
      pn = c + beta * po;
      apn = ar + beta * bld((const T*)Ap, nb, vo, so);
      if constexpr (XD) bst(x, nb, vo, so, bld((const T*)x, nb, vo, so) + xalpha * po);
    }
    bst(pnew, nb, vo, so, pn);
    bst(Ap, nb, vo, so, apn);
    red[0] += (double)pn * (double)apn;
  }
  // the same update with p_old, (A p)_old (and x) loaded a plane ahead (iteration 0 has
  // no p_old: beta = 0 and the loaded values, whatever they hold, are not used; x is
  // stored back unchanged)
  static constexpr int NPRE = XD ? 3 : 2;
  __device__ void prefetch(uint32_t nb, uint32_t vo, uint32_t so, T* pre) const {
    pre[0] = bld((const T*)pnew, nb, vo, so);
    pre[1] = bld((const T*)Ap, nb, vo, so);
    if constexpr (XD) pre[2] = bld((const T*)x, nb, vo, so);
  }
  __device__ void storep(uint32_t nb, uint32_t vo, uint32_t so, T c, T ar, const T* pre, double* red) const {
    const T pn = k == 0 ? c : c + beta * pre[0];
    const T apn = k == 0 ? ar : ar + beta * pre[1];
    bst(pnew, nb, vo, so, pn);
    bst(Ap, nb, vo, so, apn);
    if constexpr (XD) bst(x, nb, vo, so, k == 0 ? pre[2] : pre[2] + xalpha * pre[0]);
    red[0] += (double)pn * (double)apn;
  }
};

// The FP32 first half of schedule 1 (as CGP1LOp<float>) with p and A p interleaved in one
// array, pa[2i] = p_i and pa[2i + 1] = (A p)_i: each node operand pair is one 8-byte
// load and one 8-byte store instead of two 4-byte ones.  The pair array must stay below
// 4 GiB (the caller checks).
struct CGP1LIOp : CGP1Op<float> {
  static constexpr bool NEEDC = true;
  static constexpr bool LATE_BEGIN = true;  // the stencil input r needs no scalar
  float* pa;
  __device__ float load(long long i) const { return r[i]; }
  __device__ void store(long long i, int, int, int, float c, float ar, double* red) const {
    const float pn = k == 0 ? c : c + beta * pa[2 * i];
    const float apn = k == 0 ? ar : ar + beta * pa[2 * i + 1];
    pa[2 * i] = pn;
    pa[2 * i + 1] = apn;
    red[0] += (double)pn * (double)apn;
  }
  __device__ float loadb(uint32_t nb, uint32_t vo, uint32_t so) const { return bld(r, nb, vo, so); }
  __device__ void storeb(uint32_t nb, uint32_t vo, uint32_t so, int, int, int, float c, float ar,
                         double* red) const {
    PApair v{c, ar};
    if (k != 0) {
      const PApair o = bldpair(pa, 2 * nb, 2 * vo, 2 * so);
      v = PApair{c + beta * o.p, ar + beta * o.ap};
    }
    bstpair(pa, 2 * nb, 2 * vo, 2 * so, v);
    red[0] += (double)v.p * (double)v.ap;
  }
  // the pair loaded a plane ahead (iteration 0: not used)
  static constexpr int NPRE = 2;
  __device__ void prefetch(uint32_t nb, uint32_t vo, uint32_t so, float* pre) const {
    const PApair o = bldpair(pa, 2 * nb, 2 * vo, 2 * so);
    pre[0] = o.p;
    pre[1] = o.ap;
  }
  __device__ void storep(uint32_t nb, uint32_t vo, uint32_t so, float c, float ar, const float* pre,
                         double* red) const {
    const float pn = k == 0 ? c : c + beta * pre[0];
    const float apn = k == 0 ? ar : ar + beta * pre[1];
    bstpair(pa, 2 * nb, 2 * vo, 2 * so, PApair{pn, apn});
    red[0] += (double)pn * (double)apn;
  }
};

// Iteration k, second half: alpha = r.r / p.Ap; x += alpha p (x not null; else the
// first half of iteration k + 1 makes it, with alpha kept in CGState::xa);
// r -= alpha Ap; reduce r.r.
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
  int paired;  // 1: p points to the interleaved (p, A p) pairs and Ap is unused (FP32)
  template <int NT>
  __device__ bool begin() {
    if (block_read_done(st)) return false;
    const double pap = block_sum_parts<NT>(parts_in, nparts_in, 1, 0);
    const double a = ld_dev(&st->rrh[k & 1]) / pap;
    if (!isfinite(a) || pap <= 0.0) {
      if (is_block0_thread0()) {
        st->done = 2; st->iter = k; st->done_iter = k;
        set_halt(st, k);
      }
      return false;
    }
    alpha = (T)a;
    if (is_block0_thread0()) st->xa[k & 1] = a;
    return true;
  }
  __device__ void apply(long long i, int, int, int, double* red) const {
    if (x) x[i] += alpha * p[i];
    const T ri = r[i] - alpha * Ap[i];
    r[i] = ri;
    red[0] += (double)ri * (double)ri;
  }
};

// Second half of a CG iteration (CGP2Op) with one grid row per wave: each lane
// issues the loads of all its nodes of the row (up to 4 x 64 per pass) before any
// store, so a row costs one memory latency.  The first row's loads go out before
// the prologue that reduces p.Ap (they do not depend on alpha), so the two
// latencies overlap.  XU = false: x is left to the next first half (op.x null), and
// only r and A p are read.  PI: p and A p come interleaved (op.paired, FP32).
template <typename T, int NT, bool XU, bool PI = false>
__global__ void __launch_bounds__(NT) k_cg_update(Geom g, CGP2Op<T> op) {
  static_assert(!PI || (XU && sizeof(T) == 4), "interleaved pairs: FP32 with x updated here");
  CGP2Op<T> o = op;
  double red[1] = {0.0};
  const int lane = threadIdx.x & 63;
  const int nwaves = gridDim.x * (NT / 64);
  const int nrows = g.ny * g.nz;
  T* __restrict__ x = o.x;
  T* __restrict__ r = o.r;
  const T* __restrict__ p = o.p;
  const T* __restrict__ Ap = o.Ap;
  T xv[4], pv[4], rv[4], av[4];
  auto load = [&](long long rb, int i0) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int i = i0 + lane + 64 * u;
      if (i < g.nx) {
        if constexpr (PI) {
          const PApair o = reinterpret_cast<const PApair*>(p)[rb + i];
          pv[u] = o.p;
          av[u] = o.ap;
          xv[u] = x[rb + i];
        } else {
          if constexpr (XU) {
            xv[u] = x[rb + i];
            pv[u] = p[rb + i];
          }
          av[u] = Ap[rb + i];
        }
        rv[u] = r[rb + i];
      }
    }
  };
  auto rowbase = [&](int row) {
    const int j = row % g.ny, k = row / g.ny;
    return g.base + (long long)k * g.plane + (long long)j * g.px;
  };
  const int row0 = blockIdx.x * (NT / 64) + (threadIdx.x >> 6);
  if (row0 < nrows) load(rowbase(row0), 0);
  if (!o.template begin<NT>()) return;
  const T alpha = o.alpha;
  for (int row = row0; row < nrows; row += nwaves) {
    const long long rb = rowbase(row);
    for (int i0 = 0; i0 < g.nx; i0 += 4 * 64) {
      if (row != row0 || i0 != 0) load(rb, i0);
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int i = i0 + lane + 64 * u;
        if (i < g.nx) {
          if constexpr (XU) x[rb + i] = xv[u] + alpha * pv[u];
          const T ri = rv[u] - alpha * av[u];
          r[rb + i] = ri;
          red[0] += (double)ri * (double)ri;
        }
      }
    }
  }
  block_reduce_store<1, NT>(red, o.parts_out + blockIdx.x);
}

// ----------------------------------------------------------------- ops: CG with one reduction per iteration
// With w = A r and s = A p kept as vectors (Chronopoulos and Gear), the two inner
// products an iteration needs, gamma = r.r and delta = w.r, come out of the same pass,
// and p.Ap = delta - beta gamma / alpha_prev (A-conjugacy of the previous p and the
// orthogonality of successive residuals), so one launch and one reduction make an
// iteration.

// Sums of components 0 and 1 of n two-component block partials, in a fixed order
// (every thread of the block returns the same pair); both components of a partial
// come in one load.
template <int NT>
__device__ inline double2 block_sum_parts2(const double* parts, int n) {
  __shared__ double sh[2][NT / 64];
  double s0 = 0.0, s1 = 0.0;
  for (int b0 = threadIdx.x; b0 < n; b0 += 8 * NT) {
    double2 v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int b = b0 + u * NT;
      v[u] = b < n ? make_double2(ld_dev(parts + 2 * b), ld_dev(parts + 2 * b + 1)) : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      s0 += v[u].x;
      s1 += v[u].y;
    }
  }
  s0 = wave_sum(s0);
  s1 = wave_sum(s1);
  if ((threadIdx.x & 63) == 0) {
    sh[0][threadIdx.x >> 6] = s0;
    sh[1][threadIdx.x >> 6] = s1;
  }
  __syncthreads();
  double t0 = 0.0, t1 = 0.0;
#pragma unroll
  for (int w = 0; w < NT / 64; ++w) {
    t0 += sh[0][w];
    t1 += sh[1][w];
  }
  __syncthreads();
  return make_double2(t0, t1);
}

// Prologue of a one-reduction iteration k: gamma = r.r and delta = w.r from the
// previous pass; stop at gamma <= tol^2 ||rhs||^2 (or, with last set, only record
// gamma: the iteration cap was reached); else beta = gamma / gamma_prev and alpha =
// gamma / (delta - beta gamma / alpha_prev).  Block 0 keeps gamma and alpha in CGState
// indexed by k parity (no block reads a value written by the same launch).
template <int NT>
__device__ inline bool cg1r_prologue(CGState* st, const double* parts_in, int nparts_in, int k, int last, double& a,
                                     double& b) {
  if (block_read_done(st)) return false;
  const double2 gd = block_sum_parts2<NT>(parts_in, nparts_in);
  const double gam = gd.x, del = gd.y;
  const double thresh = ld_dev(&st->thresh);
  if (!isfinite(gam) || !isfinite(del) || gam <= thresh || last) {
    if (is_block0_thread0()) {
      if (!isfinite(gam) || !isfinite(del)) st->done = 2;
      else if (gam <= thresh) st->done = 1;
      st->rr_last = gam;
      st->rrh[k & 1] = gam;
      st->iter = k;
      st->done_iter = k;
    }
    return false;
  }
  b = k == 0 ? 0.0 : gam / ld_dev(&st->rrh[(k - 1) & 1]);
  const double den = k == 0 ? del : del - b * gam / ld_dev(&st->ah[(k - 1) & 1]);
  a = gam / den;
  if (!(den > 0.0) || !isfinite(a)) {
    // p.Ap <= 0 from finite scalars: the recurrences have drifted to rounding level
    // (verdict 4, the caller restarts from the true residual); else non-finite (2)
    if (is_block0_thread0()) {
      st->done = (isfinite(den) && den <= 0.0) ? 4 : 2;
      st->rr_last = gam;
      st->rrh[k & 1] = gam;
      st->iter = k;
      st->done_iter = k;
    }
    return false;
  }
  if (is_block0_thread0()) {
    st->rrh[k & 1] = gam;
    st->ah[k & 1] = a;
    st->iter = k;
  }
  return true;
}

// Start of the recurrences: w = A r for the residual r of the initial guess, p = s = 0,
// reducing r.r and w.r.  The prologue takes ||rhs||^2 from the partials of the pass
// that formed r (component 1 of 2) and fixes the stopping threshold.
template <typename T>
struct CGWInitOp {
  static constexpr int NRED = 2;
  static constexpr bool NEEDC = true;
  static constexpr bool LATE_BEGIN = true;  // the stencil input r needs no scalar
  const T* r;
  T* w;
  T* s;
  T* p;
  T* z;  // pipelined form only (else null): z = A s starts at 0 too
  CGState* st;
  const double* parts_in;
  int nparts_in;
  double tol2;
  double* parts_out;
  template <int NT>
  __device__ bool begin() {
    const double rhs2 = block_sum_parts<NT>(parts_in, nparts_in, 2, 1);
    if (is_block0_thread0()) {
      st->rhs2 = rhs2;
      st->thresh = tol2 * rhs2;
    }
    if (rhs2 == 0.0) {
      if (is_block0_thread0()) { st->done = 3; st->rr_last = 0.0; st->iter = 0; st->done_iter = 0; }
      return false;
    }
    return true;
  }
  __device__ T load(long long i) const { return r[i]; }
  __device__ void store(long long i, int, int, int, T c, T ar, double* red) const {
    w[i] = ar;
    s[i] = T(0);
    p[i] = T(0);
    if (z) z[i] = T(0);
    red[0] += (double)c * (double)c;
    red[1] += (double)ar * (double)c;
  }
  __device__ T loadb(uint32_t nb, uint32_t vo, uint32_t so) const { return bld(r, nb, vo, so); }
  __device__ void storeb(uint32_t nb, uint32_t vo, uint32_t so, int, int, int, T c, T ar, double* red) const {
    bst(w, nb, vo, so, ar);
    bst(s, nb, vo, so, T(0));
    bst(p, nb, vo, so, T(0));
    if (z) bst(z, nb, vo, so, T(0));
    red[0] += (double)c * (double)c;
    red[1] += (double)ar * (double)c;
  }
};

// Iterate k in the pipelined form (Ghysels and Vanroose): z = A s is kept as a vector
// too, so the stencil is applied to w, an array already stored, and needs no scalar
// of this iteration -- its loads go out before the prologue's reduction:
//   m = A w,  z = m + beta z,  s = w + beta s,  p = r + beta p,  x += alpha p,
//   r -= alpha s,  w' = w - alpha z,  reducing r.r and w'.r.
// w is read at the stencil's neighbours, so it alternates between two arrays; the
// others are touched only at the node itself, in place.  w and r are recurrences here
// (rounding drifts them from A r and rhs - A x; the refined solve recomputes the
// residual in FP64).
template <typename T>
struct CGPipeOp {
  static constexpr int NRED = 2;
  static constexpr bool NEEDC = true;
  static constexpr bool LATE_BEGIN = true;  // the stencil input w needs no scalar
  const T* w;
  T* wn;
  T* r;
  T* s;
  T* z;
  T* p;
  T* x;
  CGState* st;
  const double* parts_in;
  int nparts_in, k, last;
  double* parts_out;
  T alpha, beta;
  template <int NT>
  __device__ bool begin() {
    double a, b;
    if (!cg1r_prologue<NT>(st, parts_in, nparts_in, k, last, a, b)) return false;
    alpha = (T)a;
    beta = (T)b;
    return true;
  }
  __device__ T load(long long i) const { return w[i]; }
  __device__ void store(long long i, int, int, int, T c, T m, double* red) const {
    const T zi = m + beta * z[i];
    const T si = c + beta * s[i];
    const T pi = r[i] + beta * p[i];
    const T ri = r[i] - alpha * si;
    const T wi = c - alpha * zi;
    z[i] = zi;
    s[i] = si;
    p[i] = pi;
    x[i] += alpha * pi;
    r[i] = ri;
    wn[i] = wi;
    red[0] += (double)ri * (double)ri;
    red[1] += (double)wi * (double)ri;
  }
  __device__ T loadb(uint32_t nb, uint32_t vo, uint32_t so) const { return bld(w, nb, vo, so); }
  __device__ void storeb(uint32_t nb, uint32_t vo, uint32_t so, int, int, int, T c, T m, double* red) const {
    const T zo = bld((const T*)z, nb, vo, so), so_ = bld((const T*)s, nb, vo, so);
    const T ro = bld((const T*)r, nb, vo, so), po = bld((const T*)p, nb, vo, so);
    const T xo = bld((const T*)x, nb, vo, so);
    const T zi = m + beta * zo;
    const T si = c + beta * so_;
    const T pi = ro + beta * po;
    const T ri = ro - alpha * si;
    const T wi = c - alpha * zi;
    bst(z, nb, vo, so, zi);
    bst(s, nb, vo, so, si);
    bst(p, nb, vo, so, pi);
    bst(x, nb, vo, so, xo + alpha * pi);
    bst(r, nb, vo, so, ri);
    bst(wn, nb, vo, so, wi);
    red[0] += (double)ri * (double)ri;
    red[1] += (double)wi * (double)ri;
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
  double a = 1.0;  // v = a u_start + t d (a = cos theta on the Lagrange method's great circle)
  template <int NT>
  __device__ bool begin() { return true; }
  __device__ void apply(long long i, int ii, int jj, int kk, double* red) const {
    const double vi = a * us[i] + t * d[i];
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
    const double dn = beta != 0.0 ? s[i] + beta * d[i] : s[i];  // a restart never reads the old d
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
  double mv[kUpdRed];  // this thread's copy of the moments
  const int* dom = nullptr;  // active domain rows (see Geom::dom): zero right-hand side at Dirichlet nodes
  template <int NT>
  __device__ bool begin() {
    if (mom)
      for (int q = 0; q < kUpdRed; ++q) mv[q] = ld_dev(mom + q);
    return true;
  }
  __device__ void apply(long long i, int ii, int jj, int kk, double*) const {
    if (dom) {
      const long long r = 2ll * ((long long)kk * ny + jj);
      if (ii < dom[r] || ii > dom[r + 1]) {
        rhs[i] = T(0);
        return;
      }
    }
    double val = v[i] * v[i] + b[i];
    if (mom && (ii < R || jj < R || kk < R || ii >= nx - R || jj >= ny - R || kk >= nz - R)) {
      double dx, dy, dz;
      f.rel(ii, jj, kk, dx, dy, dz);
      const double h = f.h;
      double add = 0.0;
      for (int p = 1; p <= R; ++p) {
        if (ii - p < 0) add += W.w[p] * phi_multipole(mv, dx - p * h, dy, dz);
        if (ii + p >= nx) add += W.w[p] * phi_multipole(mv, dx + p * h, dy, dz);
        if (jj - p < 0) add += W.w[p] * phi_multipole(mv, dx, dy - p * h, dz);
        if (jj + p >= ny) add += W.w[p] * phi_multipole(mv, dx, dy + p * h, dz);
        if (kk - p < 0) add += W.w[p] * phi_multipole(mv, dx, dy, dz - p * h);
        if (kk + p >= nz) add += W.w[p] * phi_multipole(mv, dx, dy, dz + p * h);
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
    shift = -eta + ld_dev(Cptr) * inv_mu;
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
    red[G_UG] += u * g;
  }
};

}  // namespace alofdft
