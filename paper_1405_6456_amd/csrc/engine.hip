// Host engine and C ABI of the MI355X AL orbital-free DFT solve.
//
// The host owns control flow only: the augmented Lagrangian / penalty outer
// loop (Sec. 3, Algorithm AugLag; Sec. 5.3.2), the nonlinear CG line-search
// logic (Sec. 4) and convergence tests.  Every grid-sized step runs in the gfx950
// kernels of kernels.hip; the Poisson CG keeps its scalars on the device and the
// host only polls its done flag every cg_check_every iterations.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <condition_variable>
#include <deque>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/alofdft.h"
#include "common.h"
#include "kernels_misc.h"
#include "launch.h"

using namespace alofdft;

struct alofdft_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;
  std::atomic<int> cancel{0};  // set by alofdft_cancel; the running solve stops at its next check
  std::map<std::string, std::pair<void*, size_t>> bufs;
  double* pin = nullptr;  // pinned host scalars
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  int variant = -1;       // stencil tile variant (-1: chosen per grid)
  int target_blocks = 0;  // 0: one round of resident workgroups
  int inner_tol_exp = 6;  // FP32 inner CG reduces the residual by 10^-inner_tol_exp
  int progress = 0;       // ALOFDFT_PROGRESS set: one stderr line per 100 NLCG steps and per AL step
  int cg_schedule = -1;   // CG launches: 0 stencil of p + update, 1 stencil of r (linearity) + update,
                          // 2 pipelined (one launch, one reduction); -1 automatic (cg_schedule_for)
  // geometry each padded work array was last zeroed for (its halo is zero only then)
  std::map<std::string, std::string> geom_key;
  // sampled event timing of the CG stencil kernel (index 0: FP64, 1: FP32)
  int prof_every = 0;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> prof_pool;
  long long prof_count[2] = {0, 0};
  double prof_ms[2] = {0.0, 0.0};      // kernel time of the sampled iterations (all their launches)
  double prof_ms_first[2] = {0.0, 0.0};   // of their first launch (the stencil)
  double prof_ms_second[2] = {0.0, 0.0};  // of their second launch (x and r update; schedules 0, 1)
  long long prof_points[2] = {0, 0};
  int prof_sched[2] = {-1, -1};  // CG schedule of the timed launches
  // opt-in trace of every Poisson solve (ALOFDFT_TRACE=path at creation): one line per
  // solve with the request's tag, its sequence number, the CG counts and verdicts, and
  // exact hashes of the right-hand side and of phi before and after
  bool trace = false;       // ALOFDFT_TRACE=path: counts, verdicts and the host sums of each evaluation
  bool trace_hash = false;  // ALOFDFT_TRACE_HASH set as well: exact hashes of rhs and phi (syncs per solve)
  uint64_t trace_tag = 0;
  long long trace_seq = 0;
};

namespace {

// ----------------------------------------------------------------- errors
struct Fail {
  int code;
};

void set_err(alofdft_ctx* c, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (c) c->err = buf;
}

#define HIPC(c, x)                                                              \
  do {                                                                          \
    hipError_t e_ = (x);                                                        \
    if (e_ != hipSuccess) {                                                     \
      set_err(c, "%s failed: %s (%s:%d)", #x, hipGetErrorString(e_), __FILE__, __LINE__); \
      throw Fail{e_ == hipErrorOutOfMemory ? ALOFDFT_OUT_OF_MEMORY : ALOFDFT_DEVICE_ERROR}; \
    }                                                                           \
  } while (0)

#define CHECK_LAUNCH(c) HIPC(c, hipGetLastError())

void require(alofdft_ctx* c, bool ok, const char* msg) {
  if (!ok) {
    set_err(c, "%s", msg);
    throw Fail{ALOFDFT_INVALID_ARGUMENT};
  }
}

// A pending cancellation ends the running call (checked at every host read of a CG
// solve's state and at every nonlinear CG step); the flag is consumed.
void check_cancel(alofdft_ctx* c) {
  if (c && c->cancel.exchange(0)) {
    set_err(c, "cancelled");
    throw Fail{ALOFDFT_CANCELLED};
  }
}

// ----------------------------------------------------------------- buffers
void zero_bytes(alofdft_ctx* c, void* p, size_t bytes);

void* buf(alofdft_ctx* c, const std::string& name, size_t bytes) {
  auto it = c->bufs.find(name);
  if (it != c->bufs.end()) {
    if (it->second.second >= bytes) return it->second.first;
    HIPC(c, hipFree(it->second.first));
    c->bufs.erase(it);
  }
  void* p = nullptr;
  bytes = (bytes + 7) / 8 * 8;
  HIPC(c, hipMalloc(&p, bytes));
  zero_bytes(c, p, bytes);
  c->bufs[name] = {p, bytes};
  return p;
}
template <typename T>
T* bufT(alofdft_ctx* c, const std::string& name, size_t count) {
  return (T*)buf(c, name, count * sizeof(T));
}

void sync(alofdft_ctx* c) { HIPC(c, hipStreamSynchronize(c->stream)); }

// ----------------------------------------------------------------- layout and weights
int roundup(int a, int b) { return (a + b - 1) / b * b; }

Geom make_geom(const int n[3], int R) {
  Geom g;
  g.nx = n[0];
  g.ny = n[1];
  g.nz = n[2];
  g.R = R;
  const int ox = 16;  // >= R, keeps interior rows 64-byte aligned for float and double
  g.px = roundup(ox + roundup(n[0], 64) + R, 16);
  g.py = R + roundup(n[1], 32) + R;
  g.pz = n[2] + 2 * R;
  g.plane = (long long)g.px * g.py;
  g.base = (long long)R * g.plane + (long long)R * g.px + ox;
  g.total = g.plane * g.pz;
  g.dom = nullptr;
  return g;
}

// Laplacian weights of Eq. FD:Laplacian: w_0 = -(1/h^2) sum_q 1/q^2,
// w_p = 2(-1)^(p+1)/(h^2 p^2) (n!)^2/((n-p)!(n+p)!).
void lap_weights(int n, double h, double* w) {
  double s = 0.0;
  for (int q = 1; q <= n; ++q) s += 1.0 / (double(q) * q);
  w[0] = -s / (h * h);
  double ratio = 1.0;
  for (int p = 1; p <= n; ++p) {
    ratio *= double(n - p + 1) / double(n + p);
    w[p] = ((p & 1) ? 2.0 : -2.0) / (h * h * p * p) * ratio;
  }
}
// Gradient weights of Sec. 4: w~_p = (-1)^(p+1)/(h p) (n!)^2/((n-p)!(n+p)!).
void grad_weights(int n, double h, double* w) {
  w[0] = 0.0;
  double ratio = 1.0;
  for (int p = 1; p <= n; ++p) {
    ratio *= double(n - p + 1) / double(n + p);
    w[p] = ((p & 1) ? 1.0 : -1.0) / (h * p) * ratio;
  }
}
template <typename T>
StencilW<T> stencil_weights(int n, double h, double scale) {
  double w[kMaxRadius + 1];
  lap_weights(n, h, w);
  StencilW<T> W;
  W.c0 = (T)(6.0 * w[0] * scale);
  for (int p = 0; p <= kMaxRadius; ++p) W.w[p] = (T)(p <= n && p > 0 ? w[p] * scale : 0.0);
  return W;
}

// ----------------------------------------------------------------- launches
int pw_blocks(const Geom& g) {
  const int rows = g.ny * g.nz;
  const int waves_per_block = kPointwiseThreads / 64;
  return std::max(1, std::min(kPointwiseBlocks, (rows + waves_per_block - 1) / waves_per_block));
}

template <class Op>
int launch_pw(alofdft_ctx* c, const Geom& g, const Op& op) {
  const int nb = pw_blocks(g);
  hipLaunchKernelGGL((k_pointwise<Op, kPointwiseThreads>), dim3(nb), dim3(kPointwiseThreads), 0, c->stream, g, op);
  CHECK_LAUNCH(c);
  return nb;
}

// Second half of a CG iteration: one row per wave, at most kPointwiseBlocks blocks
// (op.x null: r only, x is updated by the next first half).
template <typename T>
int launch_cg_update(alofdft_ctx* c, const Geom& g, const CGP2Op<T>& op, hipEvent_t ev_start = nullptr,
                     hipEvent_t ev_stop = nullptr) {
  const int rows = g.ny * g.nz;
  const int nb = std::max(1, std::min(kPointwiseBlocks, (rows + 3) / 4));
  auto kern = op.x ? k_cg_update<T, 256, true> : k_cg_update<T, 256, false>;
  if constexpr (sizeof(T) == 4) {
    if (op.paired) kern = k_cg_update<T, 256, true, true>;
  }
  if (ev_start)  // the runtime stamps the events with the kernel's own start and end
    hipExtLaunchKernelGGL(kern, dim3(nb), dim3(256), 0, c->stream, ev_start, ev_stop, 0, g, op);
  else
    hipLaunchKernelGGL(kern, dim3(nb), dim3(256), 0, c->stream, g, op);
  CHECK_LAUNCH(c);
  return nb;
}

template <typename T, class Op>
int launch_stencil(alofdft_ctx* c, const Geom& g, const StencilW<T>& W, const Op& op, hipEvent_t ev_start = nullptr,
                   hipEvent_t ev_stop = nullptr) {
  const LaunchCfg lc{c->stream, c->variant, c->target_blocks, ev_start, ev_stop};
  int nb = 0;
  hipError_t e = hipErrorInvalidValue;
  switch (g.R) {
    case 1: e = launch_stencil_r<1>(lc, g, W, op, &nb); break;
    case 2: e = launch_stencil_r<2>(lc, g, W, op, &nb); break;
    case 3: e = launch_stencil_r<3>(lc, g, W, op, &nb); break;
    case 4: e = launch_stencil_r<4>(lc, g, W, op, &nb); break;
    case 5: e = launch_stencil_r<5>(lc, g, W, op, &nb); break;
    case 6: e = launch_stencil_r<6>(lc, g, W, op, &nb); break;
    case 7: e = launch_stencil_r<7>(lc, g, W, op, &nb); break;
    case 8: e = launch_stencil_r<8>(lc, g, W, op, &nb); break;
    default:
      set_err(c, "fd_half_width %d out of range", g.R);
      throw Fail{ALOFDFT_INVALID_ARGUMENT};
  }
  HIPC(c, e);
  return nb;
}

void finalize(alofdft_ctx* c, const double* parts, int nparts, int nred, double scale, double* out) {
  hipLaunchKernelGGL((k_finalize<256>), dim3(1), dim3(256), 0, c->stream, parts, nparts, nred, scale, out);
  CHECK_LAUNCH(c);
}

template <typename T>
void fill(alofdft_ctx* c, T* a, long long n, T v) {
  const int nb = (int)std::min<long long>(2048, (n + 255) / 256);
  hipLaunchKernelGGL((k_fill<T>), dim3(std::max(nb, 1)), dim3(256), 0, c->stream, a, n, v);
  CHECK_LAUNCH(c);
}

// Device memory is cleared by a fill kernel on the context stream rather than by
// hipMemsetAsync, so every clearing is an ordinary kernel of the stream (also for a caller
// that captures the stream into a graph).  Bytes: a multiple of 8.
void zero_bytes(alofdft_ctx* c, void* p, size_t bytes) {
  fill<unsigned long long>(c, (unsigned long long*)p, (long long)(bytes / 8), 0ull);
}
// A padded work array whose halo and padding are zero for geometry g: zeroed
// whenever it is first used with a geometry other than the last one.
template <typename T>
T* gridbuf(alofdft_ctx* c, const std::string& name, const Geom& g) {
  T* p = bufT<T>(c, name, g.total);
  const std::string key = std::to_string(g.nx) + "," + std::to_string(g.ny) + "," + std::to_string(g.nz) + "," +
                          std::to_string(g.R) + "," + std::to_string((unsigned long long)(uintptr_t)p);
  auto it = c->geom_key.find(name);
  if (it == c->geom_key.end() || it->second != key) {
    fill<T>(c, p, g.total, T(0));
    c->geom_key[name] = key;
  }
  return p;
}

template <typename TS, typename TD>
void pack(alofdft_ctx* c, const Geom& g, const TS* dense, TD* padded, int absval = 0) {
  hipLaunchKernelGGL((k_pack<TS, TD>), dim3(2048), dim3(256), 0, c->stream, g, dense, padded, absval);
  CHECK_LAUNCH(c);
}
template <typename TS, typename TD>
void unpack(alofdft_ctx* c, const Geom& g, const TS* padded, TD* dense, int absval = 0) {
  hipLaunchKernelGGL((k_unpack<TS, TD>), dim3(2048), dim3(256), 0, c->stream, g, padded, dense, absval);
  CHECK_LAUNCH(c);
}

// ----------------------------------------------------------------- pointwise helpers of the refined solve
struct ToFloatOp {  // r32 = (float) r64; p32 = r32; x32 = 0; reduce r32.r32 twice (rr, "rhs2")
  static constexpr int NRED = 2;
  const double* r64;
  float* r32;
  float* p32;
  float* x32;
  double* parts_out;
  template <int NT>
  __device__ bool begin() { return true; }
  __device__ void apply(long long i, int, int, int, double* red) const {
    const float r = (float)r64[i];
    r32[i] = r;
    p32[i] = r;
    x32[i] = 0.0f;
    const double rd = r;
    red[0] += rd * rd;
    red[1] += rd * rd;
  }
};
struct AddFloatOp {  // x64 += (double) x32
  static constexpr int NRED = 0;
  double* x64;
  const float* x32;
  double* parts_out;
  template <int NT>
  __device__ bool begin() { return true; }
  __device__ void apply(long long i, int, int, int, double*) const { x64[i] += (double)x32[i]; }
};

// out = c0 a + c1 b + c2 c over the interior (b, c nullable when their coefficient is 0).
struct CombineOp {
  static constexpr int NRED = 0;
  double* out;
  const double* a;
  const double* b;
  const double* c;
  double c0, c1, c2;
  double* parts_out;
  template <int NT>
  __device__ bool begin() { return true; }
  __device__ void apply(long long i, int, int, int, double*) const {
    double v = c0 * a[i];
    if (b) v += c1 * b[i];
    if (c) v += c2 * c[i];
    out[i] = v;
  }
};

// ----------------------------------------------------------------- Poisson CG
struct CGResult {
  long long iters = 0;
  double relres = 0.0;
  int done = 0;
  int extra_mv = 0;  // stencil applications beyond one per iteration and the initial residual
  int late = 0;      // a launch after the verdict updated the iterate (the final iteration != done_iter)
};

// Largest grid (nodes) on which the automatic schedule runs FP64 solves pipelined: the
// fused launch saves a launch and a reduction per iteration, which pays while the
// iteration is latency bound; above it the extra bytes (12 arrays per node against
// 11 for the two launches) cost more.
constexpr long long kPipeMaxNodes = 1500000;

// CG schedule of a solve: the context's choice, the automatic one for -1; FP32 solves
// never run pipelined (its recurrences for w and r lose accuracy near 1e-4 in FP32).
int cg_schedule_for(const alofdft_ctx* c, const Geom& g, bool fp64) {
  int s = c->cg_schedule;
  if (s < 0) s = (fp64 && (long long)g.nx * g.ny * g.nz <= kPipeMaxNodes) ? 2 : 1;
  if (s == 2 && !fp64) s = 1;
  return s;
}

// Host polls of a CG solve's state (each a copy and a stream synchronisation): first
// after `every` launches, then timed by the residual reduction observed between polls so
// that the poll lands just past the predicted last iteration (at most `every` launches
// ahead) -- launches queued after convergence only run their prologue, but cost a launch.
struct PollPlan {
  long long every, next, k_last = 0;
  double rr_last = -1.0;
  PollPlan(long long e, long long first) : every(e), next(std::max(1LL, std::min(e, first))) {}
  bool due(long long k) const { return k + 1 >= next; }
  void update(long long k, double rr, double thresh) {
    long long step = every;
    if (rr_last > 0 && rr > thresh && rr < rr_last && thresh > 0) {
      const double per_it = std::log(rr / rr_last) / (double)(k + 1 - k_last);  // < 0
      const double need = std::log(thresh / rr) / per_it;                          // > 0
      if (std::isfinite(need)) step = std::max(2LL, std::min(every, (long long)std::ceil(need) + 1));
    }
    rr_last = rr;
    k_last = k + 1;
    next = k + 1 + step;
  }
};

// Default of the most CG launches between two host reads of a solve's state.
constexpr int kCheckEvery = 32;

// Iterations without r.r halving after which a rounding-limited (FP32) solve stops:
// CG on the Laplacian can plateau for a number of iterations that grows with the grid's
// longest side, so the window does too (256 up to 128 nodes per side).
long long stall_window(const Geom& g) {
  return std::max(256LL, 2LL * std::max(g.nx, std::max(g.ny, g.nz)));
}

// Whether CG launch k carries timing events: every prof_every-th launch, offset from
// the host's polls of the solve state (every check_every launches), after which the
// device has drained and the next launch starts cold.
bool sampled(const alofdft_ctx* c, long long k) {
  if (c->prof_every <= 0) return false;
  const long long off = c->prof_every > 8 ? 5 : 0;
  return k % c->prof_every == off;
}

// Kernel-stamped event pair number `used` of the context's pool (created on demand).
// The events only time the kernel they stamp: without the system-scope fence their
// recording neither writes back nor invalidates the caches, which would lengthen the
// stamped kernel and slow the next.
std::pair<hipEvent_t, hipEvent_t> prof_pair(alofdft_ctx* c, size_t used) {
  if (used == c->prof_pool.size()) {
    hipEvent_t a, b;
    HIPC(c, hipEventCreateWithFlags(&a, hipEventDisableSystemFence));
    HIPC(c, hipEventCreateWithFlags(&b, hipEventDisableSystemFence));
    c->prof_pool.push_back({a, b});
  }
  return c->prof_pool[used];
}

// The same CG in the pipelined form (one launch and one reduction per iteration,
// CGPipeOp), after the residual of the guess and w = A r (CGWInitOp).  Same
// arguments, stopping tests and result as cg_solve, plus verdict 4 (rounding breakdown).
template <typename T>
CGResult cg_solve_pipe(alofdft_ctx* c, const Geom& g, const StencilW<T>& A, const T* rhs, T* x, double tol,
                       long long max_it, int check_every, const char* tag, bool init, const double* init_parts,
                       int init_nparts, bool stop_on_stagnation, int first_poll) {
  const std::string t(tag);
  T* r = gridbuf<T>(c, t + ".r", g);
  T* wv[2] = {gridbuf<T>(c, t + ".w0", g), gridbuf<T>(c, t + ".w1", g)};
  T* sv = gridbuf<T>(c, t + ".Ap", g);
  T* z = gridbuf<T>(c, t + ".z", g);
  T* p = gridbuf<T>(c, t + ".p0", g);
  const int maxsb = max_stencil_blocks(g, c->target_blocks);
  double* partsI = bufT<double>(c, t + ".partsI", (size_t)std::max(maxsb, kPointwiseBlocks) * 2);
  double* pp[2] = {bufT<double>(c, t + ".partsC", (size_t)maxsb * 2), bufT<double>(c, t + ".partsD", (size_t)maxsb * 2)};
  CGState* st = bufT<CGState>(c, t + ".state", 1);
  static_assert(sizeof(CGState) % 8 == 0, "CGState is cleared in 8-byte words");
  zero_bytes(c, st, sizeof(CGState));
  const double* prev = init_parts;
  int nprev = init_nparts;
  if (init) {
    CGInitOp<T> op{x, rhs, r, nullptr, partsI};
    nprev = launch_stencil(c, g, A, op);
    prev = partsI;
  }
  const double tol2 = tol * tol;
  {
    CGWInitOp<T> op{r, wv[0], sv, p, z, st, prev, nprev, tol2, pp[0]};
    nprev = launch_stencil(c, g, A, op);
    prev = pp[0];
  }
  const int pi = sizeof(T) == 8 ? 0 : 1;
  std::vector<std::pair<long long, size_t>> pending;
  size_t pool_used = 0;
  auto harvest = [&](long long stop_iter) {
    for (auto& pe : pending) {
      if (pe.first >= stop_iter) continue;
      float ms = 0.f;
      HIPC(c, hipEventElapsedTime(&ms, c->prof_pool[pe.second].first, c->prof_pool[pe.second].second));
      c->prof_ms[pi] += ms;
      c->prof_ms_first[pi] += ms;
      c->prof_count[pi]++;
      c->prof_points[pi] = (long long)g.nx * g.ny * g.nz;
      c->prof_sched[pi] = 2;
    }
    pending.clear();
    pool_used = 0;
  };
  // iterate k reads the partials of the previous pass (pp[k & 1]) and writes pp[(k+1) & 1]
  auto launch_k = [&](long long k, int last, hipEvent_t e0, hipEvent_t e1) {
    const int a = (int)(k & 1), b = a ^ 1;
    const CGPipeOp<T> op{wv[a], wv[b], r, sv, z, p, x, st, prev, nprev, (int)k, last, pp[b], T(0), T(0)};
    nprev = launch_stencil(c, g, A, op, e0, e1);  // events stamp the kernel itself
    prev = pp[b];
  };
  long long k = 0;
  double best_rr = HUGE_VAL;
  long long best_k = 0;
  PollPlan poll(check_every, first_poll);
  for (;; ++k) {
    if (k >= max_it) break;
    const bool timed = sampled(c, k);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (timed) std::tie(e0, e1) = prof_pair(c, pool_used);
    launch_k(k, 0, e0, e1);
    if (timed) pending.push_back({k, pool_used++});
    if (poll.due(k)) {
      HIPC(c, hipMemcpyAsync(c->pin, st, sizeof(CGState), hipMemcpyDeviceToHost, c->stream));
      sync(c);
      check_cancel(c);
      const CGState* sp = (CGState*)c->pin;
      harvest(sp->done ? sp->iter : k + 1);
      if (sp->done) break;
      const double rr = sp->rrh[sp->iter & 1];
      poll.update(k, rr, sp->thresh);
      if (stop_on_stagnation) {
        if (rr < 0.5 * best_rr) {
          best_rr = rr;
          best_k = k;
        } else if (k - best_k >= stall_window(g)) {
          ++k;
          break;
        }
      }
    }
  }
  HIPC(c, hipMemcpyAsync(c->pin, st, sizeof(CGState), hipMemcpyDeviceToHost, c->stream));
  sync(c);
  CGState s = *(CGState*)c->pin;
  harvest(s.done ? s.iter : k);
  if (!s.done) {
    // verdict on the last residual without another update
    launch_k(k, 1, nullptr, nullptr);
    HIPC(c, hipMemcpyAsync(c->pin, st, sizeof(CGState), hipMemcpyDeviceToHost, c->stream));
    sync(c);
    s = *(CGState*)c->pin;
  }
  CGResult res;
  res.done = s.done;
  res.extra_mv = 1;
  res.late = s.done && s.iter != s.done_iter;
  if (s.done == 3) {
    fill<T>(c, x, g.total, T(0));
    return res;
  }
  res.iters = s.iter;
  const double rr = s.done ? s.rr_last : s.rrh[s.iter & 1];
  res.relres = s.rhs2 > 0 ? std::sqrt(rr / s.rhs2) : 0.0;
  return res;
}

// CG on A x = rhs (A = -(1/4 pi) Delta_h, zero ghosts) from the guess in x, to
// r.r <= tol^2 ||rhs||^2 (init = true: the residual is formed here; otherwise r,
// p0 and the init partials are already prepared by the caller).
template <typename T>
CGResult cg_solve(alofdft_ctx* c, const Geom& g, const StencilW<T>& A, const T* rhs, T* x, double tol, long long max_it,
                  int check_every, const char* tag, bool init = true, const double* init_parts = nullptr,
                  int init_nparts = 0, bool stop_on_stagnation = false, int first_poll = 1 << 30) {
  const int sched = cg_schedule_for(c, g, sizeof(T) == 8);
  if (sched == 2)
    return cg_solve_pipe<T>(c, g, A, rhs, x, tol, max_it, check_every, tag, init, init_parts, init_nparts,
                            stop_on_stagnation, first_poll);
  const std::string t(tag);
  // FP32 schedule 1 keeps p and A p interleaved: one 8-byte access per node for the pair
  // (the pair array is as large as an FP64 array, which require_addressable keeps below 4 GiB)
  const bool paired = sched == 1 && sizeof(T) == 4;
  T* r = gridbuf<T>(c, t + ".r", g);
  T* p0 = gridbuf<T>(c, t + ".p0", g);
  T* p1 = sched == 0 ? gridbuf<T>(c, t + ".p1", g) : p0;
  T* Ap = paired ? nullptr : gridbuf<T>(c, t + ".Ap", g);
  T* pa = paired ? reinterpret_cast<T*>(gridbuf<double>(c, t + ".pa", g)) : nullptr;  // 2 x total
  // first half of schedule 1 (interleaved pairs, or x made here in FP64, or neither)
  auto launch_first = [&](const CGP1Op<T>& op1, hipEvent_t ea, hipEvent_t eb) -> int {
    if constexpr (sizeof(T) == 4) {
      CGP1LIOp opi{op1};
      opi.pa = pa;
      return launch_stencil(c, g, A, opi, ea, eb);
    } else {
      CGP1LOp<T> opl{op1};
      opl.x = x;  // also makes the pending x += alpha p
      return launch_stencil(c, g, A, opl, ea, eb);
    }
  };
  const int maxsb = max_stencil_blocks(g, c->target_blocks);
  double* partsI = bufT<double>(c, t + ".partsI", (size_t)std::max(maxsb, kPointwiseBlocks) * 2);
  double* partsA = bufT<double>(c, t + ".partsA", (size_t)maxsb);
  double* partsB = bufT<double>(c, t + ".partsB", (size_t)kPointwiseBlocks);
  CGState* st = bufT<CGState>(c, t + ".state", 1);
  static_assert(sizeof(CGState) % 8 == 0, "CGState is cleared in 8-byte words");
  zero_bytes(c, st, sizeof(CGState));
  const double* prev = partsI;
  int nprev = 0;
  if (init) {
    CGInitOp<T> op{x, rhs, r, p0, partsI};
    nprev = launch_stencil(c, g, A, op);
  } else {
    prev = init_parts;
    nprev = init_nparts;
  }
  int nred_prev = 2;
  CGResult res;
  const double tol2 = tol * tol;
  const int pi = sizeof(T) == 8 ? 0 : 1;
  // sampled launches: (iteration, event pair index); pairs are read back at the
  // next host synchronisation and kept only for iterations before convergence
  std::vector<std::pair<long long, size_t>> pending;
  size_t pool_used = 0;
  auto harvest = [&](long long stop_iter) {
    for (auto& pe : pending) {
      if (pe.first >= stop_iter) continue;
      float ms = 0.f, ms2 = 0.f;
      HIPC(c, hipEventElapsedTime(&ms, c->prof_pool[pe.second].first, c->prof_pool[pe.second].second));
      HIPC(c, hipEventElapsedTime(&ms2, c->prof_pool[pe.second + 1].first, c->prof_pool[pe.second + 1].second));
      c->prof_ms[pi] += ms + ms2;
      c->prof_ms_first[pi] += ms;
      c->prof_ms_second[pi] += ms2;
      c->prof_count[pi]++;
      c->prof_points[pi] = (long long)g.nx * g.ny * g.nz;
      c->prof_sched[pi] = sched;
    }
    pending.clear();
    pool_used = 0;
  };
  long long k = 0;
  double best_rr = HUGE_VAL;
  long long best_k = 0;
  PollPlan poll(check_every, first_poll);
  for (;; ++k) {
    if (k >= max_it) break;
    T* pold = (k & 1) ? p1 : p0;
    T* pnew = (k & 1) ? p0 : p1;
    CGP1Op<T> op1{r, pold, pnew, Ap, st, prev, nprev, nred_prev, (int)k, tol2, partsA, T(0)};
    if (sched == 1) op1.pold = op1.pnew = p0;  // p and A p updated in place
    const bool timed = sampled(c, k);
    hipEvent_t e0 = nullptr, e1 = nullptr, e2 = nullptr, e3 = nullptr;
    if (timed) {  // both launches of the iteration carry a pair (pool entries pool_used, pool_used + 1)
      std::tie(e0, e1) = prof_pair(c, pool_used);
      std::tie(e2, e3) = prof_pair(c, pool_used + 1);
    }
    // FP64 schedule 1 moves x += alpha p into the next first half
    const bool defer_x = sched == 1 && CGP1LOp<T>::XD;
    const int nb1 = sched == 1 ? launch_first(op1, e0, e1)
                               : launch_stencil(c, g, A, op1, e0, e1);  // events stamp the kernel itself
    CGP2Op<T> op2{defer_x ? nullptr : x, r, paired ? pa : op1.pnew, Ap, st, partsA, nb1, (int)k, partsB, T(0)};
    op2.paired = paired ? 1 : 0;
    nprev = launch_cg_update(c, g, op2, e2, e3);
    if (timed) {
      pending.push_back({k, pool_used});
      pool_used += 2;
    }
    prev = partsB;
    nred_prev = 1;
    if (poll.due(k)) {
      HIPC(c, hipMemcpyAsync(c->pin, st, sizeof(CGState), hipMemcpyDeviceToHost, c->stream));
      sync(c);
      check_cancel(c);
      const CGState* sp = (CGState*)c->pin;
      harvest(sp->done ? sp->iter : k + 1);
      if (sp->done) break;
      const double rr = sp->rrh[sp->iter & 1];
      poll.update(k, rr, sp->thresh);
      if (stop_on_stagnation) {
        // rounding-limited (FP32) solve: give up when r.r has not halved within the window
        if (rr < 0.5 * best_rr) {
          best_rr = rr;
          best_k = k;
        } else if (k - best_k >= stall_window(g)) {
          ++k;
          break;
        }
      }
    }
  }
  // one more half iteration to test the last residual if the loop ended without a verdict
  HIPC(c, hipMemcpyAsync(c->pin, st, sizeof(CGState), hipMemcpyDeviceToHost, c->stream));
  sync(c);
  CGState s = *(CGState*)c->pin;
  harvest(s.done ? s.iter : k);
  if (!s.done && k < max_it + 1) {
    T* pold = (k & 1) ? p1 : p0;
    T* pnew = (k & 1) ? p0 : p1;
    CGP1Op<T> op1{r, pold, pnew, Ap, st, prev, nprev, nred_prev, (int)k, tol2, partsA, T(0)};
    if (sched == 1) {
      op1.pold = op1.pnew = p0;
      launch_first(op1, nullptr, nullptr);
    } else {
      launch_stencil(c, g, A, op1);
    }
    HIPC(c, hipMemcpyAsync(c->pin, st, sizeof(CGState), hipMemcpyDeviceToHost, c->stream));
    sync(c);
    s = *(CGState*)c->pin;
  }
  res.done = s.done;
  res.late = s.done && s.iter != s.done_iter;
  if (s.done == 3) {  // zero right-hand side: the solution is zero
    fill<T>(c, x, g.total, T(0));
    res.iters = 0;
    res.relres = 0.0;
    return res;
  }
  res.iters = s.done ? s.iter : k;  // iterations run (the cap, or fewer after a stagnation stop)
  const double rr = s.done ? s.rr_last : s.rrh[(s.iter) & 1];
  res.relres = s.rhs2 > 0 ? std::sqrt(rr / s.rhs2) : 0.0;
  return res;
}

struct PoissonStats {
  long long iters = 0, mv64 = 0, mv32 = 0, refinements = 0;
  double relres = 0.0;
  int status = 0;
  int restarts = 0;  // CG solves after the first (pipelined verification restarts)
  int late = 0;      // CG solves in which a launch after the verdict updated the iterate
  std::string verdicts;  // verdict and iterations of every CG solve, for the trace
};

// FP64 solve, or FP32 inner CG (FP64 dots) inside an FP64 iterative-refinement loop.
PoissonStats poisson(alofdft_ctx* c, const Geom& g, int fdn, double h, int precision, const double* rhs, double* x,
                     double tol, long long max_cg, int check_every) {
  PoissonStats ps;
  const StencilW<double> A64 = stencil_weights<double>(fdn, h, -0.25 / M_PI);
  if (precision == ALOFDFT_FP64) {
    // the pipelined recurrences carry r rather than recompute it, so their verdict is
    // checked once more from the true residual (a restart that stops at once when it
    // holds); a rounding breakdown (verdict 4) also restarts from the current iterate
    const bool pipe = cg_schedule_for(c, g, true) == 2;
    for (int restart = 0; restart < 8; ++restart) {
      // a restart after a converged pipelined solve is expected to stop at once: poll after
      // its first launch
      CGResult r = cg_solve<double>(c, g, A64, rhs, x, tol, max_cg - ps.iters, check_every, "cg64", true, nullptr,
                                    0, false, restart > 0 ? 1 : check_every);
      ps.iters += r.iters;
      ps.mv64 += r.iters + 1 + r.extra_mv;
      ps.relres = r.relres;
      ps.restarts = restart;
      ps.late += r.late;
      if (c->trace) {
        char b[96];
        std::snprintf(b, sizeof b, "%d:%lld:%.17g,", r.done, r.iters, r.relres);
        ps.verdicts += b;
      }
      const bool again = pipe && ((r.done == 1 && r.iters > 0) || r.done == 4);
      if (again && ps.iters < max_cg && restart < 7) continue;
      ps.status = r.done == 2 ? ALOFDFT_NUMERICAL : (r.done == 1 || r.done == 3 ? 0 : ALOFDFT_NOT_CONVERGED);
      return ps;
    }
    ps.status = ALOFDFT_NOT_CONVERGED;
    return ps;
  }
  const StencilW<float> A32 = stencil_weights<float>(fdn, h, -0.25 / M_PI);
  double* r64 = gridbuf<double>(c, "ref.r64", g);
  float* r32 = gridbuf<float>(c, "cg32.r", g);
  float* p32 = gridbuf<float>(c, "cg32.p0", g);
  float* x32 = gridbuf<float>(c, "ref.x32", g);
  const int maxsb = max_stencil_blocks(g, c->target_blocks);
  double* partsR = bufT<double>(c, "ref.parts", (size_t)std::max(maxsb, kPointwiseBlocks) * 2);
  double* partsF = bufT<double>(c, "ref.partsF", (size_t)kPointwiseBlocks * 2);
  double* sc = bufT<double>(c, "ref.sc", 4);
  const double inner_tol = std::pow(10.0, -c->inner_tol_exp);
  double rhs2 = -1.0;
  for (int ref = 0; ref < 60; ++ref) {
    // FP64 residual r64 = rhs - A x, with r.r and rhs.rhs
    CGInitOp<double> op{x, rhs, r64, nullptr, partsR};
    const int nb = launch_stencil(c, g, A64, op);
    ps.mv64++;
    finalize(c, partsR, nb, 2, 1.0, sc);
    HIPC(c, hipMemcpyAsync(c->pin, sc, 2 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    sync(c);
    const double rr = c->pin[0];
    rhs2 = c->pin[1];
    if (!std::isfinite(rr)) { ps.status = ALOFDFT_NUMERICAL; return ps; }
    if (rhs2 == 0.0) {
      fill<double>(c, x, g.total, 0.0);
      ps.relres = 0.0;
      return ps;
    }
    ps.relres = std::sqrt(rr / rhs2);
    if (ps.relres <= tol) return ps;
    if (ps.iters >= max_cg) { ps.status = ALOFDFT_NOT_CONVERGED; return ps; }
    ps.refinements++;
    // inner FP32 CG on A e = r64 from e = 0
    ToFloatOp tf{r64, r32, p32, x32, partsF};
    const int nbf = launch_pw(c, g, tf);
    // aim below the outer tolerance without asking FP32 for more than it can give
    const double want = std::max(inner_tol, 0.5 * tol / ps.relres);
    CGResult ir = cg_solve<float>(c, g, A32, nullptr, x32, want, max_cg - ps.iters, check_every, "cg32", false,
                                  partsF, nbf, true);
    ps.iters += ir.iters;
    ps.mv32 += ir.iters + ir.extra_mv;
    ps.late += ir.late;
    if (c->trace) ps.verdicts += std::to_string(ir.done) + ":" + std::to_string(ir.iters) + " ";
    if (ir.done == 2) { ps.status = ALOFDFT_NUMERICAL; return ps; }
    AddFloatOp add{x, x32, nullptr};
    launch_pw(c, g, add);
  }
  ps.status = ALOFDFT_NOT_CONVERGED;
  return ps;
}

// ----------------------------------------------------------------- trace
std::mutex g_trace_mu;
FILE* g_trace_file = nullptr;

// FNV-1a hash of the interior bytes of a padded FP64 grid array (a host copy).
uint64_t grid_hash(alofdft_ctx* c, const Geom& g, const double* a) {
  std::vector<double> h((size_t)g.total);
  HIPC(c, hipMemcpyAsync(h.data(), a, sizeof(double) * g.total, hipMemcpyDeviceToHost, c->stream));
  sync(c);
  uint64_t x = 1469598103934665603ull;
  for (int k = 0; k < g.nz; ++k)
    for (int j = 0; j < g.ny; ++j)
      for (int i = 0; i < g.nx; ++i) {
        uint64_t v;
        std::memcpy(&v, &h[g.base + (size_t)k * g.plane + (size_t)j * g.px + i], 8);
        for (int b = 0; b < 8; ++b) x = (x ^ ((v >> (8 * b)) & 0xff)) * 1099511628211ull;
      }
  return x;
}

void trace_line(const char* fmt, ...) {
  std::lock_guard<std::mutex> lk(g_trace_mu);
  if (!g_trace_file) return;
  va_list ap;
  va_start(ap, fmt);
  std::vfprintf(g_trace_file, fmt, ap);
  va_end(ap);
  std::fflush(g_trace_file);
}

// ----------------------------------------------------------------- nuclei on the device
struct DevAtoms {
  AtomsDev a;
};

DevAtoms upload_atoms(alofdft_ctx* c, const alofdft_system* sys, double rc) {
  const int M = sys->M;
  // cell list with cells of side >= rc over the box
  double lo[3], hi[3];
  for (int a = 0; a < 3; ++a) {
    lo[a] = sys->origin[a] - rc;
    hi[a] = sys->origin[a] + (sys->n[a] - 1) * sys->h + rc;
  }
  const double cs = std::max(rc, 1e-6);
  int cd[3];
  for (int a = 0; a < 3; ++a) cd[a] = std::max(1, (int)std::ceil((hi[a] - lo[a]) / cs));
  const int ncell = cd[0] * cd[1] * cd[2];
  std::vector<int> cell_of(M), start(ncell + 1, 0), order(M);
  for (int J = 0; J < M; ++J) {
    int ci[3];
    for (int a = 0; a < 3; ++a)
      ci[a] = std::min(cd[a] - 1, std::max(0, (int)std::floor((sys->R[3 * J + a] - lo[a]) / cs)));
    cell_of[J] = (ci[2] * cd[1] + ci[1]) * cd[0] + ci[0];
    start[cell_of[J] + 1]++;
  }
  for (int i = 0; i < ncell; ++i) start[i + 1] += start[i];
  std::vector<int> fillp(start.begin(), start.end() - 1);
  for (int J = 0; J < M; ++J) order[fillp[cell_of[J]]++] = J;
  double* dR = bufT<double>(c, "atoms.R", 3 * (size_t)M);
  double* dZ = bufT<double>(c, "atoms.Z", (size_t)M);
  int* dS = bufT<int>(c, "atoms.start", (size_t)ncell + 1);
  int* dA = bufT<int>(c, "atoms.order", (size_t)M);
  HIPC(c, hipMemcpyAsync(dR, sys->R, 3 * sizeof(double) * M, hipMemcpyHostToDevice, c->stream));
  HIPC(c, hipMemcpyAsync(dZ, sys->Z, sizeof(double) * M, hipMemcpyHostToDevice, c->stream));
  HIPC(c, hipMemcpyAsync(dS, start.data(), sizeof(int) * (ncell + 1), hipMemcpyHostToDevice, c->stream));
  HIPC(c, hipMemcpyAsync(dA, order.data(), sizeof(int) * M, hipMemcpyHostToDevice, c->stream));
  sync(c);  // host vectors go out of scope
  DevAtoms d;
  d.a.R = dR;
  d.a.Z = dZ;
  d.a.cell_start = dS;
  d.a.cell_atoms = dA;
  d.a.M = M;
  for (int a = 0; a < 3; ++a) {
    d.a.cdim[a] = cd[a];
    d.a.clo[a] = lo[a];
  }
  d.a.csize = cs;
  return d;
}

// Device description of b_J for the parameters: the Gaussian, or the discrete Laplacian of
// V_J (Sec. 4) with the order-2n weights of the grid.
PseudoDev pseudo_of(const alofdft_params* p, double h) {
  PseudoDev P{};
  P.mode = p->pseudocharge;
  P.R = p->fd_half_width;
  P.s = p->gauss_width;
  P.rc = p->r_cut;
  P.h = h;
  double w[kMaxRadius + 1];
  lap_weights(p->fd_half_width, h, w);
  for (int q = 0; q <= kMaxRadius; ++q) P.w[q] = q <= p->fd_half_width ? w[q] : 0.0;
  return P;
}

void pseudocharge_dev(alofdft_ctx* c, const Geom& g, const alofdft_system* sys, const DevAtoms& at,
                      const PseudoDev& P, double* b) {
  fill<double>(c, b, g.total, 0.0);
  hipLaunchKernelGGL(k_pseudocharge, dim3(4096), dim3(256), 0, c->stream, g, sys->h, sys->origin[0], sys->origin[1],
                     sys->origin[2], at.a, P, b);
  CHECK_LAUNCH(c);
}

// Superposition of atomic densities (Sec. 4) as the initial u, into a dense device
// array: rho = sum_J Z_J (pi w^2)^(-3/2) exp(-r^2/w^2) (r <= 5w) + floor N/V, scaled to
// h^3 sum rho = N, u = sqrt(rho).
void atomic_guess_dev(alofdft_ctx* c, const alofdft_system* sys, const alofdft_params* prm, double* u_dense) {
  const Geom g = make_geom(sys->n, prm->fd_half_width);
  const double w = prm->guess_width;
  const DevAtoms at = upload_atoms(c, sys, 5.0 * w);
  double* rho = bufT<double>(c, "guess.rho", g.total);
  const int nb = 1024;
  double* parts = bufT<double>(c, "guess.parts", nb);
  double* tot = bufT<double>(c, "guess.sum", 1);
  const double h3 = sys->h * sys->h * sys->h;
  const double floor_rho = prm->guess_floor * sys->N_elec / ((double)sys->n[0] * sys->n[1] * sys->n[2] * h3);
  hipLaunchKernelGGL((k_atomic_density<256>), dim3(nb), dim3(256), 0, c->stream, g, sys->h, sys->origin[0],
                     sys->origin[1], sys->origin[2], at.a, w, floor_rho, rho, parts);
  CHECK_LAUNCH(c);
  finalize(c, parts, nb, 1, 1.0, tot);
  hipLaunchKernelGGL(k_density_to_u, dim3(2048), dim3(256), 0, c->stream, g, rho, tot, sys->N_elec, h3, u_dense);
  CHECK_LAUNCH(c);
}

// per-atom sums: self energy (phi == nullptr) or force sums (phi != nullptr)
void atom_sums(alofdft_ctx* c, const Geom& g, const alofdft_system* sys, const DevAtoms& at, const PseudoDev& P,
               int fdn, const double* phi, std::vector<double>* self, std::vector<double>* force) {
  const int M = sys->M;
  double* out = bufT<double>(c, "atoms.out", 4 * (size_t)M);
  StencilW<double> wt;
  double w[kMaxRadius + 1];
  grad_weights(fdn, sys->h, w);
  wt.c0 = 0.0;
  for (int p = 0; p <= kMaxRadius; ++p) wt.w[p] = p <= fdn ? w[p] : 0.0;
  hipLaunchKernelGGL((k_atom_sums<256>), dim3(M), dim3(256), 0, c->stream, g, sys->h, sys->origin[0],
                     sys->origin[1], sys->origin[2], at.a, P, wt, fdn, phi, self ? out : nullptr,
                     force ? out + M : nullptr);
  CHECK_LAUNCH(c);
  std::vector<double> host(4 * (size_t)M);
  HIPC(c, hipMemcpyAsync(host.data(), out, sizeof(double) * 4 * M, hipMemcpyDeviceToHost, c->stream));
  sync(c);
  if (self) self->assign(host.begin(), host.begin() + M);
  if (force) force->assign(host.begin() + M, host.begin() + 4 * M);
}

// Appendix-A correction for Gaussian pseudocharges: E_c = 1/2 sum_{I!=J} Z_I Z_J
// erfc(R_IJ/(sqrt2 s))/R_IJ and f^c = -dE_c/dR.  Pairs beyond 7 sqrt2 s
// (erfc < 5e-23) are skipped through a cell list.
double overlap_correction(const alofdft_system* sys, double s, std::vector<double>* fc) {
  const int M = sys->M;
  const double a = std::sqrt(2.0) * s, rcut = 7.0 * a;
  if (fc) fc->assign(3 * (size_t)M, 0.0);
  double lo[3], hi[3];
  for (int d = 0; d < 3; ++d) {
    lo[d] = 1e300;
    hi[d] = -1e300;
    for (int J = 0; J < M; ++J) {
      lo[d] = std::min(lo[d], sys->R[3 * J + d]);
      hi[d] = std::max(hi[d], sys->R[3 * J + d]);
    }
  }
  int cd[3];
  for (int d = 0; d < 3; ++d) cd[d] = std::max(1, (int)std::ceil((hi[d] - lo[d]) / rcut + 1e-9));
  std::vector<std::vector<int>> cells((size_t)cd[0] * cd[1] * cd[2]);
  std::vector<int> ci(3 * (size_t)M);
  for (int J = 0; J < M; ++J) {
    for (int d = 0; d < 3; ++d)
      ci[3 * J + d] = std::min(cd[d] - 1, (int)std::floor((sys->R[3 * J + d] - lo[d]) / rcut));
    cells[((size_t)ci[3 * J + 2] * cd[1] + ci[3 * J + 1]) * cd[0] + ci[3 * J]].push_back(J);
  }
  double E = 0.0;
  for (int J = 0; J < M; ++J) {
    for (int z = std::max(0, ci[3 * J + 2] - 1); z <= std::min(cd[2] - 1, ci[3 * J + 2] + 1); ++z)
      for (int y = std::max(0, ci[3 * J + 1] - 1); y <= std::min(cd[1] - 1, ci[3 * J + 1] + 1); ++y)
        for (int x = std::max(0, ci[3 * J] - 1); x <= std::min(cd[0] - 1, ci[3 * J] + 1); ++x)
          for (int I : cells[((size_t)z * cd[1] + y) * cd[0] + x]) {
            if (I == J) continue;
            double dv[3];
            for (int d = 0; d < 3; ++d) dv[d] = sys->R[3 * J + d] - sys->R[3 * I + d];
            const double r = std::sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
            if (r > rcut) continue;
            const double ZZ = sys->Z[I] * sys->Z[J];
            E += 0.5 * ZZ * std::erfc(r / a) / r;
            if (fc) {
              const double dF = -std::erfc(r / a) / (r * r) - 2.0 / (a * std::sqrt(M_PI)) * std::exp(-r * r / (a * a)) / r;
              for (int d = 0; d < 3; ++d) (*fc)[3 * J + d] -= ZZ * dF * dv[d] / r;
            }
          }
  }
  return E;
}

// ----------------------------------------------------------------- validation
// The streaming kernels address a grid array through a raw buffer resource with 32-bit
// byte offsets, and the CG kernels have no other form, so every padded work array (FP64,
// or a pair of FP32 values per node) must stay below 4 GiB: cubes up to 768^3 nodes at
// n = 6.
void require_addressable(alofdft_ctx* c, const int n[3], int fdn) {
  const Geom g = make_geom(n, fdn);
  require(c, g.total * 8 < (1ll << 32), "grid too large: a padded FP64 array must stay below 4 GiB");
}

void validate(alofdft_ctx* c, const alofdft_system* s, const alofdft_params* p) {
  require(c, s && p, "null system or params");
  require(c, p->fd_half_width >= 1 && p->fd_half_width <= kMaxRadius, "fd_half_width must be in 1..8");
  require(c, std::isfinite(s->h) && s->h > 0, "h must be > 0");
  for (int a = 0; a < 3; ++a) require(c, s->n[a] >= 2 * p->fd_half_width + 1, "grid smaller than 2n+1 nodes");
  require_addressable(c, s->n, p->fd_half_width);
  require(c, s->M >= 1 && s->R && s->Z, "need at least one atom");
  require(c, std::isfinite(s->N_elec) && s->N_elec > 0, "N must be > 0");
  require(c, p->lambda > 0 && p->gauss_width > 0 && p->r_cut > 0, "lambda, gauss_width, r_cut must be > 0");
  require(c, p->method == ALOFDFT_METHOD_AUGMENTED_LAGRANGIAN || p->method == ALOFDFT_METHOD_PENALTY ||
                 p->method == ALOFDFT_METHOD_LAGRANGE,
          "method must be augmented Lagrangian, penalty or Lagrange multiplier");
  require(c, p->pseudocharge == ALOFDFT_PSEUDO_GAUSSIAN || p->pseudocharge == ALOFDFT_PSEUDO_FD_LAPLACIAN,
          "bad pseudocharge");
  require(c, p->initial_guess == ALOFDFT_GUESS_UNIFORM || p->initial_guess == ALOFDFT_GUESS_ATOMIC,
          "bad initial_guess");
  require(c, p->initial_guess != ALOFDFT_GUESS_ATOMIC || (p->guess_width > 0 && p->guess_floor > 0),
          "the atomic guess needs guess_width > 0 and guess_floor > 0");
  require(c, p->al_stop == ALOFDFT_STOP_CONSTRAINT || (p->al_stop == ALOFDFT_STOP_ENERGY_CHANGE && p->tol_energy > 0),
          "bad al_stop or tol_energy");
  require(c, p->domain == ALOFDFT_DOMAIN_BOX || p->domain == ALOFDFT_DOMAIN_ELLIPSOID, "bad domain");
  require(c, p->domain == ALOFDFT_DOMAIN_BOX || p->phi_bc == ALOFDFT_BC_ZERO,
          "the ellipsoidal domain takes zero boundary values for phi (phi_bc = ALOFDFT_BC_ZERO)");
  require(c, p->mu0 > 0 && p->kappa > 0 && p->kappa < 1, "need mu0 > 0 and 0 < kappa < 1");
  require(c, p->phi_bc == ALOFDFT_BC_ZERO || p->phi_bc == ALOFDFT_BC_MULTIPOLE, "bad phi_bc");
  require(c, p->precision == ALOFDFT_FP64 || p->precision == ALOFDFT_FP32_REFINED, "bad precision");
  require(c, p->tol_poisson > 0 && p->tol_grad > 0 && p->tol_constraint > 0, "tolerances must be > 0");
  require(c, p->cg_check_every >= 1 && p->max_cg >= 1 && p->max_inner >= 1 && p->max_outer >= 1 && p->max_secant >= 1,
          "iteration caps must be >= 1");
  for (int J = 0; J < s->M; ++J) {
    require(c, std::isfinite(s->Z[J]), "non-finite Z");
    for (int a = 0; a < 3; ++a) {
      const double x = s->R[3 * J + a];
      require(c, std::isfinite(x), "non-finite atom position");
      const double lo = s->origin[a], hi = s->origin[a] + (s->n[a] - 1) * s->h;
      require(c, x - p->r_cut >= lo - 1e-9 && x + p->r_cut <= hi + 1e-9, "an atom's r_cut ball leaves the box");
    }
  }
}

// ----------------------------------------------------------------- Lagrange-multiplier method (Sec. 5.3.2)
// gp = g - eta u (the residual projected with the Rayleigh-quotient multiplier); reduces
// gp.gp and gp.gp_old (Polak-Ribiere).
struct LMResidualOp {
  static constexpr int NRED = 2;
  const double* g;
  const double* u;
  double* gp;
  const double* gp_old;  // nullable (first step)
  double eta;
  double* parts_out;
  template <int NT>
  __device__ bool begin() { return true; }
  __device__ void apply(long long i, int, int, int, double* red) const {
    const double v = g[i] - eta * u[i];
    gp[i] = v;
    red[0] += v * v;
    if (gp_old) red[1] += v * gp_old[i];
  }
};
// d = -gp / M + beta d (constant Jacobi scaling M of the von Weizsaecker diagonal); reduces u.d.
struct LMDirectionOp {
  static constexpr int NRED = 1;
  const double* gp;
  const double* u;
  double* d;
  double inv_m, beta;
  double* parts_out;
  template <int NT>
  __device__ bool begin() { return true; }
  __device__ void apply(long long i, int, int, int, double* red) const {
    const double dn = beta != 0.0 ? -gp[i] * inv_m + beta * d[i] : -gp[i] * inv_m;
    d[i] = dn;
    red[0] += u[i] * dn;
  }
};
// d -= a u (d orthogonal to u); reduces g.d and d.d.
struct LMProjectOp {
  static constexpr int NRED = 2;
  const double* g;
  const double* u;
  double* d;
  double a;
  double* parts_out;
  template <int NT>
  __device__ bool begin() { return true; }
  __device__ void apply(long long i, int, int, int, double* red) const {
    const double dn = d[i] - a * u[i];
    d[i] = dn;
    red[0] += g[i] * dn;
    red[1] += dn * dn;
  }
};
// u = |v| over the interior (the accepted point of a line search), reduces sum u^2.
struct AbsOp {
  static constexpr int NRED = 1;
  double* u;
  const double* v;
  double scale;
  double* parts_out;
  template <int NT>
  __device__ bool begin() { return true; }
  __device__ void apply(long long i, int, int, int, double* red) const {
    const double x = scale * fabs(v[i]);
    u[i] = x;
    red[0] += x * x;
  }
};

// Minimum of f on [lo, hi] from an interior point x0 with f(x0) below both ends: Brent's
// method (golden-section steps with parabolic interpolation through the three best
// points, R. P. Brent, "Algorithms for Minimization without Derivatives", 1973, ch. 5).
// Stops when the bracket is within 2 tol |x| + eps of the best point or after maxit
// evaluations; returns the best point found.
double brent_minimise(const std::function<double(double)>& f, double lo, double hi, double x0, double f0, double tol,
                      int maxit) {
  const double golden = 0.5 * (3.0 - std::sqrt(5.0));
  double best = x0, fbest = f0;       // lowest value so far
  double second = x0, fsecond = f0;   // second lowest
  double third = x0, fthird = f0;     // previous value of second
  double step = 0.0, prev_step = 0.0;
  for (int it = 0; it < maxit; ++it) {
    const double mid = 0.5 * (lo + hi);
    const double t1 = tol * std::fabs(best) + 1e-12, t2 = 2.0 * t1;
    if (std::fabs(best - mid) <= t2 - 0.5 * (hi - lo)) break;
    bool parabolic = false;
    if (std::fabs(prev_step) > t1) {
      // vertex of the parabola through (best, second, third), as best + p/q
      const double r = (best - second) * (fbest - fthird);
      double q = (best - third) * (fbest - fsecond);
      double p = (best - third) * q - (best - second) * r;
      q = 2.0 * (q - r);
      if (q > 0.0) p = -p;
      q = std::fabs(q);
      const double keep = prev_step;
      prev_step = step;
      // accept only a step inside the bracket and shorter than half the step before last
      if (std::fabs(p) < std::fabs(0.5 * q * keep) && p > q * (lo - best) && p < q * (hi - best)) {
        step = p / q;
        const double x = best + step;
        if (x - lo < t2 || hi - x < t2) step = mid >= best ? t1 : -t1;
        parabolic = true;
      }
    }
    if (!parabolic) {
      prev_step = best >= mid ? lo - best : hi - best;
      step = golden * prev_step;
    }
    const double x = std::fabs(step) >= t1 ? best + step : best + (step > 0 ? t1 : -t1);
    const double fx = f(x);
    if (fx <= fbest) {
      if (x >= best) lo = best; else hi = best;
      third = second; fthird = fsecond;
      second = best; fsecond = fbest;
      best = x; fbest = fx;
    } else {
      if (x < best) lo = x; else hi = x;
      if (fx <= fsecond || second == best) {
        third = second; fthird = fsecond;
        second = x; fsecond = fx;
      } else if (fx <= fthird || third == best || third == second) {
        third = x; fthird = fx;
      }
    }
  }
  return best;
}

// ----------------------------------------------------------------- the solver
uint64_t splitmix64(uint64_t state) {
  uint64_t z = state + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Active domain of Sec. 5.1: the ellipsoid inscribed in the box of nodes (centre and
// semi-axes (n_a - 1)/2 in index units); a node is free when
// sum_a ((i_a - c_a) / c_a)^2 <= 1 + 1e-12, summed over the axes in order, and every row
// (j, k) of free nodes is one x range by convexity.  Device table of the ranges (Geom::dom).
const int* domain_rows(alofdft_ctx* c, const int n[3]) {
  const double cen[3] = {0.5 * (n[0] - 1), 0.5 * (n[1] - 1), 0.5 * (n[2] - 1)};
  auto term = [&](int a, int idx) {
    if (!(cen[a] > 0)) return 0.0;
    const double t = (idx - cen[a]) / cen[a];
    return t * t;
  };
  std::vector<int> rows(2 * (size_t)n[1] * n[2]);
  for (int k = 0; k < n[2]; ++k)
    for (int j = 0; j < n[1]; ++j) {
      int lo = n[0], hi = -1;
      for (int i = 0; i < n[0]; ++i) {
        double q = 0.0;
        q += term(0, i);
        q += term(1, j);
        q += term(2, k);
        if (q <= 1.0 + 1e-12) {
          lo = std::min(lo, i);
          hi = std::max(hi, i);
        }
      }
      rows[2 * ((size_t)k * n[1] + j)] = lo;
      rows[2 * ((size_t)k * n[1] + j) + 1] = hi;
    }
  int* d = bufT<int>(c, "s.dom", rows.size());
  HIPC(c, hipMemcpyAsync(d, rows.data(), rows.size() * sizeof(int), hipMemcpyHostToDevice, c->stream));
  sync(c);  // rows is released on return
  return d;
}

struct Eval {  // host copy of one evaluation's scalars
  double upd[kUpdRed];  // h^3-scaled
  double gr[G_NRED];    // raw sums
};

class Solver {
 public:
  Solver(alofdft_ctx* c, const alofdft_system* sys, const alofdft_params* prm)
      : c_(c), S_(sys), P_(prm) {
    g_ = make_geom(sys->n, prm->fd_half_width);
    if (prm->domain == ALOFDFT_DOMAIN_ELLIPSOID) g_.dom = domain_rows(c, sys->n);
    h3_ = sys->h * sys->h * sys->h;
    const size_t T = g_.total;
    us_ = bufT<double>(c, "s.us", T);
    v_ = bufT<double>(c, "s.v", T);
    d_ = bufT<double>(c, "s.d", T);
    sa_ = bufT<double>(c, "s.sa", T);
    sb_ = bufT<double>(c, "s.sb", T);
    b_ = bufT<double>(c, "s.b", T);
    phi_ = bufT<double>(c, "s.phi", T);
    rhs_ = bufT<double>(c, "s.rhs", T);
    for (int i = 0; i < 3; ++i) ph_[i] = bufT<double>(c, "s.ph" + std::to_string(i), T);
    partsU_ = bufT<double>(c, "s.partsU", (size_t)kPointwiseBlocks * kUpdRed);
    partsG_ = bufT<double>(c, "s.partsG", (size_t)max_stencil_blocks(g_, c->target_blocks) * G_NRED);
    scal_ = bufT<double>(c, "s.scal", kUpdRed + G_NRED + 8);
    double w[kMaxRadius + 1];
    lap_weights(prm->fd_half_width, sys->h, w);
    vw_diag_ = -3.0 * prm->lambda * w[0];
    Wlap_ = stencil_weights<double>(prm->fd_half_width, sys->h, 1.0);
    frame_.h = sys->h;
    frame_.hx = 0.5 * (sys->n[0] - 1);
    frame_.hy = 0.5 * (sys->n[1] - 1);
    frame_.hz = 0.5 * (sys->n[2] - 1);
    CF_ = 0.3 * std::pow(3.0 * M_PI * M_PI, 2.0 / 3.0);
  }

  // Zero all work arrays (halo included) and set up the nuclei.  warm_phi keeps phi
  // from the context's previous solve on the same grid as the first Poisson guess.
  void setup(const double* u0_dense_dev, bool u0_abs, bool warm_phi = false) {
    for (double* a : {us_, v_, d_, sa_, sb_, b_, rhs_, ph_[0], ph_[1], ph_[2]}) fill<double>(c_, a, g_.total, 0.0);
    if (!warm_phi) fill<double>(c_, phi_, g_.total, 0.0);
    at_ = upload_atoms(c_, S_, P_->r_cut);
    pseudo_ = pseudo_of(P_, S_->h);
    pseudocharge_dev(c_, g_, S_, at_, pseudo_, b_);
    std::vector<double> self;
    atom_sums(c_, g_, S_, at_, pseudo_, P_->fd_half_width, nullptr, &self, nullptr);
    E_self_ = 0.0;
    for (double x : self) E_self_ += 0.5 * h3_ * x;
    E_c_ = overlap_correction(S_, P_->gauss_width, nullptr);
    pack<double, double>(c_, g_, u0_dense_dev, us_, u0_abs ? 1 : 0);
  }

  // Evaluate at v = u_start + t d (trial) or with the direction update fused (dir).
  void eval_trial(double t, double eta, double mu, bool with_dir, double beta, Eval& ev) {
    bad_ = false;
    if (with_dir) {
      // new line: phi of the start point (t = 0) opens the history
      CombineOp cp{ph_[0], phi_, nullptr, nullptr, 1.0, 0.0, 0.0, nullptr};
      launch_pw(c_, g_, cp);
      th_[0] = 0.0;
      nh_ = 1;
      DirOp op{us_, d_, s_new(), v_, b_, beta, t, frame_, partsU_};
      nU_ = launch_pw(c_, g_, op);
      std::swap(s_cur_, s_prev_);  // the s just used becomes s_old of the next gradient
    } else {
      TrialOp op{us_, d_, b_, v_, t, frame_, partsU_};
      nU_ = launch_pw(c_, g_, op);
    }
    if (nh_ >= 2) {
      // Lagrange interpolation of phi(t) through the solved points of this line
      double L[3] = {1.0, 1.0, 1.0};
      for (int i = 0; i < nh_; ++i)
        for (int j = 0; j < nh_; ++j)
          if (i != j) L[i] *= (t - th_[j]) / (th_[i] - th_[j]);
      CombineOp cp{phi_, ph_[0], ph_[1], nh_ > 2 ? ph_[2] : nullptr, L[0], L[1], nh_ > 2 ? L[2] : 0.0, nullptr};
      launch_pw(c_, g_, cp);
    }
    eval_at_v(eta, mu, ev);
    if (!bad_ && nh_ >= 1 && nh_ < 3) {
      CombineOp cp{ph_[nh_], phi_, nullptr, nullptr, 1.0, 0.0, 0.0, nullptr};
      launch_pw(c_, g_, cp);
      th_[nh_++] = t;
    }
  }

  void eval_at_v(double eta, double mu, Eval& ev) {
    double* upd = scal_;
    double* gsc = scal_ + kUpdRed;
    finalize(c_, partsU_, nU_, kUpdRed, h3_, upd);
    RhsOp<double> rop{v_, b_, rhs_, P_->phi_bc == ALOFDFT_BC_MULTIPOLE ? upd : nullptr, Wlap_, g_.R,
                      g_.nx, g_.ny, g_.nz, frame_, nullptr};
    rop.dom = g_.dom;
    // RhsOp reads unscaled weights w[p]
    double w[kMaxRadius + 1];
    lap_weights(P_->fd_half_width, S_->h, w);
    for (int p = 0; p <= kMaxRadius; ++p) rop.W.w[p] = p <= P_->fd_half_width ? w[p] : 0.0;
    launch_pw(c_, g_, rop);
    uint64_t h_rhs = 0, h_phi0 = 0;
    if (c_->trace_hash) {
      h_rhs = grid_hash(c_, g_, rhs_);
      h_phi0 = grid_hash(c_, g_, phi_);
    }
    unsigned long long* cks = nullptr;
    if (c_->trace) {  // device checksums of rhs, phi before and phi after, read back with the sums
      cks = bufT<unsigned long long>(c_, "trace.cks", 4);
      fill<unsigned long long>(c_, cks, 4, 0ull);
      hipLaunchKernelGGL(k_checksum, dim3(256), dim3(256), 0, c_->stream, g_, rhs_, cks);
      hipLaunchKernelGGL(k_checksum, dim3(256), dim3(256), 0, c_->stream, g_, (const double*)phi_, cks + 1);
      CHECK_LAUNCH(c_);
    }
    auto t0 = std::chrono::steady_clock::now();
    PoissonStats ps = poisson(c_, g_, P_->fd_half_width, S_->h, P_->precision, rhs_, phi_, P_->tol_poisson,
                              P_->max_cg, P_->cg_check_every);
    auto t1 = std::chrono::steady_clock::now();
    const uint64_t h_phi1 = c_->trace_hash ? grid_hash(c_, g_, phi_) : 0;
    if (cks) {
      hipLaunchKernelGGL(k_checksum, dim3(256), dim3(256), 0, c_->stream, g_, (const double*)phi_, cks + 2);
      CHECK_LAUNCH(c_);
    }
    time_poisson_ += std::chrono::duration<double, std::milli>(t1 - t0).count();
    counts_.poisson_solves++;
    counts_.cg_iters += ps.iters;
    counts_.matvec_fp64 += ps.mv64;
    counts_.matvec_fp32 += ps.mv32;
    counts_.refinements += ps.refinements;
    relres_ = ps.relres;
    if (ps.status == ALOFDFT_NUMERICAL) {
      // a non-finite charge: report the trial as non-finite; phi is reset to the
      // potential at the start of the line (or zero) so later solves start clean
      bad_ = true;
      if (c_->progress)
        std::fprintf(stderr, "alofdft: Poisson solve failed (non-finite or p.Ap <= 0) after %lld CG iterations\n",
                     ps.iters);
      if (nh_ >= 1) {
        CombineOp cp{phi_, ph_[0], nullptr, nullptr, 1.0, 0.0, 0.0, nullptr};
        launch_pw(c_, g_, cp);
      } else {
        fill<double>(c_, phi_, g_.total, 0.0);
      }
      for (int i = 0; i < G_NRED; ++i) ev.gr[i] = NAN;
      for (int i = 0; i < kUpdRed; ++i) ev.upd[i] = NAN;
      return;
    }
    if (ps.status == ALOFDFT_NOT_CONVERGED) poisson_capped_ = true;
    GradOp gop{v_, phi_, b_, d_, s_old(), s_new(), gout_, upd, 0.5 * P_->lambda, eta, mu > 0 ? 1.0 / mu : 0.0,
               vw_diag_, CF_, P_->xc, partsG_, 0.0};
    gop.Cptr = upd;
    // shift uses C = h^3 sum v^2 - N: pass N through eta (eta' = eta + N/mu)
    gop.eta = eta + (mu > 0 ? S_->N_elec / mu : 0.0);
    const int nG = launch_stencil(c_, g_, Wlap_, gop);
    finalize(c_, partsG_, nG, G_NRED, 1.0, gsc);
    HIPC(c_, hipMemcpyAsync(c_->pin, scal_, sizeof(double) * (kUpdRed + G_NRED), hipMemcpyDeviceToHost, c_->stream));
    sync(c_);
    std::memcpy(ev.upd, c_->pin, sizeof(double) * kUpdRed);
    std::memcpy(ev.gr, c_->pin + kUpdRed, sizeof(double) * G_NRED);
    if (c_->trace) {
      // the density moments that fixed the right-hand side, the Poisson solve, and the
      // sums of the evaluation that used its phi, all as exact bit patterns
      std::string sums;
      char b[24];
      for (int i = 0; i < kUpdRed; ++i) {
        std::snprintf(b, sizeof b, "%016llx", (unsigned long long)__builtin_bit_cast(uint64_t, ev.upd[i]));
        sums += i ? "," : "";
        sums += b;
      }
      sums += " gr ";
      for (int i = 0; i < G_NRED; ++i) {
        std::snprintf(b, sizeof b, "%016llx", (unsigned long long)__builtin_bit_cast(uint64_t, ev.gr[i]));
        sums += i ? "," : "";
        sums += b;
      }
      unsigned long long ck[3];
      HIPC(c_, hipMemcpyAsync(ck, cks, sizeof ck, hipMemcpyDeviceToHost, c_->stream));
      sync(c_);
      trace_line("ctx %p tag %016llx seq %lld prec %d iters %lld restarts %d late %d relres %.17g rhs %016llx "
                 "phi0 %016llx phi1 %016llx ckrhs %016llx ckphi0 %016llx ckphi1 %016llx cg %s upd %s\n",
                 (void*)c_, (unsigned long long)c_->trace_tag, c_->trace_seq++, P_->precision, ps.iters, ps.restarts,
                 ps.late, ps.relres, (unsigned long long)h_rhs, (unsigned long long)h_phi0,
                 (unsigned long long)h_phi1, ck[0], ck[1], ck[2], ps.verdicts.c_str(), sums.c_str());
    }
    time_grad_ += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t1).count();
    counts_.grad_evals++;
    counts_.matvec_fp64++;
    for (int i = 0; i < G_NRED; ++i)
      if (!std::isfinite(ev.gr[i])) bad_ = true;
    if (bad_ && c_->progress) {
      std::fprintf(stderr, "alofdft: non-finite residual sums:");
      for (int i = 0; i < G_NRED; ++i) std::fprintf(stderr, " %.3e", ev.gr[i]);
      std::fprintf(stderr, " | density sums:");
      for (int i = 0; i < kUpdRed; ++i) std::fprintf(stderr, " %.3e", ev.upd[i]);
      std::fprintf(stderr, "\n");
    }
  }

  // Evaluation that must be finite (start point, new outer step, single evaluations).
  void require_finite(const char* what) {
    if (bad_) {
      set_err(c_, "non-finite value in %s", what);
      throw Fail{ALOFDFT_NUMERICAL};
    }
  }

  double C_of(const Eval& e) const { return e.upd[0] - S_->N_elec; }
  double energy(const Eval& e, alofdft_energy* out = nullptr) const {
    const double ETF = CF_ * h3_ * e.gr[G_TF];
    const double EvW = -0.5 * P_->lambda * h3_ * e.gr[G_VW];
    const double Exc = h3_ * e.gr[G_XC];
    const double Ees = 0.5 * h3_ * e.gr[G_ES] - E_self_;
    const double E = ETF + EvW + Exc + Ees + E_c_;
    if (out) {
      out->E_TF = ETF;
      out->E_vW = EvW;
      out->E_xc = Exc;
      out->E_es = Ees;
      out->E_self = E_self_;
      out->E_corr = E_c_;
      out->E_total = E;
      out->C_h = C_of(e);
      out->grad_norm = std::sqrt(h3_ * e.gr[G_GG]);
    }
    return E;
  }

  // Nonlinear CG on L(.; eta, mu) (see the line-search reading in DESIGN notes of
  // the oracle: secant on the derivative along |u + t d|, bracketed).  On entry
  // `cur` holds the evaluation at v (which is the current point).
  int nlcg(double eta, double mu, Eval& cur, double& gnorm, long long& its) {
    double gn = std::sqrt(h3_ * cur.gr[G_GG]);
    // s_cur_ holds -g/M of the current point; first direction d = s
    double delta_new = -cur.gr[G_GS_NEW];
    double beta = 0.0;
    bool restart = true;
    int since_restart = 0;
    int status = 1;
    its = 0;
    double gd_unsigned = cur.gr[G_GD];
    for (;;) {
      check_cancel(c_);
      if (!std::isfinite(gn)) { status = ALOFDFT_NUMERICAL; break; }
      if (gn < P_->tol_grad) { status = 0; break; }
      if (its >= P_->max_inner) { status = 1; break; }
      // direction d = s + beta d (beta = 0 on restart); derivative at t = 0
      double slope0 = -delta_new + (restart ? 0.0 : beta * gd_unsigned);
      if (!restart && !(slope0 < 0.0)) {
        restart = true;
        since_restart = 0;
        slope0 = -delta_new;
      }
      const double bet = restart ? 0.0 : beta;
      if (restart) {
        // d = s: DirOp with beta 0 overwrites d
      }
      // first probe fused with the direction update and the projection u = |v|
      Eval ev;
      double t_cur = P_->sigma0;
      eval_trial(t_cur, eta, mu, true, bet, ev);
      double s_cur = ev.gr[G_SLOPE];
      double a = 0.0, b = INFINITY, t_prev = 0.0, s_prev = slope0;
      // a non-finite trial overshot: it closes the bracket from above
      if (s_cur > 0.0 || bad_) b = t_cur; else a = t_cur;
      for (int j = 0; j < P_->max_secant || bad_; ++j) {
        if (bad_) {
          if (j > 60) break;
          t_prev = a;
          s_prev = slope0;
          t_cur = 0.5 * (a + b);
          eval_trial(t_cur, eta, mu, false, 0.0, ev);
          s_cur = ev.gr[G_SLOPE];
          if (s_cur > 0.0 || bad_) b = t_cur; else a = t_cur;
          continue;
        }
        if (std::fabs(s_cur) <= P_->secant_rel * std::fabs(slope0)) break;
        const double curv = (s_cur - s_prev) / (t_cur - t_prev);
        double t_new = curv > 0.0 ? t_cur - s_cur / curv : NAN;
        const double hi = std::isfinite(b) ? b : 4.0 * std::max(a, t_cur);
        if (!(t_new > a && t_new < hi)) t_new = std::isfinite(b) ? 0.5 * (a + b) : 2.0 * std::max(a, t_cur);
        t_prev = t_cur;
        s_prev = s_cur;
        t_cur = t_new;
        eval_trial(t_cur, eta, mu, false, 0.0, ev);
        s_cur = ev.gr[G_SLOPE];
        if (s_cur > 0.0 || bad_) b = std::min(b, t_cur); else a = std::max(a, t_cur);
      }
      if (bad_) {
        if (bet != 0.0) {
          // no finite point along the conjugate direction: search again from the same
          // point along s (v back to the start point, phi to its potential, the s
          // buffers to their order before this line)
          if (c_->progress) std::fprintf(stderr, "alofdft: NLCG step %lld: conjugate direction overflowed, restart\n", its);
          CombineOp cv{v_, us_, nullptr, nullptr, 1.0, 0.0, 0.0, nullptr};
          launch_pw(c_, g_, cv);
          CombineOp cp{phi_, ph_[0], nullptr, nullptr, 1.0, 0.0, 0.0, nullptr};
          launch_pw(c_, g_, cp);
          std::swap(s_cur_, s_prev_);
          restart = true;
          since_restart = 0;
          continue;
        }
        set_err(c_, "no finite point along the search direction (NLCG step %lld, last t %.3e, bracket [%.3e, %.3e])",
                its, t_cur, a, b);
        throw Fail{ALOFDFT_NUMERICAL};
      }
      cur = ev;
      gn = std::sqrt(h3_ * cur.gr[G_GG]);
      const double delta_old = delta_new;
      const double delta_mid = -cur.gr[G_GS_OLD];
      delta_new = -cur.gr[G_GS_NEW];
      beta = (delta_new - delta_mid) / delta_old;
      gd_unsigned = cur.gr[G_GD];
      ++since_restart;
      // restart also when successive residuals have lost orthogonality (Powell's test,
      // |r_new . s_old| >= 0.2 r_new . s_new), before the direction can run away
      restart = since_restart >= P_->restart_every || beta <= 0.0 || std::fabs(delta_mid) >= 0.2 * delta_new;
      if (restart) since_restart = 0;
      ++its;
      if (c_->progress && its % 100 == 0)
        std::fprintf(stderr, "alofdft: nlcg step %lld |g| %.3e cg %lld\n", its, gn, counts_.cg_iters);
    }
    gnorm = gn;
    return status;
  }

  int run(alofdft_result* res) {
    auto t0 = std::chrono::steady_clock::now();
    counts_ = alofdft_counts{};
    Eval cur;
    int status = ALOFDFT_NOT_CONVERGED;
    double gn = 0.0, dE = 0.0, eta = 0.0, eta_star = 0.0;
    if (P_->method == ALOFDFT_METHOD_LAGRANGE) {
      status = lagrange(cur, eta_star, gn);
      time_setup_ = 0.0;
    } else {
      status = augmented_lagrangian(cur, eta_star, gn, dE, t0);
    }
    if (status == ALOFDFT_OK && poisson_capped_) status = ALOFDFT_NOT_CONVERGED;
    (void)eta;
    return finish(res, cur, status, eta_star, dE, gn);
  }

  // Host sums of a pointwise pass: finalize the block partials (scaled by scale) and copy
  // the first n to the host.
  template <class Op>
  void reduce_pw(const Op& op, int n, double scale, double* out) {
    const int nb = launch_pw(c_, g_, op);
    double* dst = scal_ + kUpdRed + G_NRED;
    finalize(c_, op.parts_out, nb, Op::NRED, scale, dst);
    HIPC(c_, hipMemcpyAsync(c_->pin, dst, sizeof(double) * n, hipMemcpyDeviceToHost, c_->stream));
    sync(c_);
    std::memcpy(out, c_->pin, sizeof(double) * n);
  }

  // Lagrange-multiplier method (Sec. 5.3.2): u stays on h^3 sum u^2 = N, the multiplier is
  // the Rayleigh quotient eta = h^3 u.g / N of the residual g = H u (no multiplier terms),
  // Polak-Ribiere directions built from gp = g - eta u are projected orthogonal to u, and
  // each step minimises the energy along the great circle u cos t + sqrt(N) d sin t
  // (d normalised to h^3 d.d = 1) with Brent's method.  Converged at ||gp|| < tol_grad.
  int lagrange(Eval& cur, double& eta, double& gn) {
    const double Ne = S_->N_elec, sN = std::sqrt(Ne);
    const double M = vw_diag_;  // constant Jacobi scaling (diagonal of -(lambda/2) Delta_h)
    double* g = gridbuf<double>(c_, "lm.g", g_);
    double* gpb[2] = {gridbuf<double>(c_, "lm.gp0", g_), gridbuf<double>(c_, "lm.gp1", g_)};
    double* parts = bufT<double>(c_, "lm.parts", (size_t)kPointwiseBlocks * 2);
    gout_ = g;
    // start on the constraint surface: u = |u0| sqrt(N / h^3 sum u0^2)
    double nrm;
    reduce_pw(AbsOp{us_, us_, 1.0, parts}, 1, h3_, &nrm);
    require(c_, nrm > 0 && std::isfinite(nrm), "the initial guess has no finite norm");
    reduce_pw(AbsOp{us_, us_, std::sqrt(Ne / nrm), parts}, 1, h3_, &nrm);
    double* zero = zero_dir();
    auto eval_at = [&](double a, double t, Eval& ev) {  // v = a u + t d, energies and residual at |v|
      TrialOp op{us_, t == 0.0 ? zero : d_, b_, v_, t, frame_, partsU_};
      op.a = a;
      nU_ = launch_pw(c_, g_, op);
      bad_ = false;
      eval_at_v(0.0, 0.0, ev);
    };
    double delta_new = 1.0;
    int status = ALOFDFT_NOT_CONVERGED, since_restart = 0, cur_gp = 0;
    long long it = 0;
    for (;;) {
      check_cancel(c_);
      eval_at(1.0, 0.0, cur);
      require_finite("the residual of the Lagrange-multiplier method");
      eta = h3_ * cur.gr[G_UG] / Ne;
      double sums[2];
      reduce_pw(LMResidualOp{g, us_, gpb[cur_gp], it > 0 ? gpb[cur_gp ^ 1] : nullptr, eta, parts}, 2, 1.0, sums);
      gn = std::sqrt(h3_ * sums[0]);
      if (!std::isfinite(gn)) { status = ALOFDFT_NUMERICAL; break; }
      if (gn < P_->tol_grad) { status = ALOFDFT_OK; break; }
      if (it >= P_->max_inner) break;
      const double delta_old = delta_new, delta_mid = sums[1] / M;
      delta_new = sums[0] / M;
      double beta = it == 0 ? 0.0 : (delta_new - delta_mid) / delta_old;
      ++since_restart;
      if (it == 0 || beta <= 0.0 || since_restart >= P_->restart_every) {
        beta = 0.0;
        since_restart = 0;
      }
      double ud, gd[2];
      reduce_pw(LMDirectionOp{gpb[cur_gp], us_, d_, 1.0 / M, beta, parts}, 1, h3_, &ud);
      reduce_pw(LMProjectOp{g, us_, d_, ud / Ne, parts}, 2, h3_, gd);
      if (gd[0] >= 0.0) {  // not a descent direction: steepest descent
        reduce_pw(LMDirectionOp{gpb[cur_gp], us_, d_, 1.0 / M, 0.0, parts}, 1, h3_, &ud);
        reduce_pw(LMProjectOp{g, us_, d_, ud / Ne, parts}, 2, h3_, gd);
        since_restart = 0;
      }
      const double dn = std::sqrt(gd[1]);
      const double E0 = energy(cur);
      // energy along the circle: u(t) = u cos t + sqrt(N) (d/dn) sin t
      Eval ev;
      auto E_at = [&](double t) {
        eval_at(std::cos(t), sN * std::sin(t) / dn, ev);
        return bad_ ? HUGE_VAL : energy(ev);
      };
      const double slope = 2.0 * sN * gd[0] / dn;  // dE/dt at t = 0
      double ta = 0.0, tb = std::min(0.5, std::fabs(slope) / (2.0 * M * Ne) + 1e-6), fb = E_at(tb), tc, fc;
      bool bracketed = true;
      if (fb > E0) {  // shorten the probe until it lies below E0
        tc = tb;
        int guard = 0;
        do {
          tb *= 0.5;
          fb = E_at(tb);
          if (fb > E0) tc = tb;
        } while (fb > E0 && ++guard < 40);
        bracketed = fb <= E0;
      } else {  // lengthen it while the energy falls
        tc = 2.0 * tb;
        fc = E_at(tc);
        int guard = 0;
        while (fc < fb && ++guard < 40) {
          ta = tb;
          tb = tc;
          fb = fc;
          tc *= 2.0;
          fc = E_at(tc);
        }
      }
      if (!bracketed) break;  // no lower energy along the direction: rounding floor
      const double t = brent_minimise(E_at, ta, tc, tb, fb, 1e-8, 60);
      // accept: u = |u cos t + sqrt(N) dhat sin t|
      TrialOp op{us_, d_, b_, v_, sN * std::sin(t) / dn, frame_, partsU_};
      op.a = std::cos(t);
      launch_pw(c_, g_, op);
      reduce_pw(AbsOp{us_, v_, 1.0, parts}, 1, h3_, &nrm);
      cur_gp ^= 1;
      ++it;
      if (c_->progress && it % 20 == 0)
        std::fprintf(stderr, "alofdft: Lagrange step %lld |g - eta u| %.3e E %.12f eta %.10f\n", it, gn, E0, eta);
    }
    counts_.outer = 1;
    counts_.inner = it;
    gout_ = nullptr;
    return status;
  }

  // Algorithm AugLag (Sec. 3) around the nonlinear CG inner solver; the penalty method
  // (Sec. 5.3.2) is the same loop with eta fixed at 0.
  int augmented_lagrangian(Eval& cur, double& eta_star, double& gn, double& dE,
                           std::chrono::steady_clock::time_point t0) {
    // v = u0 (t = 0 trial from u_start = u0, d = 0)
    double eta = P_->method == ALOFDFT_METHOD_PENALTY ? 0.0 : P_->eta0;
    double mu = P_->mu0;
    eval_trial(0.0, eta, mu, false, 0.0, cur);
    require_finite("the residual at the initial guess");
    time_setup_ = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    int status = ALOFDFT_NOT_CONVERGED;
    double E_prev = 0.0;
    eta_star = eta;
    for (int q = 0; q < P_->max_outer; ++q) {
      if (q > 0) eval_at_v_refresh(eta, mu, cur);  // same u, new eta/mu: recompute residual terms
      long long its = 0;
      const int st = nlcg(eta, mu, cur, gn, its);
      counts_.inner += its;
      counts_.outer = q + 1;
      if (st == ALOFDFT_NUMERICAL) {
        status = ALOFDFT_NUMERICAL;
        break;
      }
      const double C = C_of(cur);
      const double E = energy(cur);
      dE = q == 0 ? 0.0 : E - E_prev;
      E_prev = E;
      eta_star = eta - C / mu;  // Algorithm AugLag multiplier update
      if (c_->progress)
        std::fprintf(stderr, "alofdft: AL step %d E %.12f C_h/N %.3e nlcg %lld cg %lld\n", q + 1, E,
                     std::fabs(C) / S_->N_elec, its, counts_.cg_iters);
      // the workloads stop on the constraint; Algorithm AugLag itself on the energy change
      const bool stop = P_->al_stop == ALOFDFT_STOP_ENERGY_CHANGE
                            ? (q > 0 && std::fabs(dE) / S_->M < P_->tol_energy)
                            : std::fabs(C) / S_->N_elec < P_->tol_constraint;
      if (stop && st == 0) {
        status = ALOFDFT_OK;
        break;
      }
      eta = P_->method == ALOFDFT_METHOD_PENALTY ? 0.0 : eta_star;
      mu *= P_->kappa;
    }
    return status;
  }

  int finish(alofdft_result* res, const Eval& cur, int status, double eta_star, double dE, double gn) {
    alofdft_energy en;
    energy(cur, &en);
    en.grad_norm = gn;  // the inner solver's residual norm (for the Lagrange method, of g - eta u)
    res->E_total = en.E_total;
    res->E_TF = en.E_TF;
    res->E_vW = en.E_vW;
    res->E_xc = en.E_xc;
    res->E_es = en.E_es;
    res->E_self = en.E_self;
    res->E_corr = en.E_corr;
    res->eta_star = eta_star;
    res->C_h = en.C_h;
    res->grad_norm = en.grad_norm;
    res->poisson_relres = relres_;
    res->dE_last = dE;
    res->counts = counts_;
    res->time_poisson_ms = time_poisson_;
    res->time_grad_ms = time_grad_;
    res->time_setup_ms = time_setup_;
    res->status = status;
    return status;
  }

  // Re-evaluate the residual at the same v after eta/mu changed (no Poisson
  // solve is needed: phi depends on u only, but the slope/preconditioner sums
  // do).  Implemented as a fresh evaluation at t = 0 of the current point.
  void eval_at_v_refresh(double eta, double mu, Eval& cur) {
    TrialOp op{v_, zero_dir(), b_, v_, 0.0, frame_, partsU_};
    nU_ = launch_pw(c_, g_, op);
    nh_ = 0;
    bad_ = false;
    eval_at_v(eta, mu, cur);
    require_finite("the residual at a new outer step");
  }

  double* zero_dir() {
    double* z = gridbuf<double>(c_, "s.zero", g_);
    return z;
  }

  // projection u = |v| into the dense output
  void output(double* u_dense_dev, double* phi_dense_dev) {
    if (u_dense_dev) unpack<double, double>(c_, g_, v_, u_dense_dev, 1);
    if (phi_dense_dev) unpack<double, double>(c_, g_, phi_, phi_dense_dev, 0);
  }

  void forces(double* out) {
    std::vector<double> f, fc;
    atom_sums(c_, g_, S_, at_, pseudo_, P_->fd_half_width, phi_, nullptr, &f);
    overlap_correction(S_, P_->gauss_width, &fc);
    for (int i = 0; i < 3 * S_->M; ++i) out[i] = h3_ * f[i] + fc[i];
  }

  const Geom& geom() const { return g_; }
  double* phi() { return phi_; }
  double* v() { return v_; }
  double* b() { return b_; }
  double E_self() const { return E_self_; }
  double E_c() const { return E_c_; }
  void set_gout(double* p) { gout_ = p; }
  const alofdft_counts& counts() const { return counts_; }

 private:
  double* s_new() { return s_cur_ ? sb_ : sa_; }
  double* s_old() { return s_cur_ ? sa_ : sb_; }
  alofdft_ctx* c_;
  const alofdft_system* S_;
  const alofdft_params* P_;
  Geom g_;
  double h3_;
  double *us_, *v_, *d_, *sa_, *sb_, *b_, *phi_, *rhs_, *partsU_, *partsG_, *scal_;
  // potentials already solved along the current line, for warm starts: the charge
  // (u_start + t d)^2 + b is quadratic in t (also under |.|), so phi(t) is too
  double* ph_[3];
  double th_[3];
  int nh_ = 0;
  bool bad_ = false;  // the last evaluation produced a non-finite value
  double* gout_ = nullptr;
  int s_cur_ = 0, s_prev_ = 1;
  int nU_ = 0;
  double vw_diag_, CF_;
  StencilW<double> Wlap_;
  BoxFrame frame_;
  DevAtoms at_;
  PseudoDev pseudo_{};
  double E_self_ = 0.0, E_c_ = 0.0;
  alofdft_counts counts_{};
  double relres_ = 0.0;
  bool poisson_capped_ = false;
  double time_poisson_ = 0.0, time_grad_ = 0.0, time_setup_ = 0.0;
};

int guarded(alofdft_ctx* c, const std::function<int()>& f);

}  // namespace

// ----------------------------------------------------------------- allocation-free scratch
// Scratch memory of alofdft_apply_laplacian_noalloc: the padded copies of x and y.  A
// file-scope device array of fixed size, held by every device the library runs on until
// the process ends.  In host code `scratch` names a host-side stand-in, never the device
// memory: its device address is taken once per device with hipGetSymbolAddress (with that
// device current) when a context is created there, and only that address is passed on.
constexpr size_t kScratchBytes = 64ull << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on `dev` (the current device), resolved once per device.
int resolve_scratch(alofdft_ctx* c, int dev) {
  require(c, dev >= 0 && dev < kMaxDevices, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    HIPC(c, hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    require(c, ptr != nullptr, "no device address for the scratch array");
    g_scratch_ptr[dev] = ptr;
  }
  return ALOFDFT_OK;
}

void* scratch_ptr(int dev) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return dev >= 0 && dev < kMaxDevices ? g_scratch_ptr[dev] : nullptr;
}

}  // namespace

// ================================================================= C ABI
namespace {

int guarded(alofdft_ctx* c, const std::function<int()>& f) {
  try {
    if (c) {
      hipError_t e = hipSetDevice(c->device);
      if (e != hipSuccess) {
        set_err(c, "hipSetDevice(%d): %s", c->device, hipGetErrorString(e));
        return ALOFDFT_DEVICE_ERROR;
      }
    }
    return f();
  } catch (const Fail& e) {
    return e.code;
  } catch (const std::bad_alloc&) {
    set_err(c, "host allocation failed");
    return ALOFDFT_OUT_OF_MEMORY;
  } catch (...) {
    set_err(c, "unexpected exception");
    return ALOFDFT_DEVICE_ERROR;
  }
}

// Default initial guess u0 = sqrt(N/V)(1 + 0.05 xi), xi = 2 U(SplitMix64(seed ^ i)) - 1.
std::vector<double> default_u0(const alofdft_system* s, uint64_t seed) {
  const long long n = (long long)s->n[0] * s->n[1] * s->n[2];
  const double V = (double)n * s->h * s->h * s->h;
  const double a = std::sqrt(s->N_elec / V);
  std::vector<double> u(n);
  for (long long i = 0; i < n; ++i) {
    const uint64_t z = splitmix64(seed ^ (uint64_t)i);
    const double xi = 2.0 * ((double)(z >> 11) * 0x1.0p-53) - 1.0;
    u[i] = a * (1.0 + 0.05 * xi);
  }
  return u;
}

long long npoints(const int n[3]) { return (long long)n[0] * n[1] * n[2]; }

int solve_impl(alofdft_ctx* c, const alofdft_system* sys, const alofdft_params* prm, const double* u0_dev,
               const double* u0_host, double* u_out_dev, double* phi_out_dev, double* forces, alofdft_result* res,
               bool warm_phi = false) {
  require(c, res != nullptr, "result pointer is null");
  std::memset(res, 0, sizeof(*res));
  validate(c, sys, prm);
  auto t0 = std::chrono::steady_clock::now();
  const long long n = npoints(sys->n);
  double* u0 = bufT<double>(c, "io.u0", (size_t)n);
  if (u0_dev) {
    HIPC(c, hipMemcpyAsync(u0, u0_dev, sizeof(double) * n, hipMemcpyDeviceToDevice, c->stream));
  } else if (!u0_host && prm->initial_guess == ALOFDFT_GUESS_ATOMIC) {
    atomic_guess_dev(c, sys, prm, u0);
  } else {
    std::vector<double> h = u0_host ? std::vector<double>(u0_host, u0_host + n) : default_u0(sys, prm->seed);
    for (double x : h) require(c, std::isfinite(x), "non-finite initial guess");
    HIPC(c, hipMemcpyAsync(u0, h.data(), sizeof(double) * n, hipMemcpyHostToDevice, c->stream));
    sync(c);
  }
  if (c->trace) {
    // tag: hash of the system and the parameters that shape the solve
    uint64_t x = 1469598103934665603ull;
    auto mix = [&](const void* p, size_t n) {
      const unsigned char* b = (const unsigned char*)p;
      for (size_t i = 0; i < n; ++i) x = (x ^ b[i]) * 1099511628211ull;
    };
    mix(sys->n, sizeof(sys->n));
    mix(&sys->h, sizeof(double));
    mix(sys->origin, sizeof(sys->origin));
    mix(sys->R, sizeof(double) * 3 * sys->M);
    mix(sys->Z, sizeof(double) * sys->M);
    mix(&prm->precision, sizeof(int));
    c->trace_tag = x;
    c->trace_seq = 0;
  }
  Solver S(c, sys, prm);
  S.setup(u0, true, warm_phi);
  int st = S.run(res);
  S.output(u_out_dev, phi_out_dev);
  if (forces) S.forces(forces);
  sync(c);
  res->time_total_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return st;
}

// ----------------------------------------------------------------- relaxation of the nuclei
// Ground-state configuration of the nuclei (Sec. 4): Polak-Ribiere nonlinear CG over the
// 3M positions with a secant line search, on E(R) (the ground-state energy) whose
// gradient is -F(R).  Every evaluation is a full solve at that geometry, warm-started from
// the last u and, on the same grid, the last phi.  Steps are capped so that no atom moves
// more than max_move and every r_cut ball stays in the box.
int relax_impl(alofdft_ctx* c, const alofdft_system* sys, const alofdft_params* prm, const alofdft_relax_params* rp,
               const double* u0_host, double* R_out, double* forces_out, alofdft_result* res,
               alofdft_relax_info* info) {
  require(c, rp && R_out && res && info, "null argument");
  require(c, rp->ftol > 0 && rp->max_move > 0 && rp->probe > 0 && rp->max_steps >= 1 && rp->max_secant >= 1 &&
                 rp->secant_rel > 0 && rp->secant_rel < 1,
          "relaxation parameters out of range");
  validate(c, sys, prm);
  std::memset(info, 0, sizeof(*info));
  const int M = sys->M, D = 3 * M;
  const long long n = npoints(sys->n);
  double* udev = bufT<double>(c, "relax.u", (size_t)n);
  std::vector<double> R(sys->R, sys->R + D), F(D), Ft(D), Rt(D), d(D), Fold(D);
  alofdft_result r{};
  bool first = true;
  auto evaluate = [&](const std::vector<double>& X, std::vector<double>& G, alofdft_result& out) {
    alofdft_system s = *sys;
    s.R = X.data();
    const int st = solve_impl(c, &s, prm, first ? nullptr : udev, first ? u0_host : nullptr, udev, nullptr, G.data(),
                              &out, !first);
    first = false;
    info->solves++;
    if (st < 0) throw Fail{st};  // the solve's own status and message
    return st;
  };
  auto dot = [&](const std::vector<double>& a, const std::vector<double>& b) {
    double t = 0.0;
    for (int i = 0; i < D; ++i) t += a[i] * b[i];
    return t;
  };
  auto fmax_of = [&](const std::vector<double>& G) {
    double m = 0.0;
    for (int J = 0; J < M; ++J)
      m = std::max(m, std::sqrt(G[3 * J] * G[3 * J] + G[3 * J + 1] * G[3 * J + 1] + G[3 * J + 2] * G[3 * J + 2]));
    return m;
  };
  // largest step along d keeping every atom's move <= max_move and its r_cut ball in the box
  auto max_alpha = [&](const std::vector<double>& X, const std::vector<double>& dir) {
    double dmax = 0.0, amax = HUGE_VAL;
    for (int J = 0; J < M; ++J) {
      const double* v = &dir[3 * J];
      dmax = std::max(dmax, std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]));
      for (int a = 0; a < 3; ++a) {
        const double lo = sys->origin[a] + prm->r_cut, hi = sys->origin[a] + (sys->n[a] - 1) * sys->h - prm->r_cut;
        const double x = X[3 * J + a], va = v[a];
        if (va > 0) amax = std::min(amax, (hi - x) / va);
        if (va < 0) amax = std::min(amax, (lo - x) / va);
      }
    }
    return std::make_pair(dmax, std::min(amax, dmax > 0 ? rp->max_move / dmax : 0.0));
  };

  int st = evaluate(R, F, r);
  for (int i = 0; i < D; ++i) d[i] = F[i];
  int status = ALOFDFT_NOT_CONVERGED;
  for (int step = 0; step < rp->max_steps; ++step) {
    info->fmax = fmax_of(F);
    if (info->fmax < rp->ftol) { status = ALOFDFT_OK; break; }
    info->steps = step + 1;
    // secant on the directional derivative g(a) = -F(R + a d) . d, from g(0) < 0
    const auto [dmax, amax] = max_alpha(R, d);
    if (!(amax > 0)) break;  // an atom sits at the edge of the admissible region along d
    const double g0 = -dot(F, d);
    double a_prev = 0.0, g_prev = g0;
    double a = std::min(rp->probe / dmax, amax);
    for (int j = 0; j < rp->max_secant; ++j) {
      for (int i = 0; i < D; ++i) Rt[i] = R[i] + a * d[i];
      st = evaluate(Rt, Ft, r);
      const double g = -dot(Ft, d);
      if (std::fabs(g) <= rp->secant_rel * std::fabs(g0) || j == rp->max_secant - 1) break;
      double an = a - g * (a - a_prev) / (g - g_prev);
      // a curvature of the wrong sign or a root beyond the cap: expand towards the cap
      if (!std::isfinite(an) || g - g_prev <= 0.0 || an > amax) an = std::min(2.0 * a, amax);
      if (an <= 0.0) an = 0.5 * a;
      if (an == a) break;
      a_prev = a;
      g_prev = g;
      a = an;
    }
    // accept the last evaluated point (its forces are known)
    Fold = F;
    R = Rt;
    F = Ft;
    // Polak-Ribiere with restart when the new direction is not a descent direction
    const double den = dot(Fold, Fold);
    double beta = den > 0 ? (dot(F, F) - dot(F, Fold)) / den : 0.0;
    beta = std::max(0.0, beta);
    for (int i = 0; i < D; ++i) d[i] = F[i] + beta * d[i];
    if (dot(F, d) <= 0.0)
      for (int i = 0; i < D; ++i) d[i] = F[i];
  }
  info->fmax = fmax_of(F);
  if (info->fmax < rp->ftol) status = ALOFDFT_OK;
  std::copy(R.begin(), R.end(), R_out);
  if (forces_out) std::copy(F.begin(), F.end(), forces_out);
  *res = r;
  info->E_total = r.E_total;
  info->status = st != 0 ? st : status;
  return info->status;
}

// ----------------------------------------------------------------- serving
size_t footprint(const alofdft_system* s, const alofdft_params* p) {
  const Geom g = make_geom(s->n, p->fd_half_width);
  const size_t T = (size_t)g.total;
  const size_t n = (size_t)s->n[0] * s->n[1] * s->n[2];
  // solver arrays (12), FP64 CG (7: every schedule's work arrays), refinement residual (1): double;
  // FP32 CG (7) + correction (1): float
  // (+3 for the Lagrange method's residual arrays, +1 for the atomic guess's density)
  const size_t extra = (p->method == ALOFDFT_METHOD_LAGRANGE ? 3 : 0) + (p->initial_guess == ALOFDFT_GUESS_ATOMIC ? 1 : 0);
  const size_t arrays = (12 + 7 + 1 + extra) * 8 * T + (7 + 1) * 4 * T;
  const size_t dense = 3 * 8 * n;  // initial guess, u and phi outputs
  // block partials, scalars, atom arrays and the cell list (with slack)
  const size_t small = (size_t)(max_stencil_blocks(g, 4096) + 4 * kPointwiseBlocks) * 16 * 8 + 128 * (size_t)s->M +
                       (size_t)(1 << 20);
  return arrays + dense + small;
}

size_t held_bytes(const alofdft_ctx* c) {
  size_t b = 0;
  for (auto& kv : c->bufs) b += kv.second.second;
  return b;
}

void free_all(alofdft_ctx* c) {
  (void)hipStreamSynchronize(c->stream);
  for (auto& kv : c->bufs) (void)hipFree(kv.second.first);
  c->bufs.clear();
  c->geom_key.clear();
}

struct Request {
  uint64_t id = 0;
  alofdft_system sys{};
  std::vector<double> R, Z;
  alofdft_params prm{};
  size_t fp = 0;
  std::chrono::steady_clock::time_point t_submit, t_start, t_end;
  int status = ALOFDFT_PENDING;
  int slot = -1;  // slot running it, -1 while queued
  alofdft_result res{};
  std::vector<double> u, forces;
};

}  // namespace

struct alofdft_server {
  int device = 0;
  size_t budget = 0;
  std::vector<alofdft_ctx*> ctx;
  std::vector<hipStream_t> streams;
  std::vector<size_t> held;  // bytes of cached work arrays each slot's context holds
  std::vector<std::shared_ptr<Request>> current;  // request each slot runs (null when idle)
  std::vector<std::thread> workers;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<std::shared_ptr<Request>> queue;
  std::map<uint64_t, std::shared_ptr<Request>> reqs;
  size_t reserved = 0;  // footprints of the running requests
  bool trim = false;    // the front request does not fit: idle slots drop their cached arrays
  int running = 0;
  bool stop = false;
  uint64_t next_id = 1;
  long long submitted = 0, admitted = 0, completed = 0, rejected = 0, cancelled = 0;
  std::vector<double> lat_ms;
  bool have_first = false;
  std::chrono::steady_clock::time_point first_submit, last_end;
};

namespace {

// Device bytes the server may occupy if a request of footprint fp is admitted: every
// slot's cached arrays, the full footprint of every running request, and fp.  Cached
// arrays the request may reuse are counted twice, so the bound is conservative; a request
// that does not fit makes the idle slots drop their caches (trim), after which it fits as
// soon as the running requests leave room (fp alone never exceeds the budget).
size_t demand(const alofdft_server* s, size_t fp) {
  size_t tot = s->reserved + fp;
  for (size_t h : s->held) tot += h;
  return tot;
}

void worker_loop(alofdft_server* s, int w) {
  alofdft_ctx* c = s->ctx[w];
  (void)hipSetDevice(s->device);
  for (;;) {
    std::shared_ptr<Request> r;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      for (;;) {
        if (s->stop && s->queue.empty()) return;
        if (!s->queue.empty()) {
          if (demand(s, s->queue.front()->fp) <= s->budget) break;
          if (!s->trim) {
            s->trim = true;
            s->cv.notify_all();  // wake the other idle slots to drop their caches too
          }
        }
        if (s->trim && s->held[w] > 0) {
          // drop this idle slot's cached arrays; they count in the demand until freed
          lk.unlock();
          free_all(c);
          lk.lock();
          s->held[w] = 0;
          s->cv.notify_all();
          continue;
        }
        s->cv.wait(lk);
      }
      r = s->queue.front();
      s->queue.pop_front();
      s->trim = false;
      s->reserved += r->fp;
      r->slot = w;
      s->current[w] = r;
      c->cancel.store(0);  // a cancellation meant for the previous request on this slot
      s->running++;
      s->admitted++;
    }
    r->t_start = std::chrono::steady_clock::now();
    const long long n = npoints(r->sys.n);
    r->u.assign((size_t)n, 0.0);
    r->forces.assign(3 * (size_t)r->sys.M, 0.0);
    int st = guarded(c, [&]() {
      double* du = bufT<double>(c, "io.uout", (size_t)n);
      int rc = solve_impl(c, &r->sys, &r->prm, nullptr, nullptr, du, nullptr, r->forces.data(), &r->res);
      HIPC(c, hipMemcpyAsync(r->u.data(), du, sizeof(double) * n, hipMemcpyDeviceToHost, c->stream));
      sync(c);
      return rc;
    });
    r->t_end = std::chrono::steady_clock::now();
    {
      std::lock_guard<std::mutex> lk(s->mu);
      s->held[w] = held_bytes(c);
      s->reserved -= r->fp;
      s->current[w] = nullptr;
      s->running--;
      r->status = st;
      r->res.status = st;
      if (st == ALOFDFT_CANCELLED) {
        s->cancelled++;
      } else {
        s->completed++;
        s->lat_ms.push_back(std::chrono::duration<double, std::milli>(r->t_end - r->t_submit).count());
        s->last_end = r->t_end;
      }
    }
    s->cv.notify_all();
  }
}

}  // namespace

extern "C" {

const char* alofdft_strerror(int s) {
  switch (s) {
    case ALOFDFT_OK: return "ok";
    case ALOFDFT_NOT_CONVERGED: return "not converged (outputs hold the last iterate)";
    case ALOFDFT_PENDING: return "pending";
    case ALOFDFT_INVALID_ARGUMENT: return "invalid argument";
    case ALOFDFT_OUT_OF_MEMORY: return "out of memory";
    case ALOFDFT_DEVICE_ERROR: return "device error";
    case ALOFDFT_NUMERICAL: return "non-finite value";
    case ALOFDFT_REJECTED: return "rejected";
    case ALOFDFT_CANCELLED: return "cancelled";
  }
  return "unknown status";
}

const char* alofdft_last_error(const alofdft_ctx* c) { return c ? c->err.c_str() : "null context"; }

int alofdft_default_params(alofdft_params* p) {
  if (!p) return ALOFDFT_INVALID_ARGUMENT;
  std::memset(p, 0, sizeof(*p));
  p->fd_half_width = 6;
  p->lambda = 0.2;
  p->xc = ALOFDFT_XC_LDA_PZ;
  p->gauss_width = 1.0;
  p->r_cut = 7.0;
  p->method = ALOFDFT_METHOD_AUGMENTED_LAGRANGIAN;
  p->eta0 = -0.2;
  p->mu0 = 1.0;
  p->kappa = 0.1;
  p->tol_constraint = 1e-8;
  p->tol_grad = 1e-6;
  p->tol_poisson = 1e-10;
  p->phi_bc = ALOFDFT_BC_MULTIPOLE;
  p->precision = ALOFDFT_FP64;
  p->max_outer = 30;
  p->max_inner = 20000;
  p->max_cg = 100000;
  p->sigma0 = 0.5;
  p->max_secant = 4;
  p->secant_rel = 0.1;
  p->restart_every = 50;
  p->cg_check_every = kCheckEvery;
  p->seed = 6456;
  p->pseudocharge = ALOFDFT_PSEUDO_GAUSSIAN;
  p->initial_guess = ALOFDFT_GUESS_UNIFORM;
  p->guess_width = 1.5;
  p->guess_floor = 1e-3;
  p->al_stop = ALOFDFT_STOP_CONSTRAINT;
  p->tol_energy = 3.6749e-6;
  p->domain = ALOFDFT_DOMAIN_BOX;
  return ALOFDFT_OK;
}

int alofdft_create(alofdft_ctx** out, int hip_device, void* hip_stream) {
  if (!out) return ALOFDFT_INVALID_ARGUMENT;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || hip_device < 0 || hip_device >= ndev) return ALOFDFT_DEVICE_ERROR;
  alofdft_ctx* c = new (std::nothrow) alofdft_ctx();
  if (!c) return ALOFDFT_OUT_OF_MEMORY;
  c->device = hip_device;
  c->stream = (hipStream_t)hip_stream;
  c->progress = std::getenv("ALOFDFT_PROGRESS") != nullptr;
  if (const char* tp = std::getenv("ALOFDFT_TRACE")) {
    std::lock_guard<std::mutex> lk(g_trace_mu);
    if (!g_trace_file) g_trace_file = std::fopen(tp, "a");
    c->trace = g_trace_file != nullptr;
    c->trace_hash = c->trace && std::getenv("ALOFDFT_TRACE_HASH") != nullptr;
  }
  int st = guarded(c, [&]() {  // guarded makes hip_device current
    HIPC(c, hipHostMalloc((void**)&c->pin, 4096, hipHostMallocDefault));
    HIPC(c, hipEventCreate(&c->ev0));
    HIPC(c, hipEventCreate(&c->ev1));
    return resolve_scratch(c, hip_device);
  });
  if (st != ALOFDFT_OK) {
    alofdft_destroy(c);
    return st;
  }
  *out = c;
  return ALOFDFT_OK;
}

void alofdft_destroy(alofdft_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  if (c->stream) (void)hipStreamSynchronize(c->stream); else (void)hipDeviceSynchronize();
  for (auto& kv : c->bufs) (void)hipFree(kv.second.first);
  if (c->pin) (void)hipHostFree(c->pin);
  if (c->ev0) (void)hipEventDestroy(c->ev0);
  if (c->ev1) (void)hipEventDestroy(c->ev1);
  for (auto& pr : c->prof_pool) {
    (void)hipEventDestroy(pr.first);
    (void)hipEventDestroy(pr.second);
  }
  delete c;
}

int alofdft_set_tuning(alofdft_ctx* c, int stencil_variant, int target_blocks, int inner_tol_exp) {
  const bool var_ok = (stencil_variant >= -1 && stencil_variant <= 19) || (stencil_variant >= 100 && stencil_variant <= 119);
  if (!c || !var_ok || target_blocks < 0 || inner_tol_exp < 1 || inner_tol_exp > 7)
    return ALOFDFT_INVALID_ARGUMENT;
  c->variant = stencil_variant;
  c->target_blocks = target_blocks;
  c->inner_tol_exp = inner_tol_exp;
  return ALOFDFT_OK;
}

int alofdft_set_cg_schedule(alofdft_ctx* c, int schedule) {
  if (!c || schedule < -1 || schedule > 2) return ALOFDFT_INVALID_ARGUMENT;
  c->cg_schedule = schedule;
  return ALOFDFT_OK;
}

int alofdft_profile_cg_kernel(alofdft_ctx* c, int sample_every) {
  if (!c || sample_every < 0) return ALOFDFT_INVALID_ARGUMENT;
  c->prof_every = sample_every;
  for (int i = 0; i < 2; ++i) {
    c->prof_count[i] = 0;
    c->prof_ms[i] = 0.0;
    c->prof_ms_first[i] = 0.0;
    c->prof_ms_second[i] = 0.0;
    c->prof_points[i] = 0;
    c->prof_sched[i] = -1;
  }
  return ALOFDFT_OK;
}

int alofdft_cg_kernel_stats(alofdft_ctx* c, int dtype, long long* launches, double* mean_ms, long long* points,
                            int* schedule, double* first_ms, double* second_ms) {
  if (!c || (dtype != 0 && dtype != 1) || !launches || !mean_ms || !points) return ALOFDFT_INVALID_ARGUMENT;
  if (schedule) *schedule = c->prof_sched[dtype];
  const long long n = c->prof_count[dtype];
  *launches = n;
  *mean_ms = n ? c->prof_ms[dtype] / n : 0.0;
  if (first_ms) *first_ms = n ? c->prof_ms_first[dtype] / n : 0.0;
  if (second_ms) *second_ms = n ? c->prof_ms_second[dtype] / n : 0.0;
  *points = c->prof_points[dtype];
  return ALOFDFT_OK;
}

int alofdft_solve(alofdft_ctx* c, const alofdft_system* sys, const alofdft_params* prm, const double* u0,
                  double* u_out, double* phi_out, double* forces_out, alofdft_result* res) {
  if (!c) return ALOFDFT_INVALID_ARGUMENT;
  return guarded(c, [&]() {
    require(c, sys != nullptr, "null system");
    const long long n = npoints(sys->n);
    double* du = u_out ? bufT<double>(c, "io.uout", (size_t)n) : nullptr;
    double* dp = phi_out ? bufT<double>(c, "io.phiout", (size_t)n) : nullptr;
    int st = solve_impl(c, sys, prm, nullptr, u0, du, dp, forces_out, res);
    if (u_out) HIPC(c, hipMemcpyAsync(u_out, du, sizeof(double) * n, hipMemcpyDeviceToHost, c->stream));
    if (phi_out) HIPC(c, hipMemcpyAsync(phi_out, dp, sizeof(double) * n, hipMemcpyDeviceToHost, c->stream));
    sync(c);
    return st;
  });
}

int alofdft_solve_device(alofdft_ctx* c, const alofdft_system* sys, const alofdft_params* prm, const double* u0_dev,
                         double* u_out_dev, double* phi_out_dev, double* forces_out, alofdft_result* res) {
  if (!c) return ALOFDFT_INVALID_ARGUMENT;
  return guarded(c, [&]() { return solve_impl(c, sys, prm, u0_dev, nullptr, u_out_dev, phi_out_dev, forces_out, res); });
}

int alofdft_default_relax_params(alofdft_relax_params* p) {
  if (!p) return ALOFDFT_INVALID_ARGUMENT;
  p->ftol = 1e-3;
  p->max_move = 0.3;
  p->probe = 0.05;
  p->max_steps = 50;
  p->max_secant = 3;
  p->secant_rel = 0.1;
  return ALOFDFT_OK;
}

int alofdft_relax(alofdft_ctx* c, const alofdft_system* sys, const alofdft_params* prm,
                  const alofdft_relax_params* rp, const double* u0, double* R_out, double* forces_out,
                  alofdft_result* res, alofdft_relax_info* info) {
  if (!c) return ALOFDFT_INVALID_ARGUMENT;
  return guarded(c, [&]() { return relax_impl(c, sys, prm, rp, u0, R_out, forces_out, res, info); });
}

int alofdft_apply_laplacian(alofdft_ctx* c, const int n[3], double h, int fdn, int dtype, const void* x, void* y) {
  if (!c) return ALOFDFT_INVALID_ARGUMENT;
  return guarded(c, [&]() {
    require(c, n && x && y, "null argument");
    require(c, fdn >= 1 && fdn <= kMaxRadius, "fd_half_width must be in 1..8");
    require(c, h > 0 && std::isfinite(h), "h must be > 0");
    require(c, dtype == 0 || dtype == 1, "dtype must be 0 (double) or 1 (float)");
    for (int a = 0; a < 3; ++a) require(c, n[a] >= 1, "n must be >= 1");
    const Geom g = make_geom(n, fdn);
    if (dtype == 0) {
      double* px = bufT<double>(c, "lap.x", g.total);
      double* py = bufT<double>(c, "lap.y", g.total);
      fill<double>(c, px, g.total, 0.0);
      pack<double, double>(c, g, (const double*)x, px);
      LapOp<double> op{px, py, nullptr};
      launch_stencil(c, g, stencil_weights<double>(fdn, h, 1.0), op);
      unpack<double, double>(c, g, py, (double*)y);
    } else {
      float* px = bufT<float>(c, "lapf.x", g.total);
      float* py = bufT<float>(c, "lapf.y", g.total);
      fill<float>(c, px, g.total, 0.0f);
      pack<float, float>(c, g, (const float*)x, px);
      LapOp<float> op{px, py, nullptr};
      launch_stencil(c, g, stencil_weights<float>(fdn, h, 1.0), op);
      unpack<float, float>(c, g, py, (float*)y);
    }
    sync(c);
    return ALOFDFT_OK;
  });
}

int alofdft_apply_laplacian_noalloc(alofdft_ctx* c, const int n[3], double h, int fdn, int dtype, const void* x,
                                    void* y) {
  if (!c) return ALOFDFT_INVALID_ARGUMENT;
  return guarded(c, [&]() {
    require(c, n && x && y, "null argument");
    require(c, fdn >= 1 && fdn <= kMaxRadius, "fd_half_width must be in 1..8");
    require(c, h > 0 && std::isfinite(h), "h must be > 0");
    require(c, dtype == 0 || dtype == 1, "dtype must be 0 (double) or 1 (float)");
    for (int a = 0; a < 3; ++a) require(c, n[a] >= 1, "n must be >= 1");
    const Geom g = make_geom(n, fdn);
    const size_t es = dtype == 0 ? sizeof(double) : sizeof(float);
    const size_t arr = ((size_t)g.total * es + 255) / 256 * 256;  // one padded array, 256-byte aligned
    if (2 * arr > kScratchBytes) {
      set_err(c, "grid needs %zu bytes of scratch for its padded x and y; the allocation-free Laplacian has %zu",
              2 * arr, kScratchBytes);
      throw Fail{ALOFDFT_INVALID_ARGUMENT};
    }
    unsigned char* base = (unsigned char*)scratch_ptr(c->device);
    require(c, base != nullptr, "scratch not resolved on this device");
    if (dtype == 0) {
      double* px = (double*)base;
      double* py = (double*)(base + arr);
      fill<double>(c, px, g.total, 0.0);  // the zero halo of this geometry
      pack<double, double>(c, g, (const double*)x, px);
      LapOp<double> op{px, py, nullptr};
      launch_stencil(c, g, stencil_weights<double>(fdn, h, 1.0), op);
      unpack<double, double>(c, g, py, (double*)y);
    } else {
      float* px = (float*)base;
      float* py = (float*)(base + arr);
      fill<float>(c, px, g.total, 0.0f);
      pack<float, float>(c, g, (const float*)x, px);
      LapOp<float> op{px, py, nullptr};
      launch_stencil(c, g, stencil_weights<float>(fdn, h, 1.0), op);
      unpack<float, float>(c, g, py, (float*)y);
    }
    return ALOFDFT_OK;
  });
}

int alofdft_poisson(alofdft_ctx* c, const int n[3], double h, const double origin[3], int fdn, int bc, int precision,
                    const double* rho, double* phi, double tol, int max_cg, long long* iters, double* relres) {
  if (!c) return ALOFDFT_INVALID_ARGUMENT;
  return guarded(c, [&]() {
    require(c, n && origin && rho && phi, "null argument");
    require(c, fdn >= 1 && fdn <= kMaxRadius, "fd_half_width must be in 1..8");
    require(c, h > 0 && std::isfinite(h) && tol > 0 && max_cg >= 1, "bad h, tol or max_cg");
    require(c, bc == ALOFDFT_BC_ZERO || bc == ALOFDFT_BC_MULTIPOLE, "bad bc");
    require(c, precision == ALOFDFT_FP64 || precision == ALOFDFT_FP32_REFINED, "bad precision");
    for (int a = 0; a < 3; ++a) require(c, n[a] >= 2 * fdn + 1, "grid smaller than 2n+1 nodes");
    require_addressable(c, n, fdn);
    (void)origin;  // the boundary expansion uses offsets from the box centre only
    const Geom g = make_geom(n, fdn);
    double* b = bufT<double>(c, "po.rho", g.total);
    double* zero = bufT<double>(c, "po.zero", g.total);
    double* v = bufT<double>(c, "po.v", g.total);
    double* rhs = bufT<double>(c, "po.rhs", g.total);
    double* x = bufT<double>(c, "po.x", g.total);
    double* parts = bufT<double>(c, "po.parts", (size_t)kPointwiseBlocks * kUpdRed);
    double* mom = bufT<double>(c, "po.mom", kUpdRed);
    for (double* a : {b, zero, v, rhs, x}) fill<double>(c, a, g.total, 0.0);
    pack<double, double>(c, g, rho, b);
    pack<double, double>(c, g, phi, x);
    BoxFrame f{h, 0.5 * (n[0] - 1), 0.5 * (n[1] - 1), 0.5 * (n[2] - 1)};
    TrialOp top{zero, zero, b, v, 0.0, f, parts};
    const int nb = launch_pw(c, g, top);
    finalize(c, parts, nb, kUpdRed, h * h * h, mom);
    RhsOp<double> rop{v, b, rhs, bc == ALOFDFT_BC_MULTIPOLE ? mom : nullptr, stencil_weights<double>(fdn, h, 1.0),
                      fdn, n[0], n[1], n[2], f, nullptr};
    launch_pw(c, g, rop);
    PoissonStats ps = poisson(c, g, fdn, h, precision, rhs, x, tol, max_cg, kCheckEvery);
    unpack<double, double>(c, g, x, phi);
    sync(c);
    if (iters) *iters = ps.iters;
    if (relres) *relres = ps.relres;
    return ps.status;
  });
}

int alofdft_energy_gradient(alofdft_ctx* c, const alofdft_system* sys, const alofdft_params* prm, const double* u,
                            double eta, double mu, double* phi, double* g, alofdft_energy* e) {
  if (!c) return ALOFDFT_INVALID_ARGUMENT;
  return guarded(c, [&]() {
    require(c, u && phi && e, "null argument");
    validate(c, sys, prm);
    Solver S(c, sys, prm);
    S.setup(u, false);
    pack<double, double>(c, S.geom(), phi, S.phi());
    double* gp = nullptr;
    if (g) {
      gp = bufT<double>(c, "eg.g", S.geom().total);
      S.set_gout(gp);
    }
    Eval ev;
    S.eval_trial(0.0, eta, mu, false, 0.0, ev);
    S.require_finite("the residual");
    S.energy(ev, e);
    e->L = e->E_total - eta * e->C_h + (mu > 0 ? e->C_h * e->C_h / (2.0 * mu) : 0.0);
    e->cg_iters = S.counts().cg_iters;
    unpack<double, double>(c, S.geom(), S.phi(), phi);
    if (g) unpack<double, double>(c, S.geom(), gp, g);
    sync(c);
    return ALOFDFT_OK;
  });
}

int alofdft_initial_guess(alofdft_ctx* c, const alofdft_system* sys, const alofdft_params* prm, double* u0) {
  if (!c) return ALOFDFT_INVALID_ARGUMENT;
  return guarded(c, [&]() {
    require(c, u0 != nullptr, "null argument");
    validate(c, sys, prm);
    const long long n = npoints(sys->n);
    if (prm->initial_guess == ALOFDFT_GUESS_ATOMIC) {
      atomic_guess_dev(c, sys, prm, u0);
    } else {
      std::vector<double> h = default_u0(sys, prm->seed);
      HIPC(c, hipMemcpyAsync(u0, h.data(), sizeof(double) * n, hipMemcpyHostToDevice, c->stream));
    }
    sync(c);
    return ALOFDFT_OK;
  });
}

int alofdft_pseudocharge(alofdft_ctx* c, const alofdft_system* sys, const alofdft_params* prm, double* b,
                         double* self_energy) {
  if (!c) return ALOFDFT_INVALID_ARGUMENT;
  return guarded(c, [&]() {
    require(c, b != nullptr, "null argument");
    validate(c, sys, prm);
    Solver S(c, sys, prm);
    double* z = bufT<double>(c, "pc.zero", (size_t)npoints(sys->n));
    S.setup(z, false);
    unpack<double, double>(c, S.geom(), S.b(), b);
    if (self_energy) *self_energy = S.E_self();
    sync(c);
    return ALOFDFT_OK;
  });
}

int alofdft_forces(alofdft_ctx* c, const alofdft_system* sys, const alofdft_params* prm, const double* phi,
                   double* forces) {
  if (!c) return ALOFDFT_INVALID_ARGUMENT;
  return guarded(c, [&]() {
    require(c, phi && forces, "null argument");
    validate(c, sys, prm);
    Solver S(c, sys, prm);
    double* z = bufT<double>(c, "pc.zero", (size_t)npoints(sys->n));
    S.setup(z, false);
    pack<double, double>(c, S.geom(), phi, S.phi());
    S.forces(forces);
    return ALOFDFT_OK;
  });
}

int alofdft_bench_stencil(alofdft_ctx* c, const int n[3], int fdn, int dtype, int reps, int nbuf, double* ms) {
  if (!c) return ALOFDFT_INVALID_ARGUMENT;
  return guarded(c, [&]() {
    require(c, n && ms && reps >= 1 && nbuf >= 1 && nbuf <= 64, "bad argument");
    require(c, fdn >= 1 && fdn <= kMaxRadius && (dtype == 0 || dtype == 1), "bad order or dtype");
    const Geom g = make_geom(n, fdn);
    std::vector<void*> xs(nbuf), ys(nbuf);
    const size_t es = dtype == 0 ? sizeof(double) : sizeof(float);
    for (int i = 0; i < nbuf; ++i) {
      xs[i] = buf(c, "bench.x" + std::to_string(i), g.total * es);
      ys[i] = buf(c, "bench.y" + std::to_string(i), g.total * es);
      if (dtype == 0) fill<double>(c, (double*)xs[i], g.total, 1.0 + 0.01 * i);
      else fill<float>(c, (float*)xs[i], g.total, 1.0f + 0.01f * i);
    }
    auto once = [&](int i) {
      const int b = i % nbuf;
      if (dtype == 0) {
        LapOp<double> op{(const double*)xs[b], (double*)ys[b], nullptr};
        launch_stencil(c, g, stencil_weights<double>(fdn, 0.5, 1.0), op);
      } else {
        LapOp<float> op{(const float*)xs[b], (float*)ys[b], nullptr};
        launch_stencil(c, g, stencil_weights<float>(fdn, 0.5, 1.0), op);
      }
    };
    for (int i = 0; i < std::min(reps, 10); ++i) once(i);
    HIPC(c, hipEventRecord(c->ev0, c->stream));
    for (int i = 0; i < reps; ++i) once(i);
    HIPC(c, hipEventRecord(c->ev1, c->stream));
    HIPC(c, hipEventSynchronize(c->ev1));
    float t = 0.f;
    HIPC(c, hipEventElapsedTime(&t, c->ev0, c->ev1));
    *ms = (double)t / reps;
    return ALOFDFT_OK;
  });
}

size_t alofdft_footprint_bytes(const alofdft_system* sys, const alofdft_params* prm) {
  if (!sys || !prm || prm->fd_half_width < 1 || prm->fd_half_width > kMaxRadius) return 0;
  for (int a = 0; a < 3; ++a)
    if (sys->n[a] < 1) return 0;
  return footprint(sys, prm);
}

int alofdft_server_create(alofdft_server** out, int hip_device, size_t hbm_budget_bytes, int max_slots) {
  if (!out || max_slots < 1 || max_slots > 16 || hbm_budget_bytes == 0) return ALOFDFT_INVALID_ARGUMENT;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || hip_device < 0 || hip_device >= ndev) return ALOFDFT_DEVICE_ERROR;
  if (hipSetDevice(hip_device) != hipSuccess) return ALOFDFT_DEVICE_ERROR;
  alofdft_server* s = new (std::nothrow) alofdft_server();
  if (!s) return ALOFDFT_OUT_OF_MEMORY;
  s->device = hip_device;
  s->budget = hbm_budget_bytes;
  for (int w = 0; w < max_slots; ++w) {
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
      alofdft_server_destroy(s);
      return ALOFDFT_DEVICE_ERROR;
    }
    s->streams.push_back(st);
    alofdft_ctx* c = nullptr;
    const int rc = alofdft_create(&c, hip_device, st);
    if (rc != ALOFDFT_OK) {
      alofdft_server_destroy(s);
      return rc;
    }
    c->target_blocks = ALOFDFT_SERVER_SLOT_BLOCKS;  // room for the other slots' kernels
    s->ctx.push_back(c);
    s->held.push_back(0);
    s->current.push_back(nullptr);
  }
  for (int w = 0; w < max_slots; ++w) s->workers.emplace_back(worker_loop, s, w);
  *out = s;
  return ALOFDFT_OK;
}

int alofdft_server_submit(alofdft_server* s, const alofdft_system* sys, const alofdft_params* prm, uint64_t* ticket) {
  if (!s || !sys || !prm || !ticket) return ALOFDFT_INVALID_ARGUMENT;
  auto r = std::make_shared<Request>();
  {
    alofdft_ctx tmp;  // validation only (no device work)
    try {
      validate(&tmp, sys, prm);
    } catch (const Fail& f) {
      return f.code;
    }
  }
  r->R.assign(sys->R, sys->R + 3 * (size_t)sys->M);
  r->Z.assign(sys->Z, sys->Z + (size_t)sys->M);
  r->sys = *sys;
  r->sys.R = r->R.data();
  r->sys.Z = r->Z.data();
  r->prm = *prm;
  r->fp = footprint(sys, prm);
  r->t_submit = std::chrono::steady_clock::now();
  std::lock_guard<std::mutex> lk(s->mu);
  s->submitted++;
  if (!s->have_first) {
    s->first_submit = r->t_submit;
    s->have_first = true;
  }
  if (r->fp > s->budget) {
    s->rejected++;
    return ALOFDFT_REJECTED;
  }
  r->id = s->next_id++;
  *ticket = r->id;
  s->reqs[r->id] = r;
  s->queue.push_back(r);
  s->cv.notify_all();
  return ALOFDFT_OK;
}

int alofdft_server_poll(alofdft_server* s, uint64_t ticket, alofdft_result* res, double* u_out, double* forces_out) {
  if (!s) return ALOFDFT_INVALID_ARGUMENT;
  std::shared_ptr<Request> r;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return ALOFDFT_INVALID_ARGUMENT;
    if (it->second->status == ALOFDFT_PENDING) return ALOFDFT_PENDING;
    r = it->second;
    s->reqs.erase(it);
  }
  if (res) *res = r->res;
  if (u_out) std::memcpy(u_out, r->u.data(), sizeof(double) * r->u.size());
  if (forces_out) std::memcpy(forces_out, r->forces.data(), sizeof(double) * r->forces.size());
  return r->status;
}

int alofdft_server_get_stats(alofdft_server* s, alofdft_server_stats* st) {
  if (!s || !st) return ALOFDFT_INVALID_ARGUMENT;
  std::lock_guard<std::mutex> lk(s->mu);
  std::memset(st, 0, sizeof(*st));
  st->submitted = s->submitted;
  st->admitted = s->admitted;
  st->completed = s->completed;
  st->rejected = s->rejected;
  st->cancelled = s->cancelled;
  st->queued = (int)s->queue.size();
  st->running = s->running;
  size_t hb = s->reserved;
  for (size_t h : s->held) hb += h;
  st->hbm_reserved_bytes = (double)hb;
  if (!s->lat_ms.empty()) {
    std::vector<double> v = s->lat_ms;
    std::sort(v.begin(), v.end());
    auto rank = [&](double q) {  // nearest-rank percentile
      size_t k = (size_t)std::ceil(q * v.size());
      return v[std::min(v.size() - 1, k > 0 ? k - 1 : 0)];
    };
    st->p50_ms = rank(0.50);
    st->p99_ms = rank(0.99);
    double sum = 0.0;
    for (double x : v) sum += x;
    st->mean_ms = sum / v.size();
    const double span = std::chrono::duration<double>(s->last_end - s->first_submit).count();
    st->solves_per_s = span > 0 ? s->completed / span : 0.0;
  }
  return ALOFDFT_OK;
}

int alofdft_server_cancel(alofdft_server* s, uint64_t ticket) {
  if (!s) return ALOFDFT_INVALID_ARGUMENT;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return ALOFDFT_INVALID_ARGUMENT;
  Request& r = *it->second;
  if (r.status != ALOFDFT_PENDING) return ALOFDFT_OK;  // finished already: its result stays
  if (r.slot < 0) {
    for (auto q = s->queue.begin(); q != s->queue.end(); ++q)
      if ((*q)->id == ticket) {
        s->queue.erase(q);
        break;
      }
    r.status = ALOFDFT_CANCELLED;
    r.res.status = ALOFDFT_CANCELLED;
    s->cancelled++;
    s->cv.notify_all();  // the next request may fit now
  } else {
    s->ctx[r.slot]->cancel.store(1);  // the slot's solve stops at its next check
  }
  return ALOFDFT_OK;
}

int alofdft_server_set_tuning(alofdft_server* s, int target_blocks) {
  if (!s || target_blocks < 0) return ALOFDFT_INVALID_ARGUMENT;
  std::lock_guard<std::mutex> lk(s->mu);
  // a slot's context is read by its worker only while it runs a request
  if (s->running > 0 || !s->queue.empty()) return ALOFDFT_INVALID_ARGUMENT;
  for (alofdft_ctx* c : s->ctx) c->target_blocks = target_blocks;
  return ALOFDFT_OK;
}

int alofdft_cancel(alofdft_ctx* c) {
  if (!c) return ALOFDFT_INVALID_ARGUMENT;
  c->cancel.store(1);
  return ALOFDFT_OK;
}

void alofdft_server_destroy(alofdft_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    // queued requests are cancelled, running ones stop at their next check
    for (auto& q : s->queue) {
      q->status = ALOFDFT_CANCELLED;
      q->res.status = ALOFDFT_CANCELLED;
      s->cancelled++;
    }
    s->queue.clear();
    for (size_t w = 0; w < s->current.size(); ++w)
      if (s->current[w]) s->ctx[w]->cancel.store(1);
  }
  s->cv.notify_all();
  for (auto& t : s->workers)
    if (t.joinable()) t.join();
  for (alofdft_ctx* c : s->ctx) alofdft_destroy(c);
  (void)hipSetDevice(s->device);
  for (hipStream_t st : s->streams) (void)hipStreamDestroy(st);
  delete s;
}

}  // extern "C"
