"""MI355X (gfx950) augmented Lagrangian orbital-free DFT: Python binding.

Thin ctypes marshalling over ``libalofdft.so`` (C ABI in ``include/alofdft.h``).
Every step of the computation runs in the HIP library; PyTorch supplies device
memory and the current stream.  There is no CPU fallback: if the library is not
built, or no HIP device is present, the calls raise.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libalofdft.so")

OK, NOT_CONVERGED, PENDING = 0, 1, 2
INVALID_ARGUMENT, OUT_OF_MEMORY, DEVICE_ERROR, NUMERICAL, REJECTED, CANCELLED = -1, -2, -3, -4, -5, -6
AL, PENALTY, LAGRANGE = 0, 1, 2
PSEUDO_GAUSSIAN, PSEUDO_FD_LAPLACIAN = 0, 1
GUESS_UNIFORM, GUESS_ATOMIC = 0, 1
STOP_CONSTRAINT, STOP_ENERGY_CHANGE = 0, 1
DOMAIN_BOX, DOMAIN_ELLIPSOID = 0, 1
SERVER_SLOT_BLOCKS = 256  # ALOFDFT_SERVER_SLOT_BLOCKS: default workgroups per stencil launch of a server slot
BC_ZERO, BC_MULTIPOLE = 0, 1
FP64, FP32_REFINED = 0, 1


class Params(C.Structure):
    _fields_ = [("fd_half_width", C.c_int), ("lambda_", C.c_double), ("xc", C.c_int),
                ("gauss_width", C.c_double), ("r_cut", C.c_double), ("method", C.c_int),
                ("eta0", C.c_double), ("mu0", C.c_double), ("kappa", C.c_double),
                ("tol_constraint", C.c_double), ("tol_grad", C.c_double), ("tol_poisson", C.c_double),
                ("phi_bc", C.c_int), ("precision", C.c_int), ("max_outer", C.c_int), ("max_inner", C.c_int),
                ("max_cg", C.c_int), ("sigma0", C.c_double), ("max_secant", C.c_int),
                ("secant_rel", C.c_double), ("restart_every", C.c_int), ("cg_check_every", C.c_int),
                ("seed", C.c_uint64), ("pseudocharge", C.c_int), ("initial_guess", C.c_int),
                ("guess_width", C.c_double), ("guess_floor", C.c_double), ("al_stop", C.c_int),
                ("tol_energy", C.c_double), ("domain", C.c_int)]


class SystemS(C.Structure):
    _fields_ = [("M", C.c_int), ("R", C.POINTER(C.c_double)), ("Z", C.POINTER(C.c_double)),
                ("N_elec", C.c_double), ("n", C.c_int * 3), ("h", C.c_double), ("origin", C.c_double * 3)]


class Counts(C.Structure):
    _fields_ = [(k, C.c_longlong) for k in ("outer", "inner", "grad_evals", "poisson_solves", "cg_iters",
                                             "matvec_fp64", "matvec_fp32", "refinements")]


class Result(C.Structure):
    _fields_ = [(k, C.c_double) for k in ("E_total", "E_TF", "E_vW", "E_xc", "E_es", "E_self", "E_corr",
                                           "eta_star", "C_h", "grad_norm", "poisson_relres", "dE_last")] + \
               [("counts", Counts)] + \
               [(k, C.c_double) for k in ("time_total_ms", "time_poisson_ms", "time_grad_ms", "time_setup_ms")] + \
               [("status", C.c_int)]


class Energy(C.Structure):
    _fields_ = [(k, C.c_double) for k in ("E_TF", "E_vW", "E_xc", "E_es", "E_self", "E_corr", "E_total",
                                           "C_h", "L", "grad_norm")] + [("cg_iters", C.c_longlong)]


class ServerStats(C.Structure):
    _fields_ = [(k, C.c_longlong) for k in ("submitted", "admitted", "completed", "rejected")] + \
               [("queued", C.c_int), ("running", C.c_int)] + \
               [(k, C.c_double) for k in ("p50_ms", "p99_ms", "mean_ms", "solves_per_s", "hbm_reserved_bytes")] + \
               [("cancelled", C.c_longlong)]


class RelaxParams(C.Structure):
    _fields_ = [("ftol", C.c_double), ("max_move", C.c_double), ("probe", C.c_double), ("max_steps", C.c_int),
                ("max_secant", C.c_int), ("secant_rel", C.c_double)]


class RelaxInfo(C.Structure):
    _fields_ = [("status", C.c_int), ("steps", C.c_int), ("solves", C.c_int), ("fmax", C.c_double),
                ("E_total", C.c_double)]


class AlofdftError(RuntimeError):
    def __init__(self, status, detail=""):
        super().__init__(f"alofdft status {status}: {detail}")
        self.status = status


_lib = None
_DP = C.POINTER(C.c_double)
_VP = C.c_void_p


def lib():
    """Load the HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run __graft_entry__.build() first")
        L = C.CDLL(LIB_PATH)
        L.alofdft_strerror.restype = C.c_char_p
        L.alofdft_strerror.argtypes = [C.c_int]
        L.alofdft_last_error.restype = C.c_char_p
        L.alofdft_last_error.argtypes = [_VP]
        L.alofdft_default_params.argtypes = [C.POINTER(Params)]
        L.alofdft_create.argtypes = [C.POINTER(_VP), C.c_int, _VP]
        L.alofdft_destroy.argtypes = [_VP]
        L.alofdft_destroy.restype = None
        L.alofdft_set_tuning.argtypes = [_VP, C.c_int, C.c_int, C.c_int]
        L.alofdft_set_cg_schedule.argtypes = [_VP, C.c_int]
        L.alofdft_solve.argtypes = [_VP, C.POINTER(SystemS), C.POINTER(Params), _DP, _DP, _DP, _DP,
                                    C.POINTER(Result)]
        L.alofdft_solve_device.argtypes = [_VP, C.POINTER(SystemS), C.POINTER(Params), _VP, _VP, _VP, _DP,
                                           C.POINTER(Result)]
        L.alofdft_default_relax_params.argtypes = [C.POINTER(RelaxParams)]
        L.alofdft_relax.argtypes = [_VP, C.POINTER(SystemS), C.POINTER(Params), C.POINTER(RelaxParams), _DP, _DP,
                                    _DP, C.POINTER(Result), C.POINTER(RelaxInfo)]
        L.alofdft_apply_laplacian.argtypes = [_VP, C.POINTER(C.c_int), C.c_double, C.c_int, C.c_int, _VP, _VP]
        L.alofdft_apply_laplacian_noalloc.argtypes = [_VP, C.POINTER(C.c_int), C.c_double, C.c_int, C.c_int, _VP,
                                                      _VP]
        L.alofdft_poisson.argtypes = [_VP, C.POINTER(C.c_int), C.c_double, _DP, C.c_int, C.c_int, C.c_int, _VP,
                                      _VP, C.c_double, C.c_int, C.POINTER(C.c_longlong), _DP]
        L.alofdft_energy_gradient.argtypes = [_VP, C.POINTER(SystemS), C.POINTER(Params), _VP, C.c_double,
                                              C.c_double, _VP, _VP, C.POINTER(Energy)]
        L.alofdft_pseudocharge.argtypes = [_VP, C.POINTER(SystemS), C.POINTER(Params), _VP, _DP]
        L.alofdft_initial_guess.argtypes = [_VP, C.POINTER(SystemS), C.POINTER(Params), _VP]
        L.alofdft_forces.argtypes = [_VP, C.POINTER(SystemS), C.POINTER(Params), _VP, _DP]
        L.alofdft_bench_stencil.argtypes = [_VP, C.POINTER(C.c_int), C.c_int, C.c_int, C.c_int, C.c_int, _DP]
        L.alofdft_footprint_bytes.restype = C.c_size_t
        L.alofdft_footprint_bytes.argtypes = [C.POINTER(SystemS), C.POINTER(Params)]
        L.alofdft_server_create.argtypes = [C.POINTER(_VP), C.c_int, C.c_size_t, C.c_int]
        L.alofdft_server_submit.argtypes = [_VP, C.POINTER(SystemS), C.POINTER(Params), C.POINTER(C.c_uint64)]
        L.alofdft_server_poll.argtypes = [_VP, C.c_uint64, C.POINTER(Result), _DP, _DP]
        L.alofdft_server_get_stats.argtypes = [_VP, C.POINTER(ServerStats)]
        L.alofdft_server_cancel.argtypes = [_VP, C.c_uint64]
        L.alofdft_server_set_tuning.argtypes = [_VP, C.c_int]
        L.alofdft_cancel.argtypes = [_VP]
        L.alofdft_server_destroy.argtypes = [_VP]
        L.alofdft_server_destroy.restype = None
        L.alofdft_profile_cg_kernel.argtypes = [_VP, C.c_int]
        L.alofdft_cg_kernel_stats.argtypes = [_VP, C.c_int, C.POINTER(C.c_longlong), _DP, C.POINTER(C.c_longlong),
                                              C.POINTER(C.c_int), _DP, _DP]
        _lib = L
    return _lib


def default_params(**kw) -> Params:
    """Library defaults (order 12, lambda 0.2, LDA, AL with eta0=-0.2, mu0=1, kappa=0.1,
    tolerances 1e-8 / 1e-6 / 1e-10, multipole phi boundary, FP64) with overrides."""
    p = Params()
    lib().alofdft_default_params(C.byref(p))
    for k, v in kw.items():
        setattr(p, "lambda_" if k == "lambda" else k, v)
    return p


def default_relax_params(**kw) -> RelaxParams:
    """Relaxation defaults (ftol 1e-3 Ha/Bohr, max_move 0.3 Bohr, probe 0.05 Bohr, 50 steps,
    3 solves per line search, secant_rel 0.1) with overrides."""
    p = RelaxParams()
    lib().alofdft_default_relax_params(C.byref(p))
    for k, v in kw.items():
        setattr(p, k, v)
    return p


class SystemArgs:
    """Holds the C system struct for a synth.System and keeps its arrays alive."""

    def __init__(self, system):
        self.R = np.ascontiguousarray(system.R, dtype=np.float64).reshape(-1)
        self.Z = np.ascontiguousarray(system.Z, dtype=np.float64)
        s = SystemS()
        s.M = int(len(self.Z))
        s.R = self.R.ctypes.data_as(_DP)
        s.Z = self.Z.ctypes.data_as(_DP)
        s.N_elec = float(system.N)
        for a in range(3):
            s.n[a] = int(system.grid.n[a])
            s.origin[a] = float(system.grid.origin[a])
        s.h = float(system.grid.h)
        self.s = s


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _check(ctx, st, ok=(OK,)):
    if st not in ok:
        detail = lib().alofdft_last_error(ctx.handle).decode()
        raise AlofdftError(st, f"{lib().alofdft_strerror(st).decode()}: {detail}")
    return st


class Context:
    """A library context on the current HIP device, enqueuing on torch's current stream."""

    def __init__(self, device: int | None = None, stream=None):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device: the alofdft library runs only on the GPU")
        torch.cuda.init()  # the runtime's device state exists before the library's first call
        self.device = torch.cuda.current_device() if device is None else int(device)
        with torch.cuda.device(self.device):
            s = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.stream = s
        h = C.c_void_p()
        st = lib().alofdft_create(C.byref(h), self.device, C.c_void_p(s.cuda_stream))
        if st != OK:
            raise AlofdftError(st, lib().alofdft_strerror(st).decode())
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            lib().alofdft_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def cancel(self):
        """Ask the call running on this context (from another thread) to stop; it raises
        AlofdftError(CANCELLED).  With no call running, the next call stops at its first check."""
        _check(self, lib().alofdft_cancel(self.handle))

    def set_tuning(self, variant=-1, target_blocks=0, inner_tol_exp=6):
        _check(self, lib().alofdft_set_tuning(self.handle, variant, target_blocks, inner_tol_exp))

    # ------------------------------------------------------------- full solve
    def set_cg_schedule(self, schedule=-1):
        """CG launches per iteration: 0 applies the stencil to p = r + beta p, then
        updates x and r; 1 applies it to r and forms A p = A r + beta A p by linearity,
        then updates x and r; 2 (FP64 solves only) fuses the iteration into one launch
        with one reduction in the pipelined form, the stencil applied to the stored
        w = A r; -1 (default) picks 2 for FP64 solves on grids up to 1.5e6 nodes, else 1."""
        _check(self, lib().alofdft_set_cg_schedule(self.handle, int(schedule)))

    def solve(self, system, params: Params | None = None, u0=None, want_fields=True, want_forces=True):
        """Ground state on the GPU.  u0: host numpy array (grid shape) or None for the
        library's default guess.  Returns a dict of energies, counters, u, phi, forces."""
        params = params or default_params()
        S = SystemArgs(system)
        shape = system.grid.shape
        u = np.zeros(shape) if want_fields else None
        phi = np.zeros(shape) if want_fields else None
        f = np.zeros((S.s.M, 3)) if want_forces else None
        u0c = None if u0 is None else np.ascontiguousarray(u0, dtype=np.float64)
        res = Result()
        st = lib().alofdft_solve(self.handle, C.byref(S.s), C.byref(params),
                                 None if u0c is None else u0c.ctypes.data_as(_DP),
                                 None if u is None else u.ctypes.data_as(_DP),
                                 None if phi is None else phi.ctypes.data_as(_DP),
                                 None if f is None else f.ctypes.data_as(_DP), C.byref(res))
        _check(self, st, (OK, NOT_CONVERGED))
        out = result_dict(res)
        out.update(u=u, phi=phi, forces=f)
        return out

    def relax(self, system, params: Params | None = None, relax: RelaxParams | None = None, u0=None):
        """Relaxes the nuclei from system.R (Polak-Ribiere nonlinear CG with a secant line
        search, every evaluation a full solve).  Returns a dict with R, forces, the final
        solve's result fields and steps, solves, fmax, relax_status."""
        params = params or default_params()
        relax = relax or default_relax_params()
        S = SystemArgs(system)
        R = np.zeros((S.s.M, 3))
        f = np.zeros((S.s.M, 3))
        u0c = None if u0 is None else np.ascontiguousarray(u0, dtype=np.float64)
        res, info = Result(), RelaxInfo()
        st = lib().alofdft_relax(self.handle, C.byref(S.s), C.byref(params), C.byref(relax),
                                 None if u0c is None else u0c.ctypes.data_as(_DP), R.ctypes.data_as(_DP),
                                 f.ctypes.data_as(_DP), C.byref(res), C.byref(info))
        _check(self, st, (OK, NOT_CONVERGED))
        out = result_dict(res)
        out.update(R=R, forces=f, steps=info.steps, solves=info.solves, fmax=info.fmax, relax_status=info.status)
        return out

    def solve_device(self, system, params=None, u0=None, u_out=None, phi_out=None, want_forces=True):
        """As solve() with torch device tensors (float64, grid shape) for u0/u_out/phi_out."""
        params = params or default_params()
        S = SystemArgs(system)
        f = np.zeros((S.s.M, 3)) if want_forces else None
        res = Result()
        st = lib().alofdft_solve_device(self.handle, C.byref(S.s), C.byref(params), _ptr(u0), _ptr(u_out),
                                        _ptr(phi_out), None if f is None else f.ctypes.data_as(_DP),
                                        C.byref(res))
        _check(self, st, (OK, NOT_CONVERGED))
        out = result_dict(res)
        out["forces"] = f
        return out

    # ------------------------------------------------------------- steps
    def apply_laplacian(self, x, h: float, fd_half_width: int = 6):
        """Delta_h x for a contiguous float64/float32 device tensor of shape (n3, n2, n1)."""
        import torch

        assert x.is_cuda and x.is_contiguous() and x.dim() == 3
        dtype = {torch.float64: 0, torch.float32: 1}[x.dtype]
        y = torch.empty_like(x)
        n = (C.c_int * 3)(x.shape[2], x.shape[1], x.shape[0])
        _check(self, lib().alofdft_apply_laplacian(self.handle, n, h, fd_half_width, dtype, _ptr(x), _ptr(y)))
        return y

    def poisson(self, rho, grid, phi0=None, fd_half_width=6, bc=BC_MULTIPOLE, precision=FP64, tol=1e-10,
                max_cg=100000):
        """-(1/4 pi) Delta_h phi = rho with the given boundary values; returns (phi, iters, relres)."""
        import torch

        assert rho.is_cuda and rho.dtype == torch.float64 and rho.is_contiguous()
        phi = torch.zeros_like(rho) if phi0 is None else phi0.clone()
        n = (C.c_int * 3)(*[int(v) for v in grid.n])
        org = (C.c_double * 3)(*[float(v) for v in grid.origin])
        its = C.c_longlong()
        rel = C.c_double()
        st = lib().alofdft_poisson(self.handle, n, grid.h, org, fd_half_width, bc, precision, _ptr(rho), _ptr(phi),
                                   tol, max_cg, C.byref(its), C.byref(rel))
        _check(self, st, (OK, NOT_CONVERGED))
        return phi, its.value, rel.value

    def energy_gradient(self, system, params, u, eta, mu, phi=None, want_g=True):
        """Energies and residual at u (device float64 tensor); phi is the warm start and is
        returned updated.  Returns (g, energies dict, phi)."""
        import torch

        params = params or default_params()
        S = SystemArgs(system)
        phi = torch.zeros_like(u) if phi is None else phi.clone()
        g = torch.empty_like(u) if want_g else None
        e = Energy()
        st = lib().alofdft_energy_gradient(self.handle, C.byref(S.s), C.byref(params), _ptr(u), eta, mu,
                                           _ptr(phi), _ptr(g), C.byref(e))
        _check(self, st)
        return g, {k: getattr(e, k) for k, _ in Energy._fields_}, phi

    def pseudocharge(self, system, params=None):
        import torch

        params = params or default_params()
        S = SystemArgs(system)
        b = torch.empty(system.grid.shape, dtype=torch.float64, device=f"cuda:{self.device}")
        es = C.c_double()
        _check(self, lib().alofdft_pseudocharge(self.handle, C.byref(S.s), C.byref(params), _ptr(b), C.byref(es)))
        return b, es.value

    def initial_guess(self, system, params=None):
        """The guess a solve takes without u0 (params.initial_guess), as a device tensor."""
        import torch

        params = params or default_params()
        S = SystemArgs(system)
        u = torch.empty(system.grid.shape, dtype=torch.float64, device=f"cuda:{self.device}")
        _check(self, lib().alofdft_initial_guess(self.handle, C.byref(S.s), C.byref(params), _ptr(u)))
        return u

    def forces(self, system, params, phi):
        params = params or default_params()
        S = SystemArgs(system)
        f = np.zeros((S.s.M, 3))
        _check(self, lib().alofdft_forces(self.handle, C.byref(S.s), C.byref(params), _ptr(phi),
                                          f.ctypes.data_as(_DP)))
        return f

    def profile_cg_kernel(self, sample_every=1):
        """Start (reset) sampled HIP-event timing of the CG stencil kernel; 0 stops it."""
        _check(self, lib().alofdft_profile_cg_kernel(self.handle, int(sample_every)))

    def cg_kernel_stats(self, dtype=0, split=False):
        """(timed iterations, mean kernel ms per iteration, grid points, CG schedule or -1) for
        dtype 0 (FP64) / 1 (FP32); with split=True also the mean ms of the iteration's first
        (stencil) and second (update) launch."""
        n, ms, pts, sch = C.c_longlong(), C.c_double(), C.c_longlong(), C.c_int()
        a, b = C.c_double(), C.c_double()
        _check(self, lib().alofdft_cg_kernel_stats(self.handle, dtype, C.byref(n), C.byref(ms), C.byref(pts),
                                                   C.byref(sch), C.byref(a), C.byref(b)))
        if split:
            return n.value, ms.value, pts.value, sch.value, a.value, b.value
        return n.value, ms.value, pts.value, sch.value

    def bench_stencil(self, n, fd_half_width=6, dtype=0, reps=100, nbuf=6):
        """Mean kernel time (ms) of one stencil application over a rotation of nbuf buffer pairs."""
        nn = (C.c_int * 3)(*[int(v) for v in n])
        ms = C.c_double()
        _check(self, lib().alofdft_bench_stencil(self.handle, nn, fd_half_width, dtype, reps, nbuf, C.byref(ms)))
        return ms.value


def result_dict(res: Result) -> dict:
    out = {k: getattr(res, k) for k, _ in Result._fields_ if k != "counts"}
    out.update({k: getattr(res.counts, k) for k, _ in Counts._fields_})
    return out


def footprint_bytes(system, params=None) -> int:
    """Device bytes one request of this system reserves while it is solved."""
    S = SystemArgs(system)
    return int(lib().alofdft_footprint_bytes(C.byref(S.s), C.byref(params or default_params())))


class Server:
    """Continuous-batching request loop on one GPU (see alofdft_server_* in the C ABI)."""

    def __init__(self, device=0, hbm_budget_bytes=None, max_slots=4):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device: the alofdft server runs only on the GPU")
        if hbm_budget_bytes is None:
            free, _ = torch.cuda.mem_get_info(device)
            hbm_budget_bytes = int(0.9 * free)
        h = C.c_void_p()
        st = lib().alofdft_server_create(C.byref(h), int(device), int(hbm_budget_bytes), int(max_slots))
        if st != OK:
            raise AlofdftError(st, lib().alofdft_strerror(st).decode())
        self.handle = h
        self._shapes = {}

    def submit(self, system, params=None):
        """Queue a solve; returns a ticket.  Raises AlofdftError(REJECTED) if it can never fit."""
        S = SystemArgs(system)
        t = C.c_uint64()
        st = lib().alofdft_server_submit(self.handle, C.byref(S.s), C.byref(params or default_params()),
                                         C.byref(t))
        if st != OK:
            raise AlofdftError(st, lib().alofdft_strerror(st).decode())
        self._shapes[t.value] = (system.grid.shape, S.s.M)
        return t.value

    def poll(self, ticket):
        """None while pending; else a result dict with u and forces (the ticket is released)."""
        shape, M = self._shapes[ticket]
        res = Result()
        u = np.zeros(shape)
        f = np.zeros((M, 3))
        st = lib().alofdft_server_poll(self.handle, ticket, C.byref(res), u.ctypes.data_as(_DP),
                                       f.ctypes.data_as(_DP))
        if st == PENDING:
            return None
        del self._shapes[ticket]
        out = result_dict(res)
        out.update(status=st, u=u, forces=f)
        return out

    def wait(self, ticket, poll_s=0.002):
        import time

        while True:
            r = self.poll(ticket)
            if r is not None:
                return r
            time.sleep(poll_s)

    def cancel(self, ticket):
        """Cancel a queued or running request (poll then reports status CANCELLED)."""
        st = lib().alofdft_server_cancel(self.handle, ticket)
        if st != OK:
            raise AlofdftError(st, lib().alofdft_strerror(st).decode())

    def set_tuning(self, target_blocks):
        """Workgroups per stencil launch of every slot (0: one round); only while idle."""
        st = lib().alofdft_server_set_tuning(self.handle, int(target_blocks))
        if st != OK:
            raise AlofdftError(st, lib().alofdft_strerror(st).decode())

    def stats(self):
        s = ServerStats()
        lib().alofdft_server_get_stats(self.handle, C.byref(s))
        return {k: getattr(s, k) for k, _ in ServerStats._fields_}

    def close(self):
        if getattr(self, "handle", None):
            lib().alofdft_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
