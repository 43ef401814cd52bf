"""ctypes wrapper of the plain FP64 CPU oracle (oracle.cpp).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
benchmark's CPU-baseline leg, never by the GPU library or its Python binding.
It shares no code with the GPU path; inputs come from the synthetic generators.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")

BUILD_CMD = ["g++", "-O2", "-fopenmp", "-ffp-contract=off", "-shared", "-fPIC", _SRC, "-o", _LIB]


def build() -> str:
    """Compile liboracle.so from oracle.cpp (always recompiles)."""
    subprocess.run(BUILD_CMD, check=True)
    return _LIB


class OrGrid(C.Structure):
    _fields_ = [("n", C.c_int * 3), ("h", C.c_double), ("origin", C.c_double * 3)]


class OrSystem(C.Structure):
    _fields_ = [("grid", OrGrid), ("M", C.c_int), ("R", C.POINTER(C.c_double)),
                ("Z", C.POINTER(C.c_double)), ("N", C.c_double)]


class OrParams(C.Structure):
    _fields_ = [("fd_n", C.c_int), ("lambda_", C.c_double), ("xc", C.c_int), ("gauss_s", C.c_double),
                ("r_cut", C.c_double), ("method", C.c_int), ("eta0", C.c_double), ("mu0", C.c_double),
                ("kappa", C.c_double), ("tol_constraint", C.c_double), ("tol_grad", C.c_double),
                ("tol_poisson", C.c_double), ("bc", C.c_int), ("max_al", C.c_int), ("max_nlcg", C.c_int),
                ("max_cg", C.c_int), ("sigma0", C.c_double), ("max_secant", C.c_int),
                ("secant_rel", C.c_double), ("restart_every", C.c_int), ("tf_on", C.c_int),
                ("hartree_on", C.c_int), ("vext", C.POINTER(C.c_double)), ("verbose", C.c_int),
                ("al_stop", C.c_int), ("tol_energy", C.c_double), ("pseudo", C.c_int), ("domain", C.c_int)]


class OrResult(C.Structure):
    _fields_ = [(k, C.c_double) for k in ("E_total", "E_TF", "E_vW", "E_xc", "E_es", "E_self", "E_c",
                                           "E_ext", "L", "eta", "C", "gnorm", "dE_last", "poisson_relres")] + \
               [(k, C.c_long) for k in ("al_iters", "nlcg_iters", "grad_evals", "poisson_solves",
                                         "cg_iters", "matvecs")] + [("status", C.c_int)]


class OrEnergies(C.Structure):
    _fields_ = [(k, C.c_double) for k in ("E_TF", "E_vW", "E_xc", "E_es", "E_ext", "C", "L", "E_self",
                                           "E_c", "E_total")]


_lib = None
_DP = C.POINTER(C.c_double)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = C.CDLL(_LIB)
        L.or_fd_weights.argtypes = [C.c_int, C.c_double, _DP]
        L.or_fd_grad_weights.argtypes = [C.c_int, C.c_double, _DP]
        L.or_laplacian.argtypes = [C.POINTER(OrGrid), C.c_int, _DP, _DP]
        L.or_xc_point.argtypes = [C.c_double, _DP, _DP]
        L.or_CF.restype = C.c_double
        L.or_bJ.restype = C.c_double
        L.or_bJ.argtypes = [C.c_double] * 4
        L.or_VJ.restype = C.c_double
        L.or_VJ.argtypes = [C.c_double] * 3
        L.or_pseudocharge.argtypes = [C.POINTER(OrGrid), C.c_int, _DP, _DP, C.c_double, C.c_double, C.c_int,
                                      C.c_int, _DP]
        L.or_pseudocharge_at.restype = C.c_double
        L.or_pseudocharge_at.argtypes = [C.POINTER(OrGrid), C.c_int, _DP, _DP, C.c_double, C.c_double,
                                         C.c_int, C.c_int, C.c_int, C.c_int, C.c_int]
        L.or_self_energy.restype = C.c_double
        L.or_self_energy.argtypes = [C.POINTER(OrGrid), C.c_int, _DP, _DP, C.c_double, C.c_double, C.c_int,
                                     C.c_int]
        L.or_bJ_fd.restype = C.c_double
        L.or_bJ_fd.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double, C.c_int, C.c_double, C.c_double,
                               C.c_double]
        L.or_atomic_guess.argtypes = [C.POINTER(OrGrid), C.c_int, _DP, _DP, C.c_double, C.c_double, C.c_double,
                                      _DP]
        L.or_overlap_correction.restype = C.c_double
        L.or_overlap_correction.argtypes = [C.c_int, _DP, _DP, C.c_double, _DP]
        L.or_moments.argtypes = [C.POINTER(OrGrid), _DP, _DP]
        L.or_phi_multipole.restype = C.c_double
        L.or_phi_multipole.argtypes = [_DP, _DP, _DP]
        L.or_poisson_rhs.argtypes = [C.POINTER(OrGrid), C.c_int, C.c_int, _DP, _DP]
        L.or_poisson_cg.restype = C.c_int
        L.or_poisson_cg.argtypes = [C.POINTER(OrGrid), C.c_int, _DP, _DP, C.c_double, C.c_int,
                                    C.POINTER(C.c_int), _DP]
        L.or_evaluate.restype = C.c_int
        L.or_poisson_cg_masked.argtypes = [C.POINTER(OrGrid), C.c_int, C.POINTER(C.c_ubyte), _DP, _DP,
                                            C.c_double, C.c_int, C.POINTER(C.c_int), _DP]
        L.or_domain_mask.argtypes = [C.POINTER(OrGrid), C.POINTER(C.c_ubyte)]
        L.or_domain_mask.restype = None
        L.or_domain_inside.argtypes = [C.POINTER(OrGrid), C.c_int, C.c_int, C.c_int]
        L.or_evaluate.argtypes = [C.POINTER(OrSystem), C.POINTER(OrParams), _DP, C.c_double, C.c_double,
                                  _DP, _DP, C.POINTER(OrEnergies), C.POINTER(C.c_long)]
        L.or_forces.argtypes = [C.POINTER(OrSystem), C.POINTER(OrParams), _DP, _DP]
        L.or_default_params.argtypes = [C.POINTER(OrParams)]
        L.or_solve.restype = C.c_int
        L.or_solve.argtypes = [C.POINTER(OrSystem), C.POINTER(OrParams), _DP, _DP, _DP, _DP,
                               C.POINTER(OrResult)]
        L.or_set_threads.argtypes = [C.c_int]
        L.or_get_threads.restype = C.c_int
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(_DP)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def make_grid(grid) -> OrGrid:
    g = OrGrid()
    for a in range(3):
        g.n[a] = int(grid.n[a])
        g.origin[a] = float(grid.origin[a])
    g.h = float(grid.h)
    return g


class Sys:
    """Holds the ctypes system struct and keeps its arrays alive."""

    def __init__(self, system):
        self.R = _f64(system.R).reshape(-1)
        self.Z = _f64(system.Z)
        self.grid = system.grid
        self.s = OrSystem()
        self.s.grid = make_grid(system.grid)
        self.s.M = int(len(self.Z))
        self.s.R = _p(self.R)
        self.s.Z = _p(self.Z)
        self.s.N = float(system.N)


def params(**kw) -> OrParams:
    """Default parameters (order 12, lambda 0.2, LDA on, AL eta0=-0.2 mu0=1 kappa=0.1,
    tolerances 1e-8 / 1e-6 / 1e-10, multipole phi boundary) with overrides."""
    p = OrParams()
    lib().or_default_params(C.byref(p))
    for k, v in kw.items():
        if k == "lambda":
            k = "lambda_"
        if k == "vext":
            arr = _f64(v).reshape(-1)
            p._vext_keep = arr
            p.vext = _p(arr)
            continue
        setattr(p, k, v)
    return p


def set_threads(t: int):
    lib().or_set_threads(int(t))


def get_threads() -> int:
    return int(lib().or_get_threads())


def weights(n: int, h: float) -> np.ndarray:
    w = np.zeros(n + 1)
    lib().or_fd_weights(n, h, _p(w))
    return w


def grad_weights(n: int, h: float) -> np.ndarray:
    w = np.zeros(n + 1)
    lib().or_fd_grad_weights(n, h, _p(w))
    return w


def laplacian(grid, n: int, f: np.ndarray) -> np.ndarray:
    f = _f64(f)
    out = np.zeros_like(f)
    g = make_grid(grid)
    lib().or_laplacian(C.byref(g), n, _p(f), _p(out))
    return out


def xc_point(u: float):
    e, v = C.c_double(), C.c_double()
    lib().or_xc_point(float(u), C.byref(e), C.byref(v))
    return e.value, v.value


def CF() -> float:
    return lib().or_CF()


def bJ(Z, s, rc, r) -> float:
    return lib().or_bJ(Z, s, rc, r)


def VJ(Z, s, r) -> float:
    return lib().or_VJ(Z, s, r)


def pseudocharge(system, s=1.0, rc=7.0, mode=0, fd_n=6) -> np.ndarray:
    """b on the grid: mode 0 Gaussian b_J, mode 1 -(1/4 pi) Delta_h V_J (order 2 fd_n)."""
    S = Sys(system)
    b = np.zeros(system.grid.shape)
    lib().or_pseudocharge(C.byref(S.s.grid), S.s.M, S.s.R, S.s.Z, s, rc, mode, fd_n, _p(b))
    return b


def pseudocharge_at(system, i, j, k, s=1.0, rc=7.0, mode=0, fd_n=6) -> float:
    S = Sys(system)
    return lib().or_pseudocharge_at(C.byref(S.s.grid), S.s.M, S.s.R, S.s.Z, s, rc, mode, fd_n, i, j, k)


def self_energy(system, s=1.0, rc=7.0, mode=0, fd_n=6) -> float:
    S = Sys(system)
    return lib().or_self_energy(C.byref(S.s.grid), S.s.M, S.s.R, S.s.Z, s, rc, mode, fd_n)


def bJ_fd(Z, s, rc, h, fd_n, dx, dy, dz) -> float:
    """-(1/4 pi) Delta_h V_J at offset (dx, dy, dz) from the nucleus (0 beyond rc)."""
    return lib().or_bJ_fd(Z, s, rc, h, fd_n, dx, dy, dz)


def atomic_guess(system, width=1.5, floor=1e-3) -> np.ndarray:
    """Superposition of one Gaussian of Z_J electrons per atom (width w, cut at 5w) plus
    floor x N/V, scaled to h^3 sum u^2 = N; returns u0 = sqrt(rho)."""
    S = Sys(system)
    u = np.zeros(system.grid.shape)
    lib().or_atomic_guess(C.byref(S.s.grid), S.s.M, S.s.R, S.s.Z, float(system.N), width, floor, _p(u))
    return u


def overlap_correction(system, s=1.0):
    S = Sys(system)
    fc = np.zeros((S.s.M, 3))
    E = lib().or_overlap_correction(S.s.M, S.s.R, S.s.Z, s, _p(fc))
    return E, fc


def moments(grid, rho) -> np.ndarray:
    rho = _f64(rho)
    m = np.zeros(10)
    g = make_grid(grid)
    lib().or_moments(C.byref(g), _p(rho), _p(m))
    return m


def phi_multipole(mom, c, y) -> float:
    return lib().or_phi_multipole(_p(_f64(mom)), _p(_f64(c)), _p(_f64(y)))


def poisson_rhs(grid, n, bc, rho) -> np.ndarray:
    rho = _f64(rho)
    out = np.zeros_like(rho)
    g = make_grid(grid)
    lib().or_poisson_rhs(C.byref(g), n, bc, _p(rho), _p(out))
    return out


def poisson_cg(grid, n, rhs, phi0=None, tol=1e-10, maxit=100000, mask=None):
    """CG on -(1/4pi) Delta_h phi = rhs; with a mask (uint8 grid array, e.g. domain_mask) the
    unknowns are the masked nodes and phi is zero elsewhere."""
    rhs = _f64(rhs)
    phi = np.zeros_like(rhs) if phi0 is None else _f64(phi0).copy()
    it = C.c_int()
    rel = C.c_double()
    g = make_grid(grid)
    if mask is None:
        st = lib().or_poisson_cg(C.byref(g), n, _p(rhs), _p(phi), tol, maxit, C.byref(it), C.byref(rel))
    else:
        m = np.ascontiguousarray(mask, dtype=np.uint8)
        st = lib().or_poisson_cg_masked(C.byref(g), n, m.ctypes.data_as(C.POINTER(C.c_ubyte)), _p(rhs),
                                        _p(phi), tol, maxit, C.byref(it), C.byref(rel))
    return phi, it.value, rel.value, st


def domain_mask(grid):
    """1 at the nodes of the ellipsoid inscribed in the box of nodes (Sec. 5.1), else 0;
    indexed [k, j, i] like every grid array."""
    g = make_grid(grid)
    m = np.zeros((grid.n[2], grid.n[1], grid.n[0]), dtype=np.uint8)
    lib().or_domain_mask(C.byref(g), m.ctypes.data_as(C.POINTER(C.c_ubyte)))
    return m


def evaluate(system, prm, u, eta=0.0, mu=0.0, phi=None):
    """One energy + residual evaluation; returns (g, energies dict, phi, cg_iters)."""
    S = Sys(system)
    u = _f64(u)
    phi = np.zeros_like(u) if phi is None else _f64(phi).copy()
    g = np.zeros_like(u)
    e = OrEnergies()
    its = C.c_long()
    lib().or_evaluate(C.byref(S.s), C.byref(prm), _p(u), eta, mu, _p(phi), _p(g), C.byref(e), C.byref(its))
    return g, {k: getattr(e, k) for k, _ in OrEnergies._fields_}, phi, its.value


def forces(system, prm, phi) -> np.ndarray:
    S = Sys(system)
    phi = _f64(phi)
    f = np.zeros((S.s.M, 3))
    lib().or_forces(C.byref(S.s), C.byref(prm), _p(phi), _p(f))
    return f


def solve(system, prm, u0):
    """Ground state; returns dict with energies, counters, u, phi, forces."""
    S = Sys(system)
    u0 = _f64(u0)
    u = np.zeros_like(u0)
    phi = np.zeros_like(u0)
    f = np.zeros((S.s.M, 3))
    res = OrResult()
    lib().or_solve(C.byref(S.s), C.byref(prm), _p(u0), _p(u), _p(phi), _p(f), C.byref(res))
    out = {k: getattr(res, k) for k, _ in OrResult._fields_}
    out.update(u=u, phi=phi, forces=f)
    return out
