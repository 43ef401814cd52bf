"""Seeded synthetic inputs: grids, Al-like fcc clusters, initial guesses, request streams.

This module only generates inputs.  It holds none of the method's arithmetic and
is the one piece of Python shared by the GPU path (bench, serving) and the CPU
oracle tests.  Every random number comes from SplitMix64 (Steele, Lea & Flood,
"Fast splittable pseudorandom number generators", 2014), written out below, so a
stream is reproducible from its seed alone:

    next(state):  state += 0x9E3779B97F4A7C15
                  z = state
                  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9
                  z = (z ^ (z >> 27)) * 0x94D049BB133111EB
                  return z ^ (z >> 31)

A uniform double in [0, 1) is (z >> 11) * 2**-53.

Arrays on a grid are numpy arrays of shape (n3, n2, n1) in C order, so the flat
index of node (i, j, k) is i + n1*(j + n2*k): x fastest.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

#: fcc conventional-cell basis, in units of the lattice constant
FCC_BASIS = ((0.0, 0.0, 0.0), (0.0, 0.5, 0.5), (0.5, 0.0, 0.5), (0.5, 0.5, 0.0))


def splitmix64(state: np.ndarray | int) -> np.ndarray:
    """One SplitMix64 step from each state (vectorised, wrapping uint64 arithmetic)."""
    z = np.asarray(state, dtype=np.uint64) + _GAMMA
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def uniform01(z: np.ndarray) -> np.ndarray:
    """53-bit uniform doubles in [0, 1) from SplitMix64 outputs."""
    return (np.asarray(z, dtype=np.uint64) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def stream(seed: int, count: int) -> np.ndarray:
    """The first `count` uniforms of the SplitMix64 stream started at `seed`."""
    t = np.arange(1, count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        states = np.uint64(seed) + (t - np.uint64(1)) * _GAMMA
    return uniform01(splitmix64(states))


def node_noise(seed: int, npts: int) -> np.ndarray:
    """xi in [-1, 1) per node: xi_i = 2*U(SplitMix64(seed XOR i)) - 1."""
    idx = np.arange(npts, dtype=np.uint64)
    return 2.0 * uniform01(splitmix64(np.uint64(seed) ^ idx)) - 1.0


@dataclasses.dataclass(frozen=True)
class Grid:
    """Uniform grid: node (i, j, k) sits at origin + h*(i, j, k), i < n[0] etc."""

    n: tuple
    h: float
    origin: tuple

    @property
    def shape(self):
        """numpy shape (n3, n2, n1) of a grid array."""
        return (self.n[2], self.n[1], self.n[0])

    @property
    def npts(self) -> int:
        return int(self.n[0]) * int(self.n[1]) * int(self.n[2])


@dataclasses.dataclass
class System:
    """Nuclei on a grid: positions R (M, 3), valence charges Z (M,), N electrons."""

    name: str
    grid: Grid
    R: np.ndarray
    Z: np.ndarray
    N: float

    @property
    def M(self) -> int:
        return int(self.R.shape[0])


def random_field(grid: Grid, seed: int) -> np.ndarray:
    """Uniform [-1, 1) field on the grid (stencil and solver test input)."""
    return node_noise(seed, grid.npts).reshape(grid.shape)


def initial_u(grid: Grid, N: float, seed: int = 6456, amp: float = 0.05) -> np.ndarray:
    """u0 = sqrt(N/V) (1 + amp*xi), V = n1 n2 n3 h^3, xi from node_noise(seed)."""
    V = grid.npts * grid.h ** 3
    return (math.sqrt(N / V) * (1.0 + amp * node_noise(seed, grid.npts))).reshape(grid.shape)


def atomic_guess(system, width: float = 1.5, floor: float = 1e-3) -> np.ndarray:
    """u0 = sqrt(rho0) for a superposition of one Gaussian of Z_J electrons per atom,
    rho_J(r) = Z_J (pi w^2)^(-3/2) exp(-r^2/w^2) (cut at r = 5w), plus floor x N/V, scaled
    so that h^3 sum rho0 = N: an initial guess of the atomic-density kind the paper uses
    for its clusters, for systems where the uniform guess starts too far away."""
    g = system.grid
    h = g.h
    rho = np.zeros(g.shape)
    rc = 5.0 * width
    norm = (math.pi * width * width) ** -1.5
    axes = [g.origin[a] + h * np.arange(g.n[a]) for a in range(3)]
    for J in range(system.M):
        lo = [max(0, int(math.floor((system.R[J, a] - rc - g.origin[a]) / h))) for a in range(3)]
        hi = [min(g.n[a] - 1, int(math.ceil((system.R[J, a] + rc - g.origin[a]) / h))) for a in range(3)]
        if any(lo[a] > hi[a] for a in range(3)):
            continue
        d = [axes[a][lo[a]:hi[a] + 1] - system.R[J, a] for a in range(3)]
        r2 = d[2][:, None, None] ** 2 + d[1][None, :, None] ** 2 + d[0][None, None, :] ** 2
        rho[lo[2]:hi[2] + 1, lo[1]:hi[1] + 1, lo[0]:hi[0] + 1] += system.Z[J] * norm * np.exp(-r2 / (width * width))
    V = g.npts * h ** 3
    rho += floor * system.N / V
    rho *= system.N / (h ** 3 * rho.sum())
    return np.sqrt(rho)


def displacements(M: int, seed: int, magnitude: float = 0.1) -> np.ndarray:
    """Random displacement of exactly `magnitude` Bohr per atom, uniform direction.

    Atom a takes the uniforms number 2a+1 and 2a+2 of the stream: cos(theta) =
    2*u1 - 1, azimuth = 2*pi*u2.
    """
    u = stream(seed, 2 * M).reshape(M, 2)
    ct = 2.0 * u[:, 0] - 1.0
    st = np.sqrt(np.maximum(0.0, 1.0 - ct * ct))
    az = 2.0 * math.pi * u[:, 1]
    return magnitude * np.stack([st * np.cos(az), st * np.sin(az), ct], axis=1)


def fcc_cluster(m: int, a: float = 7.6, disp: float = 0.1, seed: int = 1405,
                Z: float = 3.0, vacuum: float = 8.0, h: float = 0.5, name: str | None = None) -> System:
    """m x m x m conventional fcc cells (4 m^3 atoms, open faces), displaced.

    Atoms are ordered i, j, k (cell indices, i outermost) then basis atom.  The
    box has side L = m*a + 2*vacuum, n = round(L/h) + 1 nodes per axis, and is
    centred on the centre (m*a/2)(1,1,1) of the cell block.
    """
    pos = []
    for i in range(m):
        for j in range(m):
            for k in range(m):
                for b in FCC_BASIS:
                    pos.append((a * (i + b[0]), a * (j + b[1]), a * (k + b[2])))
    R = np.array(pos, dtype=np.float64)
    if disp:
        R = R + displacements(len(R), seed, disp)
    L = m * a + 2.0 * vacuum
    n = int(round(L / h)) + 1
    c = 0.5 * m * a
    o = c - 0.5 * (n - 1) * h
    grid = Grid((n, n, n), h, (o, o, o))
    Zs = np.full(len(R), Z, dtype=np.float64)
    return System(name or f"fcc{m}", grid, R, Zs, float(Zs.sum()))


def single_atom(L: float = 20.0, n: int = 33, Z: float = 3.0) -> System:
    """One nucleus at the centre of an L-Bohr cube sampled by n^3 nodes (inclusive)."""
    h = L / (n - 1)
    grid = Grid((n, n, n), h, (0.0, 0.0, 0.0))
    R = np.array([[L / 2, L / 2, L / 2]], dtype=np.float64)
    return System("single", grid, R, np.array([Z]), float(Z))


def config(name: str) -> System:
    """The named synthetic workloads.

    single   one Z=3 atom in a 20 Bohr cube, 33^3 nodes, h = 0.625
    fcc2     2^3 cells, 32 atoms,  63^3 nodes, h = 0.5, displacement seed 1405+2
    fcc5     5^3 cells, 500 atoms, 109^3 nodes, seed 1405+3
    fcc10    10^3 cells, 4000 atoms, 185^3 nodes, seed 1405+5
    fcc29    29^3 cells, 97556 atoms, 474^3 nodes, seed 1405+29 (the size of the paper's
             largest cluster, on one device)
    """
    if name == "single":
        return single_atom()
    if name == "fcc2":
        return fcc_cluster(2, seed=1405 + 2, name=name)
    if name == "fcc5":
        return fcc_cluster(5, seed=1405 + 3, name=name)
    if name == "fcc10":
        return fcc_cluster(10, seed=1405 + 5, name=name)
    if name == "fcc29":
        return fcc_cluster(29, seed=1405 + 29, name=name)
    raise KeyError(name)


def serving_requests(count: int = 64, seed_m: int = 2014, seed_disp0: int = 10000):
    """Request k: fcc cluster with m ~ U{1,2,3} (stream seed_m), displacement seed seed_disp0 + k."""
    u = stream(seed_m, count)
    ms = 1 + np.minimum((3.0 * u).astype(np.int64), 2)
    return [fcc_cluster(int(m), seed=seed_disp0 + k, name=f"req{k}_fcc{int(m)}") for k, m in enumerate(ms)]


def arrival_times(count: int, rate: float, seed: int = 2015) -> np.ndarray:
    """Poisson-process arrival times (s): exponential gaps -ln(1-u)/rate."""
    u = stream(seed, count)
    return np.cumsum(-np.log1p(-u) / rate)
