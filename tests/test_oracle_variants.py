"""Pins of the oracle's paper-faithful variants: the pseudocharge built as the discrete
Laplacian of the nuclear potential (Sec. 4, the b_J formula after Eq. FD:Laplacian), the
superposition of atomic densities as initial guess (Sec. 4), and the energy-change
stopping rule of Algorithm AugLag (Sec. 3)."""
import math

import numpy as np
import pytest
from scipy.special import erf

from paper_1405_6456_amd import synth


def one_atom(h, L=16.0, R=(8.03, 7.91, 8.11), Z=3.0):
    n = int(round(L / h)) + 1
    g = synth.Grid((n, n, n), h, (0.0, 0.0, 0.0))
    return synth.System("a", g, np.array([R]), np.array([Z]), Z)


@pytest.mark.parametrize("fd_n", [2, 3, 6])
def test_fd_pseudocharge_is_neutral(orc, fd_n):
    # h^3 sum_i (Delta_h V)_i over a ball equals the discrete flux of grad V through its
    # surface, which is the Coulomb flux -4 pi Z up to the stencil's truncation error
    for h in (0.5, 0.25):
        S = one_atom(h)
        b = orc.pseudocharge(S, mode=1, fd_n=fd_n)
        assert abs(h ** 3 * b.sum() + 3.0) < 2e-8 * 3.0


def test_fd_pseudocharge_converges_to_gaussian_at_stencil_order(orc):
    # -(1/4 pi) Delta_h V_J -> -(1/4 pi) Delta V_J = the Gaussian charge; order 2n = 4:
    # halving h divides the largest nodal difference by about 2^4 once h is small
    errs = []
    for h in (0.5, 0.25, 0.125):
        S = one_atom(h, L=10.0, R=(5.03, 4.91, 5.11))
        bf = orc.pseudocharge(S, mode=1, fd_n=2, rc=4.9)
        bg = orc.pseudocharge(S, mode=0, rc=4.9)
        errs.append(np.abs(bf - bg).max())
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert r1 > 12 and 14 < r2 < 18, (errs, r1, r2)


def test_fd_pseudocharge_order2_is_the_seven_point_laplacian(orc):
    # n = 1: the 7-point Laplacian (sum of the six neighbours - 6 f)/h^2 of V = -Z erf(r/s)/r
    Z, s, h = 3.0, 1.0, 0.4
    V = lambda x, y, z: -Z * erf(math.sqrt(x * x + y * y + z * z) / s) / math.sqrt(x * x + y * y + z * z)
    for d in ((0.13, -0.21, 0.37), (1.1, 0.4, -0.9), (2.3, -1.7, 0.2)):
        x, y, z = d
        lap = (V(x + h, y, z) + V(x - h, y, z) + V(x, y + h, z) + V(x, y - h, z) + V(x, y, z + h) +
               V(x, y, z - h) - 6 * V(x, y, z)) / h ** 2
        assert abs(orc.bJ_fd(Z, s, 7.0, h, 1, x, y, z) + lap / (4 * math.pi)) < 1e-12 * abs(lap)
    assert orc.bJ_fd(Z, s, 7.0, h, 1, 7.1, 0.0, 0.0) == 0.0  # outside the ball


def test_fd_pseudocharge_sampled_matches_full(orc):
    S = one_atom(0.5)
    b = orc.pseudocharge(S, mode=1, fd_n=6)
    for i, j, k in ((16, 16, 16), (10, 17, 20), (5, 16, 16), (31, 2, 4)):
        assert abs(orc.pseudocharge_at(S, i, j, k, mode=1, fd_n=6) - b[k, j, i]) < 1e-15


def test_fd_self_energy_approaches_analytic(orc):
    # 1/2 int b V for a Gaussian charge is Z^2/(s sqrt(2 pi)); the discrete Laplacian's
    # charge approaches it as h -> 0
    exact = 9.0 / math.sqrt(2 * math.pi)
    e = [abs(orc.self_energy(one_atom(h), mode=1, fd_n=6) - exact) for h in (0.5, 0.25)]
    assert e[1] < 1e-6 and e[1] < e[0]


def test_atomic_guess_single_atom_closed_form(orc):
    # one atom, no floor: the nodal sum of a Gaussian of width w = 1.5 at h = 0.5 is its
    # integral to e^{-pi^2 w^2/h^2}, and the part beyond the 5w cut is ~1e-10 of it, so the
    # scaling to N = Z is 1 to that accuracy and u^2 at a node is the Gaussian itself
    S = one_atom(0.5, L=20.0, R=(10.0, 10.0, 10.0))
    u = orc.atomic_guess(S, width=1.5, floor=0.0)
    w = 1.5
    peak = 3.0 * (math.pi * w * w) ** -1.5
    assert abs(u[20, 20, 20] ** 2 - peak) < 2e-10 * peak
    assert abs(u[20, 20, 23] ** 2 - peak * math.exp(-(1.5 ** 2) / w ** 2)) < 2e-10 * peak
    assert u[20, 20, 36] == 0.0  # beyond the 5w cut


def test_atomic_guess_normalised_and_matches_generator(orc):
    S = synth.config("fcc2")
    u = orc.atomic_guess(S)
    assert abs(S.grid.h ** 3 * np.sum(u * u) - S.N) < 1e-10 * S.N
    # the input generator builds the same guess (independent code; it cuts each Gaussian
    # to a cube of half-side 5w instead of the ball, a difference below e^-25 of the peak)
    assert np.abs(u - synth.atomic_guess(S)).max() < 1e-8 * u.max()


def test_energy_change_stopping_rule(orc):
    # Algorithm AugLag's rule |E_q - E_(q-1)| < tol per atom stops at the same minimiser
    # as the constraint rule on the two-atom system
    S = synth.System("pair", synth.Grid((21, 21, 21), 0.9, (0, 0, 0)),
                     np.array([[9.0, 9.0, 7.0], [9.05, 8.9, 11.0]]), np.array([3.0, 3.0]), 6.0)
    u0 = synth.initial_u(S.grid, S.N)
    a = orc.solve(S, orc.params(), u0)
    b = orc.solve(S, orc.params(al_stop=1, tol_energy=1e-8), u0)
    assert a["status"] == 0 and b["status"] == 0
    assert b["al_iters"] >= 2 and abs(b["dE_last"]) / S.M < 1e-8
    assert abs(a["E_total"] - b["E_total"]) / S.M < 1e-8


# ---------------------------------------------------------------- ellipsoidal active domain (Sec. 5.1)
def test_domain_mask_is_the_inscribed_ellipsoid(orc):
    # the nodes of the ellipsoid inscribed in the box of nodes: the count follows its volume
    # (4/3) pi abc in index units up to a surface term, the mask has the box's reflection
    # symmetries, holds the centre and the face centres and leaves out the corners
    g = synth.Grid((41, 33, 25), 0.5, (0.0, 0.0, 0.0))
    m = orc.domain_mask(g).astype(bool)
    a, b, c = 20.0, 16.0, 12.0
    vol = 4.0 / 3.0 * np.pi * a * b * c
    assert abs(m.sum() - vol) < 0.05 * vol
    assert np.array_equal(m, m[::-1, :, :]) and np.array_equal(m, m[:, ::-1, :]) and np.array_equal(m, m[:, :, ::-1])
    assert m[12, 16, 20] and m[12, 16, 0] and m[12, 0, 20] and m[0, 16, 20]
    assert not m[0, 0, 0] and not m[24, 32, 40]
    k, j, i = np.nonzero(m)
    assert np.all(((i - a) / a) ** 2 + ((j - b) / b) ** 2 + ((k - c) / c) ** 2 <= 1 + 1e-12)


def test_masked_poisson_is_the_restricted_dense_solve(orc):
    # A restricted to the domain (rows and columns of the free nodes), solved densely
    g = synth.Grid((9, 8, 7), 0.6, (0.0, 0.0, 0.0))
    n = 3
    m = orc.domain_mask(g).reshape(-1).astype(bool)
    N = m.size
    A = np.zeros((N, N))
    for col in range(N):
        e = np.zeros(N)
        e[col] = 1.0
        A[:, col] = -orc.laplacian(g, n, e.reshape(g.n[2], g.n[1], g.n[0])).reshape(-1) / (4 * np.pi)
    rng = np.random.default_rng(5)
    rhs = rng.standard_normal(N)
    idx = np.nonzero(m)[0]
    ref = np.zeros(N)
    ref[idx] = np.linalg.solve(A[np.ix_(idx, idx)], rhs[idx])
    phi, its, rel, st = orc.poisson_cg(g, n, rhs.reshape(g.n[2], g.n[1], g.n[0]), tol=1e-13,
                                       mask=m.reshape(g.n[2], g.n[1], g.n[0]))
    assert st == 0
    assert np.abs(phi.reshape(-1) - ref).max() < 1e-10 * np.abs(ref).max()
    assert np.all(phi.reshape(-1)[~m] == 0.0)


def test_uniform_sphere_potential_converges(orc):
    # -(1/4 pi) Delta phi = 1 in a sphere of radius a, phi = 0 outside: phi(0) = (2 pi / 3) a^2.
    # The stair-stepped Dirichlet surface makes the error first order in h (the first Dirichlet
    # nodes lie beyond a, so it is positive)
    a = 4.0
    errs = []
    for n in (17, 33, 65):
        h = 2 * a / (n - 1)
        g = synth.Grid((n, n, n), h, (-a, -a, -a))
        m = orc.domain_mask(g)
        phi, _, _, st = orc.poisson_cg(g, 6, m.astype(np.float64), tol=1e-12, mask=m)
        assert st == 0
        c = n // 2
        errs.append((phi[c, c, c] - 2 * np.pi / 3 * a * a) / (2 * np.pi / 3 * a * a))
    assert all(e > 0 for e in errs)
    assert errs[0] < 0.06 and errs[1] < 0.6 * errs[0] and errs[2] < 0.6 * errs[1]


def test_ellipsoid_domain_solve(orc):
    # an atom at the centre of the box: the ellipsoid keeps u and phi zero outside it, the
    # ground state stays close to the box's (the density decays long before the surface), and
    # the ellipsoid with multipole values for phi is refused
    S = synth.single_atom(L=16.0, n=21)
    u0 = synth.initial_u(S.grid, S.N)
    box = orc.solve(S, orc.params(bc=0), u0)
    ell = orc.solve(S, orc.params(bc=0, domain=1), u0)
    assert box["status"] == 0 and ell["status"] == 0
    m = orc.domain_mask(S.grid).astype(bool)
    assert np.all(ell["u"][~m] == 0.0) and np.all(ell["phi"][~m] == 0.0)
    assert abs(ell["E_total"] - box["E_total"]) < 2e-3
    assert abs(ell["E_total"] - box["E_total"]) > 1e-9  # the domain does change the problem
    assert abs(S.grid.h ** 3 * np.sum(ell["u"] ** 2) - S.N) / S.N < 1e-8
    bad = orc.solve(S, orc.params(bc=1, domain=1), u0)
    assert bad["status"] == -5
