"""Pins of the oracle's electrostatics: Poisson solve (Sec. 4, Eq.
Poisson:Discretized), multipole boundary values, pseudocharge and self energy
(Sec. 2), overlap correction (Appendix A)."""
import math

import numpy as np
import pytest
from scipy.special import erf

from paper_1405_6456_amd import synth
from tests import fdref


def centred_grid(n, h):
    o = -0.5 * (n - 1) * h
    return synth.Grid((n, n, n), h, (o, o, o))


def coords(g):
    z, y, x = np.meshgrid(*[g.origin[a] + g.h * np.arange(g.n[a]) for a in (2, 1, 0)], indexing="ij")
    return x, y, z


def gaussian(x, y, z, c, s):
    r2 = (x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2
    return math.pi ** -1.5 / s ** 3 * np.exp(-r2 / s ** 2)


def erf_potential(x, y, z, c, s):
    r = np.sqrt((x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2)
    with np.errstate(invalid="ignore", divide="ignore"):
        v = erf(r / s) / r
    return np.where(r == 0, 2.0 / (s * math.sqrt(math.pi)), v)


@pytest.mark.parametrize("n,nn", [(3, (9, 8, 7)), (6, (13, 13, 14))])
def test_poisson_zero_bc_matches_dense_solve(orc, n, nn):
    g = synth.Grid(nn, 0.5, (0.0, 0.0, 0.0))
    A = -fdref.dense_3d_laplacian(nn, n, g.h) / (4 * math.pi)
    rhs = synth.random_field(g, 21)
    L = np.linalg.cholesky(A)  # A is symmetric positive definite
    phi_dense = np.linalg.solve(L.T, np.linalg.solve(L, rhs.reshape(-1)))
    phi, it, rel, st = orc.poisson_cg(g, n, rhs, tol=1e-13)
    assert st == 0 and rel < 1e-13
    assert np.allclose(phi.reshape(-1), phi_dense, rtol=1e-10, atol=1e-10 * np.abs(phi_dense).max())


def test_gaussian_charge_closed_form(orc):
    # rho = pi^-3/2 s^-3 exp(-r^2/s^2) has phi = erf(r/s)/r; its multipole boundary
    # values are exact up to the tiny charge outside the box, so the error is the
    # FD truncation and shrinks fast with h (order 12).
    s = 1.5
    errs = []
    for n_nodes, h in ((29, 0.5), (57, 0.25)):
        g = centred_grid(n_nodes, h)
        x, y, z = coords(g)
        rho = gaussian(x, y, z, (0, 0, 0), s)
        rhs = orc.poisson_rhs(g, 6, 1, rho)
        phi, it, rel, st = orc.poisson_cg(g, 6, rhs, tol=1e-13)
        assert st == 0
        exact = erf_potential(x, y, z, (0, 0, 0), s)
        errs.append(np.abs(phi - exact).max())
    assert errs[1] < 1e-7
    assert errs[0] / errs[1] > 2 ** 6 or errs[1] < 1e-9


def test_multipole_expansion_far_field(orc):
    # displaced Gaussians: the monopole+dipole+quadrupole field of the grid moments
    # matches the exact potential with an error falling like r^-4 (octupole)
    g = centred_grid(41, 0.4)
    x, y, z = coords(g)
    charges = [(1.0, (1.2, -0.7, 0.5), 1.0), (-0.6, (-1.5, 0.9, -0.4), 0.8), (0.3, (0.2, 1.8, 1.1), 1.2)]
    rho = sum(q * gaussian(x, y, z, c, s) for q, c, s in charges)
    mom = orc.moments(g, rho)
    c0 = np.zeros(3)
    rng = np.random.default_rng(3)
    dirs = rng.normal(size=(20, 3))
    dirs /= np.linalg.norm(dirs, axis=1)[:, None]
    errs = {}
    for R in (10.0, 20.0, 40.0):
        e = 0.0
        for d in dirs:
            yv = R * d
            exact = sum(q * erf_potential(*[np.array(v) for v in yv], c, s) for q, c, s in charges)
            e = max(e, abs(orc.phi_multipole(mom, c0, yv) - float(exact)))
        errs[R] = e
    assert errs[10.0] < 2e-3
    assert errs[20.0] / errs[40.0] > 10  # ~16 for an r^-4 remainder
    # monopole and dipole moments equal the analytic ones
    assert abs(mom[0] - sum(q for q, _, _ in charges)) < 1e-10
    for a in range(3):
        assert abs(mom[1 + a] - sum(q * c[a] for q, c, _ in charges)) < 1e-9


def test_fold_equals_explicit_ghost_assembly(orc):
    # rhs - rho must equal (1/4 pi) Delta_h applied to a field that is zero on the
    # grid and holds phi_mp on the ghost layers (built on an enlarged grid)
    n = 6
    g = synth.Grid((15, 14, 16), 0.45, (-3.0, -2.8, -3.5))
    x, y, z = coords(g)
    rho = gaussian(x, y, z, (0.3, 0.2, -0.4), 1.0) - 0.5 * gaussian(x, y, z, (-0.5, 0.4, 0.6), 0.8)
    rhs = orc.poisson_rhs(g, n, 1, rho)
    mom = orc.moments(g, rho)
    c = np.array([g.origin[a] + 0.5 * (g.n[a] - 1) * g.h for a in range(3)])
    big = synth.Grid(tuple(m + 2 * n for m in g.n), g.h, tuple(o - n * g.h for o in g.origin))
    G = np.zeros(big.shape)
    n1, n2, n3 = g.n
    for k in range(big.n[2]):
        for j in range(big.n[1]):
            for i in range(big.n[0]):
                ii, jj, kk = i - n, j - n, k - n
                out = [not (0 <= ii < n1), not (0 <= jj < n2), not (0 <= kk < n3)]
                if sum(out) == 1:  # face ghost (star stencil never reads edges/corners)
                    yv = [big.origin[0] + i * g.h, big.origin[1] + j * g.h, big.origin[2] + k * g.h]
                    G[k, j, i] = orc.phi_multipole(mom, c, np.array(yv))
    lapG = orc.laplacian(big, n, G)[n:-n, n:-n, n:-n]
    assert np.allclose(rhs - rho, lapG / (4 * math.pi), rtol=1e-12, atol=1e-14)


def test_zero_bc_fold_is_identity(orc):
    g = synth.Grid((9, 9, 9), 0.5, (0.0, 0.0, 0.0))
    rho = synth.random_field(g, 4)
    assert np.array_equal(orc.poisson_rhs(g, 6, 0, rho), rho)


def test_pseudocharge_neutral_and_self_energy(orc):
    # h^3 sum b_J = -Z (uniform-grid quadrature of a Gaussian is spectrally
    # accurate) and the self energy tends to Z^2/(s sqrt(2 pi)) = 3.590480 for Z=3, s=1
    S = synth.single_atom()
    S.R[:] += np.array([0.123, -0.211, 0.077])
    b = orc.pseudocharge(S)
    h3 = S.grid.h ** 3
    assert abs(h3 * b.sum() + 3.0) < 1e-9
    Es = orc.self_energy(S)
    assert abs(Es - 9.0 / math.sqrt(2 * math.pi)) < 1e-6
    # sampled single-node evaluation agrees with the ball assembly
    for (i, j, k) in ((16, 16, 16), (14, 17, 18), (10, 16, 20), (0, 0, 0)):
        assert abs(orc.pseudocharge_at(S, i, j, k) - b[k, j, i]) < 1e-15


def test_overlap_correction_restores_point_repulsion(orc):
    # electrostatic energy of two bare Gaussian nuclei (u = 0) computed through the
    # grid Poisson problem, plus the Appendix-A correction, is the point-charge
    # repulsion Z^2/R
    R = 2.4
    g = centred_grid(81, 0.4)
    S = synth.System("pair", g, np.array([[-R / 2, 0.1, 0.0], [R / 2, 0.1, 0.0]]), np.array([3.0, 3.0]), 6.0)
    prm = orc.params(tf_on=0, xc=0, tol_poisson=1e-13)
    _, e, _, _ = orc.evaluate(S, prm, np.zeros(g.shape))
    # remaining error: FD/quadrature of the s = 1 Gaussians and the truncated
    # multipole boundary values (~2e-6 Ha here)
    assert abs(e["E_es"] + e["E_c"] - 9.0 / R) < 5e-6
    assert abs(e["E_c"] - 9.0 * math.erfc(R / math.sqrt(2)) / R) < 1e-14


def test_overlap_correction_forces_are_gradient(orc):
    rng = np.random.default_rng(8)
    R = rng.uniform(0, 4, size=(4, 3))
    S = synth.System("x", synth.Grid((3, 3, 3), 1.0, (0, 0, 0)), R, np.array([3.0, 2.0, 3.0, 1.0]), 9.0)
    E0, fc = orc.overlap_correction(S)
    d = 1e-6
    for J in range(4):
        for a in range(3):
            Rp, Rm = R.copy(), R.copy()
            Rp[J, a] += d
            Rm[J, a] -= d
            Ep, _ = orc.overlap_correction(synth.System("x", S.grid, Rp, S.Z, 9.0))
            Em, _ = orc.overlap_correction(synth.System("x", S.grid, Rm, S.Z, 9.0))
            assert abs(-(Ep - Em) / (2 * d) - fc[J, a]) < 1e-7
