"""Pins of the oracle's minimisers: augmented Lagrangian (Sec. 3, Algorithm
AugLag), penalty and Lagrange-multiplier variants (Sec. 5.3.2), gradient
consistency and forces (Sec. 2, Eq. Force:Nuclei)."""
import math

import numpy as np
import pytest

from paper_1405_6456_amd import synth
from tests import fdref


def centred_grid(n, h):
    o = -0.5 * (n - 1) * h
    return synth.Grid((n, n, n), h, (o, o, o))


def coords(g):
    return np.meshgrid(*[g.origin[a] + g.h * np.arange(g.n[a]) for a in (2, 1, 0)], indexing="ij")[::-1]


def pair_system(h=0.9, L=18.0, dz=0.0, shift=(0.0, 0.0, 0.0)):
    n = int(round(L / h)) + 1
    g = synth.Grid((n, n, n), h, tuple(shift))
    R = np.array([[9.0, 9.0, 7.0 + dz], [9.05, 8.9, 11.0]]) + np.array(shift)
    return synth.System("pair", g, R, np.array([3.0, 3.0]), 6.0)


# ---------------------------------------------------------------- harmonic oscillator
@pytest.fixture(scope="module")
def ho(orc):
    om, lam, Ne = 0.5, 0.2, 2.0
    g = centred_grid(29, 0.5)
    x, y, z = coords(g)
    vext = 0.5 * om ** 2 * (x * x + y * y + z * z)
    xs = g.origin[0] + g.h * np.arange(g.n[0])
    H1 = -(lam / 2) * fdref.dense_1d_second(g.n[0], 6, g.h) + np.diag(0.5 * om ** 2 * xs ** 2)
    w, V = np.linalg.eigh(H1)
    S = synth.System("ho", g, np.zeros((1, 3)), np.array([1.0]), Ne)
    return dict(S=S, vext=vext, eta=3 * w[0], psi=V[:, 0], Ne=Ne, om=om, lam=lam)


@pytest.mark.parametrize("method", [0, 1, 2])
def test_harmonic_oscillator(orc, ho, method):
    # vW + fixed V = w^2 r^2/2 only: the minimiser is the ground state of the FD
    # Hamiltonian -(lambda/2) Delta_h + V, a product of 1-D ground states whose
    # eigenvalue eta* is 3x that of the 1-D matrix (dense eigensolver).  Continuum
    # limit: eta* = 1.5 w sqrt(lambda).
    S = ho["S"]
    tolc = 1e-10 if method == 0 else 1e-8
    tolg = 1e-8 if method == 0 else 1e-6
    prm = orc.params(tf_on=0, xc=0, hartree_on=0, vext=ho["vext"], method=method, tol_grad=tolg,
                     tol_constraint=tolc)
    r = orc.solve(S, prm, synth.initial_u(S.grid, ho["Ne"]))
    assert r["status"] in ((0,) if method < 2 else (0, 1))
    eta_tol = {0: 1e-8, 1: 1e-6, 2: 1e-8}[method]
    assert abs(r["eta"] - ho["eta"]) < eta_tol
    assert abs(r["E_total"] / ho["Ne"] - ho["eta"]) < 1e-8
    assert abs(ho["eta"] - 1.5 * ho["om"] * math.sqrt(ho["lam"])) < 1e-5
    # minimiser shape: u*/sqrt(N) equals the separable product of 1-D ground states
    p = np.abs(ho["psi"]) / math.sqrt(S.grid.h)
    prod = np.einsum("k,j,i->kji", p, p, p) * math.sqrt(ho["Ne"])
    assert np.abs(r["u"] - prod).max() < 2e-4 * prod.max()


# ---------------------------------------------------------------- small Hartree system
@pytest.fixture(scope="module")
def pair_runs(orc):
    S = pair_system()
    u0 = synth.initial_u(S.grid, S.N)
    out = {}
    for method in (0, 1, 2):
        out[method] = orc.solve(S, orc.params(method=method), u0)
    return S, out


def test_al_converges(pair_runs):
    S, runs = pair_runs
    r = runs[0]
    assert r["status"] == 0
    assert abs(r["C"]) / S.N < 1e-8 and r["gnorm"] < 1e-6 and r["poisson_relres"] < 1e-10


@pytest.mark.slow
def test_variants_agree(pair_runs):
    # the same minimiser from the augmented Lagrangian, penalty and Lagrange
    # multiplier methods (the paper's Table 5 shows agreement to 1e-4 eV/atom)
    S, runs = pair_runs
    E = [runs[m]["E_total"] for m in (0, 1, 2)]
    assert max(E) - min(E) < 1e-6 * S.M
    for m in (1, 2):
        assert np.abs(runs[m]["forces"] - runs[0]["forces"]).max() < 1e-4
        assert abs(runs[m]["eta"] - runs[0]["eta"]) < 1e-5
    assert runs[2]["gnorm"] < 1e-5


def test_multiplier_is_rayleigh_quotient(orc, pair_runs):
    # at the minimiser eta* = [h^3 u.(-lambda/2 Delta u) + h^3 V_eff u^2]/N, i.e.
    # h^3 u.(H u)/N with H u the residual taken at eta = 0 and no penalty
    S, runs = pair_runs
    r = runs[0]
    g0, e, _, _ = orc.evaluate(S, orc.params(), r["u"], eta=0.0, mu=0.0, phi=r["phi"])
    rq = S.grid.h ** 3 * (r["u"] * g0).sum() / S.N
    assert abs(rq - r["eta"]) < 1e-7


def test_forces_balance_for_pair(pair_runs):
    S, runs = pair_runs
    f = runs[0]["forces"]
    # two identical atoms: equal and opposite forces along the axis up to the
    # egg-box effect of the grid
    assert abs(f[0, 2] + f[1, 2]) < 1e-4
    assert f[0, 2] < 0 < f[1, 2]  # Gaussian cores 4 Bohr apart repel


# ---------------------------------------------------------------- gradient consistency
def test_residual_is_half_derivative_of_L(orc):
    # with the zero-Dirichlet phi the discrete problem is exactly variational:
    # 2 h^3 g.v = dL/d eps (u + eps v) (central difference, phi re-solved)
    S = pair_system(h=1.0)
    u = synth.initial_u(S.grid, S.N)
    v = 0.3 * synth.random_field(S.grid, 77) * u
    prm = orc.params(bc=0, tol_poisson=1e-14)
    eta, mu = -0.15, 0.7
    g, _, _, _ = orc.evaluate(S, prm, u, eta, mu)
    eps = 1e-4
    _, ep, _, _ = orc.evaluate(S, prm, u + eps * v, eta, mu)
    _, em, _, _ = orc.evaluate(S, prm, u - eps * v, eta, mu)
    fd = (ep["L"] - em["L"]) / (2 * eps)
    an = 2 * S.grid.h ** 3 * (g * v).sum()
    assert abs(fd - an) < 1e-7 * max(1.0, abs(an))


# ---------------------------------------------------------------- forces vs energy
@pytest.mark.slow
@pytest.mark.parametrize("pseudo", [0, 1])
def test_forces_match_energy_difference(orc, pseudo):
    # f_z on atom 0 against -dE/dz by a central difference of converged energies
    # (zero-Dirichlet phi, so the energy is exactly variational in phi).  The force
    # formula (App. A) takes the order-2n finite-difference gradient of the sampled
    # pseudocharge, not its exact derivative, so it matches the energy difference only
    # up to that gradient's error on the Gaussian: about 2e-4 Ha/Bohr at h = 0.75,
    # 2e-5 at h = 0.6 (it falls like a high power of h).  Hence h = 0.6 here.  pseudo 1:
    # the pseudocharge built as the discrete Laplacian of V_J (Sec. 4), same formula.
    d = 0.01
    h = 0.6
    prm = orc.params(bc=0, tol_constraint=1e-10, tol_grad=1e-8, tol_poisson=1e-12, pseudo=pseudo)
    base = pair_system(h=h)
    u0 = synth.initial_u(base.grid, base.N)
    r0 = orc.solve(base, prm, u0)
    Ep = orc.solve(pair_system(h=h, dz=d), prm, r0["u"])["E_total"]
    Em = orc.solve(pair_system(h=h, dz=-d), prm, r0["u"])["E_total"]
    assert abs(-(Ep - Em) / (2 * d) - r0["forces"][0, 2]) < 1e-4


# ---------------------------------------------------------------- invariances
def test_translation_invariance(orc):
    # atoms and grid shifted together: the discrete problem is unchanged
    prm = orc.params()
    a = pair_system(h=1.0)
    b = pair_system(h=1.0, shift=(3.25, -1.5, 0.75))
    u = synth.initial_u(a.grid, a.N)
    _, ea, _, _ = orc.evaluate(a, prm, u, -0.2, 1.0)
    _, eb, _, _ = orc.evaluate(b, prm, u, -0.2, 1.0)
    assert abs(ea["E_total"] - eb["E_total"]) < 1e-10 * abs(ea["E_total"])


def test_single_atom_symmetry(orc):
    # an atom on a node at the box centre: the minimiser has the cube symmetry and
    # the force vanishes
    S = synth.single_atom(L=16.0, n=21)
    r = orc.solve(S, orc.params(), synth.initial_u(S.grid, S.N))
    assert r["status"] == 0
    assert np.abs(r["forces"]).max() < 1e-8
    u = r["u"]
    for t in (u.transpose(1, 0, 2), u.transpose(2, 1, 0), u[::-1], u[:, ::-1], u[:, :, ::-1]):
        assert np.abs(t - u).max() < 1e-5 * u.max()
