"""GPU ground-state solves against the CPU oracle (energy per atom, forces, u, phi)."""
import numpy as np
import pytest

from paper_1405_6456_amd import synth
from tests.gpu_util import ctx, golden

pytestmark = pytest.mark.gpu

E_TOL_FP64 = 1e-6   # Ha/atom
F_TOL = 1e-4        # Ha/Bohr
E_TOL_MIXED = 1e-5  # Ha/atom


@pytest.fixture(scope="module")
def C():
    c = ctx()
    yield c
    c.close()


def small_pair():
    n = 21
    g = synth.Grid((n, n, n), 0.9, (0.0, 0.0, 0.0))
    R = np.array([[9.0, 9.0, 7.0], [9.05, 8.9, 11.0]])
    return synth.System("pair", g, R, np.array([3.0, 3.0]), 6.0)


@pytest.fixture(scope="module")
def pair_ref(orc):
    S = small_pair()
    return orc.solve(S, orc.params(), synth.initial_u(S.grid, S.N))


@pytest.mark.parametrize("method", [0, 1, 2])
def test_small_pair_matches_oracle_live(C, pair_ref, method):
    # the augmented Lagrangian, the penalty and the Lagrange-multiplier runs land on the
    # minimiser the oracle's augmented Lagrangian run finds (Sec. 5.3.2: same energies;
    # the oracle's own three methods agree on this system in the CPU tests)
    import paper_1405_6456_amd as lib

    S = small_pair()
    u0 = synth.initial_u(S.grid, S.N)
    ref = pair_ref
    assert ref["status"] == 0
    out = C.solve(S, lib.default_params(method=method), u0)
    if method == 2:
        # the Brent search on the energy reaches the energy's rounding floor near
        # ||g - eta u|| ~ 1e-6 (the oracle's run stops there too, at 1.03e-6): a stop on
        # that floor reports NOT_CONVERGED with the residual it reached
        assert out["status"] in (0, 1) and out["grad_norm"] < 3e-6
        assert abs(out["C_h"]) / S.N < 1e-12  # the constraint holds at every step
    else:
        assert out["status"] == 0
    assert abs(out["E_total"] - ref["E_total"]) / S.M < E_TOL_FP64
    assert np.abs(out["forces"] - ref["forces"]).max() < F_TOL
    assert abs(out["eta_star"] - ref["eta"]) < (1e-6 if method == 0 else 1e-5)
    assert np.abs(out["u"] - ref["u"]).max() < 1e-5 * np.abs(ref["u"]).max()


def test_energy_change_stopping_rule_matches_oracle(C, pair_ref):
    # Algorithm AugLag's |Delta E| rule (Sec. 3) reaches the same minimiser
    import paper_1405_6456_amd as lib

    S = small_pair()
    out = C.solve(S, lib.default_params(al_stop=lib.STOP_ENERGY_CHANGE, tol_energy=1e-8),
                  synth.initial_u(S.grid, S.N))
    assert out["status"] == 0 and out["outer"] >= 2 and abs(out["dE_last"]) / S.M < 1e-8
    assert abs(out["E_total"] - pair_ref["E_total"]) / S.M < E_TOL_FP64
    assert np.abs(out["forces"] - pair_ref["forces"]).max() < F_TOL


def test_fd_pseudocharge_solve_matches_oracle(C, orc):
    # the pseudocharge built as the discrete Laplacian of V_J (Sec. 4) through a whole solve
    import paper_1405_6456_amd as lib

    S = small_pair()
    u0 = synth.initial_u(S.grid, S.N)
    ref = orc.solve(S, orc.params(pseudo=1), u0)
    out = C.solve(S, lib.default_params(pseudocharge=lib.PSEUDO_FD_LAPLACIAN), u0)
    assert ref["status"] == 0 and out["status"] == 0
    assert abs(out["E_total"] - ref["E_total"]) / S.M < E_TOL_FP64
    assert np.abs(out["forces"] - ref["forces"]).max() < F_TOL
    assert abs(out["E_self"] - ref["E_self"]) < 1e-11 * abs(ref["E_self"])


def test_atomic_guess_solve_matches_oracle(C, orc):
    # the library's own atomic-density guess (no u0 passed) starts the fcc2 solve and it
    # reaches the oracle's minimiser from the uniform guess
    import paper_1405_6456_amd as lib

    gold = golden("fcc2")
    S = synth.config("fcc2")
    out = C.solve(S, lib.default_params(initial_guess=lib.GUESS_ATOMIC), None)
    assert out["status"] == 0
    assert abs(out["E_total"] - gold["result"]["E_total"]) / S.M < E_TOL_FP64
    assert np.abs(out["forces"] - np.array(gold["forces"])).max() < F_TOL


@pytest.mark.parametrize("name", ["single", "fcc2"])
@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("schedule", [1, 2])
def test_workload_matches_oracle_fixture(C, name, precision, schedule):
    import paper_1405_6456_amd as lib

    gold = golden(name)
    S = synth.config(name)
    C.set_cg_schedule(schedule)
    try:
        out = C.solve(S, lib.default_params(precision=precision), synth.initial_u(S.grid, S.N))
    finally:
        C.set_cg_schedule(-1)
    assert out["status"] == 0
    etol = E_TOL_FP64 if precision == 0 else E_TOL_MIXED
    assert abs(out["E_total"] - gold["result"]["E_total"]) / S.M < etol
    assert np.abs(out["forces"] - np.array(gold["forces"])).max() < F_TOL
    assert abs(out["C_h"]) / S.N < 1e-8
    u, phi = out["u"], out["phi"]
    us = np.array([u[k, j, i] for i, j, k in gold["sample_nodes"]])
    ps = np.array([phi[k, j, i] for i, j, k in gold["sample_nodes"]])
    # the minimiser is unique; two runs that stop at ||g|| < 1e-6 by different paths differ
    # in u and phi by O(||g||), far below 1e-5 of their maxima
    assert np.abs(us - np.array(gold["u_samples"])).max() < 1e-5 * np.abs(u).max()
    assert np.abs(ps - np.array(gold["phi_samples"])).max() < 1e-5 * np.abs(phi).max()


@pytest.mark.parametrize("precision,schedule", [(0, 1), (1, 1), (0, 2)])
def test_fcc5_solution_is_the_oracle_minimiser(C, orc, precision, schedule):
    # 500 atoms, 109^3 nodes: instead of a full oracle minimisation (hours on the host),
    # check the defining property of the result with the oracle's own arithmetic.  The
    # discrete minimiser under C_h(u) = 0 is unique; at the GPU's u* with its multiplier
    # eta*, the oracle's residual of the Euler-Lagrange equation (Sec. 4, mu term off)
    # must vanish to the solver's tolerance, and the oracle's energy and Hellmann-Feynman
    # forces at u* must equal the GPU's.  An energy error of the minimiser is then of
    # order ||g||^2, far below 1e-6 Ha/atom.
    import paper_1405_6456_amd as lib

    S = synth.config("fcc5")
    C.set_cg_schedule(schedule)
    try:
        out = C.solve(S, lib.default_params(precision=precision), synth.initial_u(S.grid, S.N))
    finally:
        C.set_cg_schedule(-1)
    assert out["status"] == 0
    assert abs(out["C_h"]) / S.N < 1e-8
    prm = orc.params()
    g, e, phi_o, _ = orc.evaluate(S, prm, out["u"], eta=out["eta_star"], mu=0.0, phi=out["phi"])
    h3 = S.grid.h ** 3
    gnorm = float(np.sqrt(h3 * np.sum(g * g)))
    assert gnorm < 1e-5
    assert abs(e["E_total"] - out["E_total"]) / S.M < 1e-9
    f_o = orc.forces(S, prm, phi_o)
    assert np.abs(f_o - out["forces"]).max() < 1e-6


@pytest.mark.timeout(900)
def test_fcc10_fp32_refined_solution_is_the_oracle_minimiser(orc, capsys):
    # 4000 atoms, 185^3 nodes, FP32 stencil and CG inside FP64 refinement, from the
    # library's atomic-density guess: the same check as for fcc5 (the oracle's Euler-Lagrange
    # residual, energy and forces at the GPU's u* and eta*).  The solve takes minutes; the
    # library's own progress lines (one per 100 NLCG steps and per AL step) go to stderr.
    import os

    import paper_1405_6456_amd as lib

    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    S = synth.config("fcc10")
    os.environ["ALOFDFT_PROGRESS"] = "1"
    try:
        c = lib.Context(0)
    finally:
        del os.environ["ALOFDFT_PROGRESS"]
    try:
        with capsys.disabled():
            out = c.solve(S, lib.default_params(precision=lib.FP32_REFINED, initial_guess=lib.GUESS_ATOMIC), None)
    finally:
        c.close()
    assert out["status"] == 0
    assert abs(out["C_h"]) / S.N < 1e-8
    prm = orc.params()
    g, e, phi_o, _ = orc.evaluate(S, prm, out["u"], eta=out["eta_star"], mu=0.0, phi=out["phi"])
    gnorm = float(np.sqrt(S.grid.h ** 3 * np.sum(g * g)))
    assert gnorm < 1e-5
    assert abs(e["E_total"] - out["E_total"]) / S.M < 1e-9
    f_o = orc.forces(S, prm, phi_o)
    assert np.abs(f_o - out["forces"]).max() < 1e-6


@pytest.mark.parametrize("precision", [0, 1])
def test_ellipsoid_domain_solve_matches_oracle(C, orc, precision):
    # the atom off the centre of a 16 Bohr box, the Dirichlet conditions on the inscribed
    # ellipsoid (Sec. 5.1): the GPU's ground state equals the oracle's, with u and phi zero at
    # every node outside
    import paper_1405_6456_amd as lib

    S = synth.single_atom(L=16.0, n=21)
    S.R[0] += np.array([0.13, -0.07, 0.05])
    u0 = synth.initial_u(S.grid, S.N)
    ref = orc.solve(S, orc.params(bc=0, domain=1), u0)
    out = C.solve(S, lib.default_params(phi_bc=0, domain=lib.DOMAIN_ELLIPSOID, precision=precision), u0)
    assert ref["status"] == 0 and out["status"] == 0
    m = orc.domain_mask(S.grid).astype(bool)
    assert np.all(out["u"][~m] == 0.0) and np.all(out["phi"][~m] == 0.0)
    etol = E_TOL_FP64 if precision == 0 else E_TOL_MIXED
    assert abs(out["E_total"] - ref["E_total"]) / S.M < etol
    assert np.abs(out["forces"] - ref["forces"]).max() < F_TOL
    assert np.abs(out["u"] - ref["u"]).max() < 1e-5 * np.abs(ref["u"]).max()
