"""Relaxation of the nuclei (Sec. 4: Polak-Ribiere nonlinear CG with a secant line search
over the positions, every evaluation a ground-state solve) against the oracle."""
import numpy as np
import pytest

from paper_1405_6456_amd import synth
from tests.gpu_util import ctx

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def C():
    c = ctx()
    yield c
    c.close()


def pair(d, n=27, h=0.9):
    # two Z = 3 atoms on the z axis through the box centre, d apart, slightly off axis
    g = synth.Grid((n, n, n), h, (0.0, 0.0, 0.0))
    c = 0.5 * (n - 1) * h
    R = np.array([[c, c, c - 0.5 * d], [c + 0.05, c - 0.1, c + 0.5 * d]])
    return synth.System("pair", g, R, np.array([3.0, 3.0]), 6.0)


def test_relaxed_pair_is_a_stationary_point_of_the_oracle_energy(C, orc):
    # from 4.0 Bohr apart (repulsive) the pair relaxes to its equilibrium; the defining
    # property of the result is checked with the oracle's own arithmetic: its forces at the
    # relaxed geometry vanish below the threshold (the oracle's forces are pinned to its
    # energy differences), and the energy went down
    import paper_1405_6456_amd as lib

    S = pair(4.0)
    u0 = synth.initial_u(S.grid, S.N)
    start = C.solve(S, lib.default_params(), u0, want_fields=False)
    out = C.relax(S, lib.default_params(), lib.default_relax_params(ftol=2e-4), u0)
    assert out["relax_status"] == 0 and out["status"] == 0
    assert out["fmax"] < 2e-4
    assert out["E_total"] < start["E_total"]
    # the oracle's force along the bond changes sign between 4.6 Bohr (3.7e-5 Ha/Bohr,
    # repulsive) and 5.2 Bohr (7.1e-3, attractive), close to 4.6
    d = np.linalg.norm(out["R"][1] - out["R"][0])
    assert 4.58 < d < 4.8
    Sr = synth.System("pair", S.grid, out["R"], S.Z, S.N)
    ref = orc.solve(Sr, orc.params(), synth.initial_u(S.grid, S.N))
    assert ref["status"] == 0
    assert np.linalg.norm(ref["forces"], axis=1).max() < 2e-4 + 1e-5
    assert abs(ref["E_total"] - out["E_total"]) / S.M < 1e-6


def test_relax_of_a_relaxed_geometry_takes_no_step(C):
    import paper_1405_6456_amd as lib

    S = pair(4.0)
    out = C.relax(S, lib.default_params(), lib.default_relax_params(ftol=2e-4))
    S2 = synth.System("pair", S.grid, out["R"], S.Z, S.N)
    again = C.relax(S2, lib.default_params(), lib.default_relax_params(ftol=2e-4))
    assert again["steps"] == 0 and again["solves"] == 1
    assert np.abs(again["R"] - out["R"]).max() == 0.0


def test_relax_step_cap_and_invalid_parameters(C):
    import paper_1405_6456_amd as lib

    S = pair(4.0)
    capped = C.relax(S, lib.default_params(), lib.default_relax_params(ftol=1e-9, max_steps=1))
    assert capped["relax_status"] == lib.NOT_CONVERGED and capped["steps"] == 1
    # no atom moved more than max_move in the one step
    assert np.linalg.norm(capped["R"] - S.R, axis=1).max() <= 0.3 + 1e-12
    with pytest.raises(lib.AlofdftError):
        C.relax(S, lib.default_params(), lib.default_relax_params(ftol=-1.0))
