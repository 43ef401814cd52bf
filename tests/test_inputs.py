"""Seeded synthetic inputs (host only): the workloads' grids and atoms, the initial guesses."""
import numpy as np

from paper_1405_6456_amd import synth


def test_atomic_guess_normalised_positive_and_deterministic():
    S = synth.config("fcc2")
    u = synth.atomic_guess(S)
    assert u.shape == S.grid.shape and np.all(u > 0)
    assert abs(S.grid.h ** 3 * np.sum(u * u) - S.N) <= 1e-9 * S.N
    assert np.array_equal(u, synth.atomic_guess(S))


def test_atomic_guess_peaks_at_the_atoms():
    # a lone atom at a node: the density is largest there and symmetric about it
    g = synth.Grid((25, 25, 25), 0.5, (-6.0, -6.0, -6.0))
    S = synth.System("one", g, np.array([[0.0, 0.0, 0.0]]), np.array([3.0]), 3.0)
    u = synth.atomic_guess(S)
    k, j, i = np.unravel_index(np.argmax(u), u.shape)
    assert (i, j, k) == (12, 12, 12)
    assert np.allclose(u, u[::-1, :, :]) and np.allclose(u, u[:, ::-1, :]) and np.allclose(u, u[:, :, ::-1])
    assert np.allclose(u, np.transpose(u, (2, 1, 0)))


def test_uniform_guess_mean_and_noise():
    g = synth.Grid((33, 33, 33), 0.625, (0.0, 0.0, 0.0))
    u = synth.initial_u(g, 3.0)
    base = np.sqrt(3.0 / (g.npts * g.h ** 3))
    assert np.all(np.abs(u / base - 1.0) <= 0.05 + 1e-15)
    assert abs(np.mean(u / base) - 1.0) < 5e-3


def test_workload_grids():
    # box side m*a + 16 Bohr, n = round(L/h) + 1 at h = 0.5: 63^3, 109^3, 185^3, 474^3 for
    # m = 2, 5, 10, 29
    for name, m, n in (("fcc2", 2, 63), ("fcc5", 5, 109), ("fcc10", 10, 185), ("fcc29", 29, 474)):
        S = synth.config(name)
        assert S.grid.n == (n, n, n) and S.M == 4 * m ** 3 and S.N == 3 * S.M
        assert np.all(S.R >= np.array(S.grid.origin) + 7.0)
        assert np.all(S.R <= np.array(S.grid.origin) + (n - 1) * S.grid.h - 7.0)
