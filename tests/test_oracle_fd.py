"""Pins of the oracle's FD weights and stencil (Sec. 4, Eq. FD:Laplacian and the
gradient weights used for the forces) against independent derivations."""
from fractions import Fraction

import numpy as np
import pytest

from paper_1405_6456_amd import synth
from tests import fdref

# Textbook central second-difference coefficients (centre, then p = 1..n), h = 1.
TEXTBOOK_D2 = {
    1: [-2, 1],
    2: [Fraction(-5, 2), Fraction(4, 3), Fraction(-1, 12)],
    3: [Fraction(-49, 18), Fraction(3, 2), Fraction(-3, 20), Fraction(1, 90)],
    4: [Fraction(-205, 72), Fraction(8, 5), Fraction(-1, 5), Fraction(8, 315), Fraction(-1, 560)],
}
# Textbook central first-difference coefficients (p = 1..n), h = 1.
TEXTBOOK_D1 = {
    1: [Fraction(1, 2)],
    2: [Fraction(2, 3), Fraction(-1, 12)],
    3: [Fraction(3, 4), Fraction(-3, 20), Fraction(1, 60)],
    4: [Fraction(4, 5), Fraction(-1, 5), Fraction(4, 105), Fraction(-1, 280)],
}


@pytest.mark.parametrize("n", [1, 2, 3, 4])
def test_weights_match_textbook(orc, n):
    w = orc.weights(n, 1.0)
    # the 1-D centre coefficient is 2 w_0 (the p = 0 term appears as f_i + f_i)
    got = [2 * w[0]] + list(w[1:])
    assert np.allclose(got, [float(x) for x in TEXTBOOK_D2[n]], rtol=1e-14, atol=1e-15)
    wt = orc.grad_weights(n, 1.0)
    assert np.allclose(wt[1:], [float(x) for x in TEXTBOOK_D1[n]], rtol=1e-14, atol=1e-15)


@pytest.mark.parametrize("n", range(1, 9))
@pytest.mark.parametrize("h", [1.0, 0.5, 0.625])
def test_weights_match_moment_conditions(orc, n, h):
    c = fdref.second_derivative(n)
    w = orc.weights(n, h)
    assert np.allclose([2 * w[0] * h * h] + list(w[1:] * h * h), [float(x) for x in c], rtol=1e-13, atol=1e-16)
    ct = fdref.first_derivative(n)
    wt = orc.grad_weights(n, h)
    assert np.allclose(wt[1:] * h, [float(x) for x in ct], rtol=1e-13, atol=1e-16)


def test_order12_rationals(orc):
    # order 12 (n = 6): w_0 = -5369/3600, w_1..w_6 as exact rationals (h = 1)
    w = orc.weights(6, 1.0)
    exact = [Fraction(-5369, 3600), Fraction(12, 7), Fraction(-15, 56), Fraction(10, 189),
             Fraction(-1, 112), Fraction(2, 1925), Fraction(-1, 16632)]
    assert np.allclose(w, [float(x) for x in exact], rtol=1e-14)
    # consistency: a constant has zero Laplacian, x^2 has second derivative 2
    assert abs(2 * w[0] + 2 * w[1:].sum()) < 1e-13
    assert abs(sum(p * p * w[p] for p in range(1, 7)) - 1.0) < 1e-13
    wt = orc.grad_weights(6, 1.0)
    assert abs(sum(2 * p * wt[p] for p in range(1, 7)) - 1.0) < 1e-13


def _poly_grid(nn, h):
    return synth.Grid(tuple(nn), h, (-0.5 * (nn[0] - 1) * h, -0.5 * (nn[1] - 1) * h, -0.5 * (nn[2] - 1) * h))


@pytest.mark.parametrize("n", [3, 6])
def test_stencil_exact_on_polynomials(orc, n):
    # x^a y^b z^c with every exponent <= 2n+1 is differentiated exactly on nodes at
    # least n away from the boundary (the taps never reach a ghost there).
    nn = (2 * n + 5, 2 * n + 4, 2 * n + 3)
    h = 0.37
    g = _poly_grid(nn, h)
    z, y, x = np.meshgrid(*[g.origin[a] + h * np.arange(nn[a]) for a in (2, 1, 0)], indexing="ij")
    rng = np.random.default_rng(5)
    for _ in range(12):
        a, b, c = rng.integers(0, 2 * n + 2, size=3)
        f = x ** a * y ** b * z ** c
        lap = orc.laplacian(g, n, f)

        def d2(e, t):
            return e * (e - 1) * t ** (e - 2) if e >= 2 else 0.0 * t

        exact = d2(a, x) * y ** b * z ** c + x ** a * d2(b, y) * z ** c + x ** a * y ** b * d2(c, z)
        sl = (slice(n, nn[2] - n), slice(n, nn[1] - n), slice(n, nn[0] - n))
        scale = max(1.0, np.abs(exact[sl]).max())
        assert np.abs(lap[sl] - exact[sl]).max() <= 1e-10 * scale, (a, b, c)


@pytest.mark.parametrize("n", [1, 3, 6])
def test_stencil_matches_dense_kronecker(orc, n):
    nn = (7, 6, 5) if n < 6 else (13, 14, 13)
    h = 0.5
    g = synth.Grid(nn, h, (0.0, 0.0, 0.0))
    D = fdref.dense_3d_laplacian(nn, n, h)
    f = synth.random_field(g, seed=11)
    got = orc.laplacian(g, n, f).reshape(-1)
    assert np.allclose(got, D @ f.reshape(-1), rtol=1e-12, atol=1e-12)


def test_stencil_symbol(orc):
    # a plane wave maps to its FD symbol; the symbol approaches -|k|^2 at order 2n
    n, h = 6, 0.5
    nn = (40, 36, 32)
    g = synth.Grid(nn, h, (0.0, 0.0, 0.0))
    z, y, x = np.meshgrid(*[h * np.arange(nn[a]) for a in (2, 1, 0)], indexing="ij")
    k = np.array([0.7, -1.1, 0.4])
    f = np.cos(k[0] * x + k[1] * y + k[2] * z)
    lap = orc.laplacian(g, n, f)
    c = [float(v) for v in fdref.second_derivative(n)]
    sym = sum((c[0] + 2 * sum(c[p] * np.cos(p * ka * h) for p in range(1, n + 1))) / h ** 2 for ka in k)
    sl = (slice(n, nn[2] - n), slice(n, nn[1] - n), slice(n, nn[0] - n))
    assert np.abs(lap[sl] - sym * f[sl]).max() < 1e-11
    assert abs(sym + (k ** 2).sum()) < 1e-7


def test_operator_symmetric_definite(orc):
    n, h = 6, 0.5
    g = synth.Grid((15, 14, 16), h, (0.0, 0.0, 0.0))
    a = synth.random_field(g, 1)
    b = synth.random_field(g, 2)
    la, lb = orc.laplacian(g, n, a), orc.laplacian(g, n, b)
    assert abs((a * lb).sum() - (la * b).sum()) < 1e-12 * np.abs(a * lb).sum()
    assert (a * la).sum() < 0 and (b * lb).sum() < 0
