"""Finite-difference coefficients derived independently of the oracle.

The order-2n central coefficients are obtained here by solving the moment
(Vandermonde) conditions exactly in rational arithmetic, which is a different
route from the closed-form weights printed in Sec. 4 of the paper.  Used only by
tests to pin the oracle.
"""
from fractions import Fraction

import numpy as np


def _solve(A, b):
    n = len(b)
    M = [row[:] + [b[i]] for i, row in enumerate(A)]
    for c in range(n):
        piv = next(r for r in range(c, n) if M[r][c] != 0)
        M[c], M[piv] = M[piv], M[c]
        for r in range(n):
            if r != c and M[r][c] != 0:
                f = M[r][c] / M[c][c]
                M[r] = [x - f * y for x, y in zip(M[r], M[c])]
    return [M[i][n] / M[i][i] for i in range(n)]


def second_derivative(n):
    """c_0..c_n with f''(0) h^2 ~ c_0 f_0 + sum_p c_p (f_p + f_-p), exact to degree 2n+1."""
    A, b = [], []
    for k in range(n + 1):
        # f = x^(2k): sum over offsets -n..n of c_|p| p^(2k)
        row = [Fraction(1 if k == 0 else 0)] + [Fraction(2 * p ** (2 * k)) for p in range(1, n + 1)]
        A.append(row)
        b.append(Fraction(2 if k == 1 else 0))
    return _solve(A, b)


def first_derivative(n):
    """c~_1..c~_n with f'(0) h ~ sum_p c~_p (f_p - f_-p), exact to degree 2n."""
    A, b = [], []
    for k in range(n):
        A.append([Fraction(2 * p ** (2 * k + 1)) for p in range(1, n + 1)])
        b.append(Fraction(1 if k == 0 else 0))
    return _solve(A, b)


def dense_1d_second(npts, n, h):
    """1-D order-2n second-difference matrix with zero ghosts."""
    c = [float(x) for x in second_derivative(n)]
    D = np.zeros((npts, npts))
    for i in range(npts):
        D[i, i] = c[0]
        for p in range(1, n + 1):
            if i + p < npts:
                D[i, i + p] = c[p]
            if i - p >= 0:
                D[i, i - p] = c[p]
    return D / h ** 2


def dense_3d_laplacian(nn, n, h):
    """Kronecker-sum 3-D Laplacian for arrays of shape (n3, n2, n1) flattened in C order."""
    n1, n2, n3 = nn
    D1, D2, D3 = (dense_1d_second(m, n, h) for m in (n1, n2, n3))
    I1, I2, I3 = np.eye(n1), np.eye(n2), np.eye(n3)
    return np.kron(I3, np.kron(I2, D1)) + np.kron(I3, np.kron(D2, I1)) + np.kron(D3, np.kron(I2, I1))
