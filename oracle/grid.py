"""Radial grid, finite-difference matrices and radial quadrature (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section 2 of the paper: radial points r_n, n = 1..N, may be placed anywhere in
[0, 1]; by default they are Chebyshev points bunched towards the boundary, and
radial derivatives are finite differences on a stencil of (by default) 9 points,
so that derivative matrices are banded; 1st / 2nd derivatives are then of
8th / 7th order.

Readings taken where the paper is silent:
  * nodes: the N non-negative Gauss-Lobatto points of T_{2N-1}; the wall is a
    node, the axis is not;
  * stencils: 9 consecutive points of the symmetric set {.., -r_2, -r_1, r_1,
    r_2, ..} centred on the row's node, shifted inwards at the wall; a value
    at a mirror point -r_j is s * f(r_j) with the parity s = (-1)^mu of the
    component's azimuthal wavenumber mu, so mirror weights fold onto r_j;
  * quadrature for int_0^1 g(r) r dr (g even in r): on each interval
    [r_{j-1}, r_j] (r_0 = 0) integrate the Lagrange interpolant of g through
    node j's stencil exactly.
The weights are written from their definition: derivatives of the Lagrange
basis polynomials of the stencil.
"""
import numpy as np


def radial_nodes(N):
    """r_n = cos(pi (N - n) / (2N - 1)), n = 1..N (ascending, r_N = 1)."""
    n = np.arange(1, N + 1, dtype=np.float64)
    return np.cos(np.pi * (N - n) / (2.0 * N - 1.0))


def lagrange_derivative_weights(x0, x):
    """Weights (w1, w2) with f'(x0) ~ sum_j w1_j f(x_j), f''(x0) ~ sum_j w2_j f(x_j):
    the first and second derivatives at x0 of the Lagrange basis polynomials
    L_j(x) = prod_{i != j} (x - x_i) / (x_j - x_i)."""
    x = np.asarray(x, dtype=np.float64)
    n = len(x)
    d = x0 - x
    w1 = np.zeros(n)
    w2 = np.zeros(n)
    for j in range(n):
        others = [i for i in range(n) if i != j]
        den = np.prod([x[j] - x[i] for i in others])
        s1 = 0.0
        s2 = 0.0
        for a in others:
            s1 += np.prod([d[i] for i in others if i != a])
            for b in others:
                if b != a:
                    s2 += np.prod([d[i] for i in others if i != a and i != b])
        w1[j] = s1 / den
        w2[j] = s2 / den
    return w1, w2


def stencil_window(n, N, width=9):
    """Extended indices of row n's stencil (0-based).  Index e >= 0 is node
    r[e]; e < 0 is the mirror point -r[-e-1]."""
    start = min(n - width // 2, N - width)
    return list(range(start, start + width))


def _ext_point(r, e):
    return r[e] if e >= 0 else -r[-e - 1]


def fd_matrices(r, parity, width=9):
    """Dense N x N first and second derivative matrices for a radial function
    of axis parity `parity` (+1 even, -1 odd)."""
    r = np.asarray(r, dtype=np.float64)
    N = len(r)
    D1 = np.zeros((N, N))
    D2 = np.zeros((N, N))
    for n in range(N):
        idx = stencil_window(n, N, width)
        x = [_ext_point(r, e) for e in idx]
        w1, w2 = lagrange_derivative_weights(r[n], x)
        for e, a, b in zip(idx, w1, w2):
            col = e if e >= 0 else -e - 1
            sgn = 1.0 if e >= 0 else float(parity)
            D1[n, col] += sgn * a
            D2[n, col] += sgn * b
    return D1, D2


def quadrature_weights(r, width=9):
    """w_n with int_0^1 g(r) r dr ~ sum_n w_n g(r_n) for g even in r."""
    r = np.asarray(r, dtype=np.float64)
    N = len(r)
    xg, wg = np.polynomial.legendre.leggauss(8)
    w = np.zeros(N)
    for j in range(N):
        a = 0.0 if j == 0 else r[j - 1]
        b = r[j]
        rq = 0.5 * (b - a) * xg + 0.5 * (b + a)
        wq = 0.5 * (b - a) * wg
        idx = stencil_window(j, N, width)
        x = np.array([_ext_point(r, e) for e in idx])
        for t, e in enumerate(idx):
            others = [i for i in range(width) if i != t]
            basis = np.prod([(rq - x[i]) / (x[t] - x[i]) for i in others], axis=0)
            col = e if e >= 0 else -e - 1
            w[col] += np.sum(wq * basis * rq)
    return w
