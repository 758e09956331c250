"""Pins of the oracle's radial grid, finite-difference weights and quadrature.

Section 2: 9-point finite differences give 1st / 2nd derivatives to 8th / 7th
order; nodes are Chebyshev points bunched at the boundary.  The pins are
closed forms: exactness on polynomials of the right axis parity, measured
convergence order, and exact integrals of polynomials.
"""
import numpy as np
import pytest

from inputs import chebyshev_nodes
from oracle.grid import fd_matrices, quadrature_weights, radial_nodes


@pytest.mark.parametrize("N", [12, 24, 64])
def test_nodes_closed_form(N):
    r = radial_nodes(N)
    assert r[-1] == 1.0
    assert np.all(np.diff(r) > 0) and r[0] > 0
    # first node = sin(pi / (2 (2N - 1))): the axis is not a node
    assert abs(r[0] - np.sin(np.pi / (2 * (2 * N - 1)))) < 1e-15
    # bunched towards the wall
    assert r[-1] - r[-2] < 0.25 * (r[1] - r[0])
    assert np.array_equal(r, chebyshev_nodes(N))


@pytest.mark.parametrize("N", [12, 24, 48])
@pytest.mark.parametrize("parity", [+1, -1])
def test_fd_exact_on_parity_polynomials(N, parity):
    """D1, D2 reproduce derivatives of r^j exactly for j <= 8 of the given
    parity (the stencil folds mirror points with that parity)."""
    r = radial_nodes(N)
    D1, D2 = fd_matrices(r, parity)
    scale1 = np.max(np.abs(D1))
    scale2 = np.max(np.abs(D2))
    for j in range(0 if parity == 1 else 1, 9, 2):
        f = r ** j
        d1 = j * r ** (j - 1) if j > 0 else 0 * r
        d2 = j * (j - 1) * r ** (j - 2) if j > 1 else 0 * r
        assert np.max(np.abs(D1 @ f - d1)) <= 1e-13 * scale1
        assert np.max(np.abs(D2 @ f - d2)) <= 1e-13 * scale2


def test_fd_band_and_wall_stencil():
    N = 24
    r = radial_nodes(N)
    D1, D2 = fd_matrices(r, 1)
    for n in range(N):
        nz = np.nonzero(D2[n])[0]
        assert nz.min() >= n - 8 and nz.max() <= n + 4
    # one-sided at the wall: uses the 9 outermost nodes, exact for any degree <= 8
    for j in range(9):
        f = (r - 0.3) ** j
        d1 = j * (r - 0.3) ** (j - 1) if j > 0 else 0 * r
        assert abs((D1 @ f)[-1] - d1[-1]) < 1e-10 * np.max(np.abs(D1))


def test_fd_convergence_order():
    """Error of D1 / D2 on smooth functions falls at >= 7th / 6th order
    (the paper states 8th / 7th for 9 points)."""
    for parity, f, d1, d2 in [
            (-1, lambda r: np.sin(3 * r), lambda r: 3 * np.cos(3 * r), lambda r: -9 * np.sin(3 * r)),
            (+1, lambda r: np.cos(3 * r), lambda r: -3 * np.sin(3 * r), lambda r: -9 * np.cos(3 * r))]:
        e1, e2, Ns = [], [], (12, 16, 24)
        for N in Ns:
            r = radial_nodes(N)
            D1, D2 = fd_matrices(r, parity)
            e1.append(np.max(np.abs(D1 @ f(r) - d1(r))))
            e2.append(np.max(np.abs(D2 @ f(r) - d2(r))))
        # order p with error ~ N^-p; beyond N ~ 32 the wall rows of D2 reach
        # their round-off floor (weights ~ 1/h^2 with h ~ 1/N^2 at the wall)
        s1 = [np.log(e1[i] / e1[i + 1]) / np.log(Ns[i + 1] / Ns[i]) for i in range(2)]
        s2 = [np.log(e2[i] / e2[i + 1]) / np.log(Ns[i + 1] / Ns[i]) for i in range(2)]
        assert min(s1) > 7.0, (parity, s1)
        assert min(s2) > 6.0, (parity, s2)


@pytest.mark.parametrize("N", [12, 24, 64])
def test_quadrature_exact(N):
    r = radial_nodes(N)
    w = quadrature_weights(r)
    for j in range(5):  # even polynomials of degree <= 8
        assert abs(w @ r ** (2 * j) - 1.0 / (2 * j + 2)) < 1e-14
    assert abs(w @ (1 - r ** 2) - 0.25) < 1e-15        # laminar flux
    assert abs(w @ (1 - r ** 2) ** 2 - 1.0 / 6.0) < 1e-15  # laminar energy
    assert abs(np.sum(w) - 0.5) < 1e-15
