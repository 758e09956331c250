"""Band structure of the radial operators' LU factors (Section 2.2: banded
LU per Fourier mode), on the oracle's own dense operators.

The library stores per LU column 8 entries of L below the diagonal and 4 of
U above it, and in the forward substitution uses only the first four L
entries for columns j < N - 9: no row whose stencil reaches more than four
columns left of the diagonal starts before N - 9 (the clamped wall
stencils), and elimination without pivoting fills nothing left of a row's
first nonzero.  These tests factor the oracle's Helmholtz and pressure
operators (wall row as the boundary condition) without pivoting and check
that pattern entry by entry, and that it is tight.
"""
import numpy as np
import pytest

from oracle import Oracle, Params


def lu_nopivot(A):
    """Doolittle elimination without pivoting: unit-lower L, upper U."""
    n = A.shape[0]
    U = A.astype(np.float64).copy()
    L = np.eye(n)
    for j in range(n - 1):
        l = U[j + 1:, j] / U[j, j]
        L[j + 1:, j] = l
        U[j + 1:, j:] -= np.outer(l, U[j, j:])
        U[j + 1:, j] = 0.0
    return L, U


def operators(N, mp=1):
    o = Oracle(Params(N=N, M=6, K=4, mp=mp, alpha=1.3, Re=2500.0, dt=0.004))
    kaps = [0.0, 1.3, 3.9]
    for mu in (0, 1, 2, 3, 6):
        for H in o.helm(mu, kaps):
            yield f"helm mu={mu}", H
    for m in (0, 1, 4):
        for i, A in enumerate(o.ppe(m, kaps)):
            if m == 0 and i == 0:
                continue  # (0,0) has no pressure solve
            yield f"ppe m={m}", A


@pytest.mark.parametrize("N", [12, 13, 21, 32, 48, 64])
def test_lu_fits_the_record_band(N):
    for name, A in operators(N):
        L, U = lu_nopivot(A)
        assert np.allclose(L @ U, A, rtol=0, atol=1e-9 * np.abs(A).max()), name
        i, j = np.nonzero(L - np.eye(N))
        assert np.all(i - j <= 8), name  # at most 8 entries of L per column
        i, j = np.nonzero(U)
        assert np.all(j - i <= 4), name  # at most 4 entries of U per column


@pytest.mark.parametrize("N", [12, 13, 21, 32, 48, 64])
def test_deep_l_entries_only_in_the_last_columns(N):
    narrow = N - 9
    for name, A in operators(N):
        L, _ = lu_nopivot(A)
        deep = np.tril(L, -5)  # entries more than four rows below the diagonal
        assert np.all(deep[:, :narrow] == 0.0), name  # exact zeros, not rounding
    # the bound is tight: the wall rows reach back to column N - 9
    _, A = next(operators(N))
    L, _ = lu_nopivot(A)
    assert np.any(np.tril(L, -5)[:, narrow] != 0.0)
