"""Pins of the oracle's transforms, vorticity and dealiased nonlinear term.

Eq. (1) with the 3/2 rule (Section 2) and pseudospectral nonlinear terms
(Section 2.2).  Pins: the direct double sum of Eq. (1); the brute-force
truncated convolution (what 3/2 dealiasing computes exactly); and Cartesian
polynomial fields whose curl and u x curl u are known in closed form.
"""
import numpy as np
import pytest

from inputs import normals
from oracle import Params, Oracle
from oracle.spectral import to_physical, to_spectral, nonlinear


def random_spectral(M, K, N, seed, ncomp=3):
    g = normals(seed, 2 * ncomp * M * (2 * K - 1) * N).reshape(2, ncomp, M, 2 * K - 1, N)
    a = g[0] + 1j * g[1]
    for k in range(1, K):  # reality at m = 0
        a[:, 0, K - 1 - k] = np.conj(a[:, 0, K - 1 + k])
    a[:, 0, K - 1] = a[:, 0, K - 1].real
    return a


def test_to_physical_is_eq1_direct_sum():
    M, K, N, mp, alpha = 4, 3, 2, 2, 1.25
    A = random_spectral(M, K, N, 11, 1)[0]
    f = to_physical(A, M, K)
    th = 2 * np.pi * np.arange(3 * M) / (3 * M * mp)
    z = 2 * np.pi * np.arange(3 * K) / (3 * K * alpha)
    ref = np.zeros((N, 3 * M, 3 * K), dtype=np.complex128)
    for m in range(-(M - 1), M):
        for k in range(-(K - 1), K):
            c = A[m, k + K - 1] if m >= 0 else np.conj(A[-m, -k + K - 1])
            ref += c[:, None, None] * np.exp(1j * (alpha * k * z[None, None, :]
                                                   + mp * m * th[None, :, None]))
    assert np.max(np.abs(ref.imag)) < 1e-12
    assert np.max(np.abs(f - ref.real)) < 1e-12


def test_round_trip():
    M, K, N = 5, 4, 3
    A = random_spectral(M, K, N, 12, 1)[0]
    B = to_spectral(to_physical(A, M, K), M, K)
    assert np.max(np.abs(A - B)) < 1e-14 * np.max(np.abs(A)) * 10


def brute_force_cross(a, b, M, K):
    """(a x b)_mk = sum over (m1,k1)+(m2,k2) = (m,k) of a_{m1 k1} x b_{m2 k2},
    all |m_i| < M, |k_i| < K, truncated to 0 <= m < M, |k| < K."""
    N = a.shape[-1]

    def coef(x, m, k):
        if abs(m) >= M or abs(k) >= K:
            return np.zeros((3, N), dtype=np.complex128)
        return x[:, m, k + K - 1] if m >= 0 else np.conj(x[:, -m, -k + K - 1])

    out = np.zeros((3, M, 2 * K - 1, N), dtype=np.complex128)
    for m in range(M):
        for k in range(-(K - 1), K):
            acc = np.zeros((3, N), dtype=np.complex128)
            for m1 in range(-(M - 1), M):
                for k1 in range(-(K - 1), K):
                    x = coef(a, m1, k1)
                    y = coef(b, m - m1, k - k1)
                    acc += np.stack([x[1] * y[2] - x[2] * y[1],
                                     x[2] * y[0] - x[0] * y[2],
                                     x[0] * y[1] - x[1] * y[0]])
            out[:, m, k + K - 1] = acc
    return out


def test_dealiased_product_equals_truncated_convolution():
    M, K, N = 4, 4, 12
    p = Params(N=N, M=M, K=K)
    o = Oracle(p)
    u = random_spectral(M, K, N, 21)
    w = random_spectral(M, K, N, 22)
    got = nonlinear(u, o.g, omega=w)
    ref = brute_force_cross(u, w, M, K)
    assert np.max(np.abs(got - ref)) < 1e-13 * np.max(np.abs(ref))


def _cartesian_case(mp):
    """Polynomial-in-(x, y), single-harmonic-in-z velocity with its curl, both
    written out by hand; invariant under rotation by 2 pi / mp."""
    def fields(X, Y, c, s, alpha):
        if mp == 1:
            ux = Y ** 2 + s * X
            uy = X * Y * c - X
            uz = X ** 3 + Y + c * Y ** 2
            wx = 1 + 2 * Y * c + alpha * X * Y * s
            wy = alpha * X * c - 3 * X ** 2
            wz = Y * c - 1 - 2 * Y
        else:
            ux = X ** 3 - X * Y ** 2 * s
            uy = Y + X ** 2 * Y
            uz = X ** 2 - Y ** 2 * c + 1
            wx = -2 * Y * c
            wy = -X * Y ** 2 * alpha * c - 2 * X
            wz = 2 * X * Y - (-2 * X * Y * s)
        return (ux, uy, uz), (wx, wy, wz)
    return fields


@pytest.mark.parametrize("mp", [1, 2])
def test_vorticity_and_product_of_cartesian_polynomials(mp):
    M, K, N, alpha = 8, 4, 12, 1.25
    p = Params(N=N, M=M, K=K, mp=mp, alpha=alpha)
    o = Oracle(p)
    r = o.g.r
    th = 2 * np.pi * np.arange(3 * M) / (3 * M * mp)
    z = 2 * np.pi * np.arange(3 * K) / (3 * K * alpha)
    R, TH, Z = np.meshgrid(r, th, z, indexing="ij")
    X, Y = R * np.cos(TH), R * np.sin(TH)
    (ux, uy, uz), (wx, wy, wz) = _cartesian_case(mp)(X, Y, np.cos(alpha * Z), np.sin(alpha * Z), alpha)

    def cyl(ax, ay):
        return ax * np.cos(TH) + ay * np.sin(TH), -ax * np.sin(TH) + ay * np.cos(TH)

    def spec(f):  # coefficients of the sampled field (input preparation)
        F = np.fft.fft2(f, axes=(1, 2)) / (9 * M * K)
        A = np.zeros((M, 2 * K - 1, N), dtype=np.complex128)
        for m in range(M):
            for ki, k in enumerate(range(-(K - 1), K)):
                A[m, ki] = F[:, m, k % (3 * K)]
        return A

    ur, ut = cyl(ux, uy)
    u = np.stack([spec(ur), spec(ut), spec(uz)])
    w = o.vorticity(u)
    wr, wt = cyl(wx, wy)
    for c, ref in enumerate([wr, wt, wz]):
        assert np.max(np.abs(to_physical(w[c], M, K) - ref)) < 1e-12
    n = o.nonlinear(u)
    nx, ny, nz = uy * wz - uz * wy, uz * wx - ux * wz, ux * wy - uy * wx
    nr, nt = cyl(nx, ny)
    for c, ref in enumerate([nr, nt, nz]):
        assert np.max(np.abs(to_physical(n[c], M, K) - ref)) < 1e-12
