"""Transforms, vorticity and the dealiased nonlinear term (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Eq. (1): A(r, theta, z) = sum_{|k|<K} sum_{|m|<M} A_km(r_n) e^{i(alpha k z + mp m theta)}.
Following the 3/2 rule of Section 2 the sums are evaluated on a 3M x 3K grid,
theta_j = 2 pi j / (3M mp), z_l = 2 pi l / (3K alpha), products are formed
there and transformed back, keeping |k| < K, 0 <= m < M (the forward transform
carries the factor 1/(9KM)).  Section 2.2 evaluates nonlinear terms
pseudospectrally; the rotational form u x omega is used (the pressure is then
the Bernoulli head p + |u|^2/2).

Vector fields are stored as [3][M][2K-1][N] complex in (r, theta, z)
components; the radial work uses u+- = u_r +- i u_theta, which decouples the
vector Laplacian (textbook cylindrical vector calculus):
    omega_+ = (i m / r) u_z - i u_z' - kappa u_+
    omega_- = (i m / r) u_z + i u_z' + kappa u_-
    omega_z = -(i/2) [u_+' + (1+m) u_+ / r] + (i/2) [u_-' + (1-m) u_- / r]
with m the azimuthal wavenumber mp*m and kappa = alpha*k.
"""
import numpy as np


def to_physical(A, M, K):
    """Spectral [M][2K-1][N] -> physical [N][3M][3K] real (inverse of Eq. (1))."""
    N = A.shape[-1]
    F = np.zeros((N, 3 * M, 3 * K), dtype=np.complex128)
    for m in range(M):
        for ki, k in enumerate(range(-(K - 1), K)):
            F[:, m, k % (3 * K)] = A[m, ki, :]
            if m > 0:
                F[:, (3 * M - m) % (3 * M), (-k) % (3 * K)] = np.conj(A[m, ki, :])
    return np.fft.ifft2(F, axes=(1, 2)).real * (9.0 * K * M)


def to_spectral(f, M, K):
    """Physical [N][3M][3K] real -> spectral [M][2K-1][N] (truncated)."""
    F = np.fft.fft2(f, axes=(1, 2)) / (9.0 * K * M)
    N = f.shape[0]
    A = np.zeros((M, 2 * K - 1, N), dtype=np.complex128)
    for m in range(M):
        for ki, k in enumerate(range(-(K - 1), K)):
            A[m, ki, :] = F[:, m, k % (3 * K)]
    return A


def to_pm(u):
    """(r, theta, z) -> (+, -, z)."""
    return np.stack([u[0] + 1j * u[1], u[0] - 1j * u[1], u[2]])


def from_pm(v):
    """(+, -, z) -> (r, theta, z)."""
    return np.stack([0.5 * (v[0] + v[1]), (v[0] - v[1]) / 2j, v[2]])


def _d1(D, f):
    return f @ D.T


def vorticity(u, grid):
    """omega = curl u, both in (r, theta, z) spectral form; radial derivatives
    by the finite-difference matrix of each component's axis parity."""
    M, nk, N = u.shape[1:]
    K = (nk + 1) // 2
    v = to_pm(u)
    w = np.zeros_like(v)
    r = grid.r
    for mi in range(M):
        m = grid.mp * mi
        pz = grid.D1[m % 2]          # parity of u_z: (-1)^m
        ppm = grid.D1[(m + 1) % 2]   # parity of u_+-: (-1)^(m+-1)
        kap = grid.alpha * np.arange(-(K - 1), K)[:, None]
        up, um, uz = v[0, mi], v[1, mi], v[2, mi]
        duz = _d1(pz, uz)
        w[0, mi] = 1j * m * uz / r - 1j * duz - kap * up
        w[1, mi] = 1j * m * uz / r + 1j * duz + kap * um
        w[2, mi] = (-0.5j * (_d1(ppm, up) + (1 + m) * up / r)
                    + 0.5j * (_d1(ppm, um) + (1 - m) * um / r))
    return from_pm(w)


def cross_physical(u, w):
    """Pointwise u x omega of physical (r, theta, z) components."""
    return np.stack([u[1] * w[2] - u[2] * w[1],
                     u[2] * w[0] - u[0] * w[2],
                     u[0] * w[1] - u[1] * w[0]])


def nonlinear(u, grid, omega=None):
    """Dealiased u x omega in spectral (r, theta, z) form."""
    M, nk = u.shape[1], u.shape[2]
    K = (nk + 1) // 2
    if omega is None:
        omega = vorticity(u, grid)
    up = np.stack([to_physical(u[c], M, K) for c in range(3)])
    wp = np.stack([to_physical(omega[c], M, K) for c in range(3)])
    n = cross_physical(up, wp)
    return np.stack([to_spectral(n[c], M, K) for c in range(3)])
