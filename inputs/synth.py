"""Seeded synthetic pipe-flow states.

Everything here is input data.  An initial condition is Hagen-Poiseuille flow
plus a divergence-free, no-slip perturbation u' = curl A, where the vector
potential A has polynomial radial profiles with Gaussian random coefficients.
The curl is taken analytically (exact polynomial derivatives), so the generator
uses no finite differences, transforms or solves.

Spectral layout of a state (the library's external layout):
    complex128 array [3][M][2K-1][N]
    component order (u_r, u_theta, u_z); azimuthal index m = 0..M-1 (the
    wavenumber is mp*m); axial index k = -(K-1)..K-1 stored at position k+K-1;
    radial node n = 0..N-1 (r ascending, r[N-1] = 1).
Negative m are implied by reality: A(-m,-k) = conj(A(m,k)).

Random numbers come from the SplitMix64 generator (Steele, Lea & Flood, 2014):
state_i = seed + (i+1)*0x9E3779B97F4A7C15, output = mix(state_i), with
Box-Muller for normal deviates.  It is counter based, so a draw's value depends
only on (seed, index).
"""
import math

import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def chebyshev_nodes(N):
    """Default radial nodes: the N non-negative Gauss-Lobatto points of the
    Chebyshev polynomial T_{2N-1}, r_n = cos(pi (N-n) / (2N-1)), n = 1..N.
    The wall r = 1 is a node, the axis is not; nodes bunch towards r = 1."""
    n = np.arange(1, N + 1, dtype=np.float64)
    return np.cos(np.pi * (N - n) / (2.0 * N - 1.0))


def splitmix64(seed, count):
    """`count` 64-bit SplitMix64 outputs for `seed` (vectorised, counter based)."""
    with np.errstate(over="ignore"):
        i = np.arange(1, count + 1, dtype=np.uint64)
        z = np.uint64(seed) + i * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniforms(seed, count):
    """Uniform deviates in (0, 1]: top 53 bits of SplitMix64, plus 2^-53."""
    z = splitmix64(seed, count)
    return ((z >> np.uint64(11)).astype(np.float64) + 1.0) * (2.0 ** -53)


def normals(seed, count):
    """Standard normal deviates by Box-Muller on consecutive uniform pairs."""
    npair = (count + 1) // 2
    u = uniforms(seed, 2 * npair)
    u1, u2 = u[0::2], u[1::2]
    rad = np.sqrt(-2.0 * np.log(u1))
    out = np.empty(2 * npair)
    out[0::2] = rad * np.cos(2.0 * np.pi * u2)
    out[1::2] = rad * np.sin(2.0 * np.pi * u2)
    return out[:count]


def _profile(r, p, xi):
    """Radial profile f(r) = r^p (1-r^2)^2 q(r^2), q(s) = sum_j xi_j s^j, with
    f'(r) and f(r)/r, evaluated at r > 0.  xi: [..., 4] complex."""
    r = np.asarray(r, dtype=np.float64)
    s = r * r
    q = np.zeros(np.broadcast_shapes(xi.shape[:-1] + (1,), r.shape), dtype=np.complex128)
    dq = np.zeros_like(q)
    for j in range(xi.shape[-1] - 1, -1, -1):  # Horner in s
        dq = dq * s + q
        q = q * s + xi[..., j:j + 1]
    w = 1.0 - s
    rp1 = r ** (p - 1.0)  # p may be an array of exponents (broadcast)
    f_over_r = rp1 * w * w * q
    f = f_over_r * r
    df = rp1 * w * (p * w * q - 4.0 * s * q + 2.0 * s * w * dq)
    return f, df, f_over_r


def _curl_of_potential(r, M, K, mp, alpha, xi, axis_power=0):
    """u = curl A in (+,-,z) form for A_{+-} = u_r +- i u_theta style components.

    A_+ ~ r^|m+1|, A_- ~ r^|m-1|, A_z ~ r^|m| (m = mp*m_index) times
    r^(2 axis_power) (1-r^2)^2 q(r^2): regular on the axis, A = A' = 0 at the
    wall, so u is regular, divergence-free and vanishes at r = 1.
    axis_power > 0 moves the disturbance away from the axis towards the wall.
    Returns u_plus, u_minus, u_z with shape [M][2K-1][len(r)].
    """
    mi = np.arange(M, dtype=np.float64)[:, None, None]
    ks = np.arange(-(K - 1), K, dtype=np.float64)[None, :, None]
    m = mp * mi
    kap = alpha * ks
    q2 = 2.0 * axis_power
    ap, dap, ap_r = _profile(r, np.abs(m + 1.0) + q2, xi[:, :, 0, :])
    am, dam, am_r = _profile(r, np.abs(m - 1.0) + q2, xi[:, :, 1, :])
    az, daz, az_r = _profile(r, np.abs(m) + q2, xi[:, :, 2, :])
    i = 1j
    u_p = i * m * az_r - i * daz - kap * ap
    u_m = i * m * az_r + i * daz + kap * am
    u_z = -0.5 * i * (dap + (1.0 + m) * ap_r) + 0.5 * i * (dam + (1.0 - m) * am_r)
    return u_p, u_m, u_z


def _hermitian_m0(a):
    """Make the m = 0 column of an r/theta/z spectral array that of a real field."""
    K = (a.shape[-2] + 1) // 2
    for k in range(1, K):
        a[..., 0, K - 1 - k, :] = np.conj(a[..., 0, K - 1 + k, :])
    a[..., 0, K - 1, :] = a[..., 0, K - 1, :].real
    return a


def _energy(u_p, u_m, u_z, mp, alpha, rq, wq):
    """Kinetic energy 1/2 int |u|^2 dV of a (+,-,z) field sampled at the
    Gauss-Legendre points rq (weights wq for int_0^1 f dr)."""
    dens = 0.5 * (np.abs(u_p) ** 2 + np.abs(u_m) ** 2) + np.abs(u_z) ** 2
    per_mode = np.sum(dens * (rq * wq), axis=-1)  # int |u_mk|^2 r dr
    cm = np.full(per_mode.shape[0], 2.0)
    cm[0] = 1.0
    lz = 2.0 * np.pi / alpha
    return 0.5 * (2.0 * np.pi * lz / mp) * float(np.sum(cm[:, None] * per_mode))


def laminar_state(N, M, K, r):
    """Hagen-Poiseuille flow u_z = 1 - r^2 (centre-line speed 1, flux 1/4)."""
    u = np.zeros((3, M, 2 * K - 1, N), dtype=np.complex128)
    u[2, 0, K - 1, :] = 1.0 - np.asarray(r) ** 2
    return u


def make_state(N, M, K, mp, alpha, r, energy_frac, decay_m, decay_k, seed,
               laminar=True, axis_power=0):
    """HPF plus a random divergence-free perturbation of energy
    energy_frac * E_lam, E_lam = pi Lz / (6 mp), whose coefficient amplitudes
    decay as exp(-|m|/decay_m - |k|/decay_k).

    Draw order: for m, for k ascending, for component (+, -, z), for j < 4:
    one complex coefficient (real part, imaginary part) -- 24 normals per mode.
    """
    r = np.asarray(r, dtype=np.float64)
    nk = 2 * K - 1
    g = normals(seed, M * nk * 3 * 4 * 2).reshape(M, nk, 3, 4, 2)
    xi = g[..., 0] + 1j * g[..., 1]
    mabs = np.arange(M, dtype=np.float64)[:, None]
    kabs = np.abs(np.arange(-(K - 1), K, dtype=np.float64))[None, :]
    xi = xi * np.exp(-mabs / decay_m - kabs / decay_k)[:, :, None, None]
    # reality of A at m = 0: A_-(0,-k) = conj A_+(0,k), A_z(0,-k) = conj A_z(0,k)
    for k in range(0, K):
        kp, kn = K - 1 + k, K - 1 - k
        xi[0, kn, 1] = np.conj(xi[0, kp, 0])
        xi[0, kn, 0] = np.conj(xi[0, kp, 1]) if k > 0 else xi[0, kn, 0]
        xi[0, kn, 2] = np.conj(xi[0, kp, 2]) if k > 0 else xi[0, kn, 2].real
    # exact energy from Gauss-Legendre quadrature on [0, 1]
    nq = int(mp * M + 2 * axis_power + 24)
    x, w = np.polynomial.legendre.leggauss(nq)
    rq, wq = 0.5 * (x + 1.0), 0.5 * w
    e_raw = _energy(*_curl_of_potential(rq, M, K, mp, alpha, xi, axis_power), mp, alpha, rq, wq)
    lz = 2.0 * np.pi / alpha
    e_lam = math.pi * lz / (6.0 * mp)
    scale = math.sqrt(energy_frac * e_lam / e_raw) if e_raw > 0 else 0.0
    u_p, u_m, u_z = _curl_of_potential(r, M, K, mp, alpha, xi, axis_power)
    u = np.empty((3, M, nk, N), dtype=np.complex128)
    u[0] = 0.5 * (u_p + u_m)
    u[1] = (u_p - u_m) / 2j
    u[2] = u_z
    u *= scale
    u[:, :, :, -1] = 0.0  # the wall value is zero analytically
    _hermitian_m0(u)
    if laminar:
        u[2, 0, K - 1, :] += 1.0 - r * r
    return u


def ensemble_members(count=96, base_seed=1000):
    """Member parameters of the uneven 96-trajectory ensemble: three resolution
    classes of 32 members, Re ~ U[1800, 2600], alpha ~ U[0.8, 1.6],
    perturbation energy log-uniform in [1e-4, 1e-1], dt = 0.01."""
    classes = [(32, 16, 24), (48, 24, 32), (64, 32, 48)]
    out = []
    for i in range(count):
        N, M, K = classes[min(i * len(classes) // count, len(classes) - 1)]
        u = uniforms(base_seed + i, 3)
        out.append(dict(N=N, M=M, K=K, mp=1, alpha=0.8 + 0.8 * u[0],
                        Re=1800.0 + 800.0 * u[1], dt=0.01,
                        energy_frac=10.0 ** (-4.0 + 3.0 * u[2]),
                        decay_m=4.0, decay_k=4.0, seed=base_seed + i))
    return out


def workload_state(w, r):
    """Initial state of a workload dict (see WORKLOADS) on nodes r."""
    return make_state(w["N"], w["M"], w["K"], w["mp"], w["alpha"], r, w["energy_frac"],
                      w["decay_m"], w["decay_k"], w["seed"], axis_power=w.get("axis_power", 0))


#: Workloads named by what they are.  "tiny" is the small FP64 parity case,
#: "pipe64" the N=64 turbulent-scale throughput case, "nk" the travelling-wave
#: Newton-Krylov case.  The pipe64 disturbance carries an extra r^2 in its
#: vector potential: it sits towards the wall, as turbulent fluctuations do,
#: and its cross-axis flow stays within the explicit advection limit of the
#: predictor-corrector step at the innermost nodes for dt = 0.005.
WORKLOADS = {
    "tiny": dict(N=24, M=8, K=8, mp=1, alpha=1.25, Re=2400.0, dt=0.01,
                 energy_frac=1e-3, decay_m=4.0, decay_k=4.0, seed=1, steps=100),
    "pipe64": dict(N=64, M=48, K=64, mp=1, alpha=0.5, Re=5300.0, dt=0.005,
                   energy_frac=0.1, decay_m=24.0, decay_k=32.0, seed=2, steps=1000,
                   axis_power=1),
    "nk": dict(N=48, M=24, K=32, mp=2, alpha=1.25, Re=2400.0, dt=0.01,
               energy_frac=1e-4, decay_m=4.0, decay_k=4.0, seed=5000, T=20.0),
}
