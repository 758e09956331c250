"""Pins of the oracle's prescribed wall velocity (boundary values driven
through the influence-matrix vector g): laminar flow plus solid-body
rotation is a steady state of a rotating pipe (u x omega is a radial
gradient); spin-up from rest follows the Bessel series
u_theta = V r - sum_n 2 V J1(j_n r) / (j_n J2(j_n)) exp(-j_n^2 t / Re),
j_n the zeros of J1; and a general wall velocity is met exactly by every
mode after a step."""
import numpy as np
from scipy.special import j1, jn_zeros

from inputs import laminar_state, make_state
from oracle import Oracle, Params


def wall_rotation(M, K, V):
    b = np.zeros((3, M, 2 * K - 1), dtype=complex)
    b[1, 0, K - 1] = V
    return b


def test_rotating_pipe_laminar_state_is_steady():
    N, M, K, V = 16, 3, 3, 0.4
    o = Oracle(Params(N=N, M=M, K=K, alpha=1.25, Re=500.0, dt=0.01, wall=wall_rotation(M, K, V)))
    r = o.g.r
    u = laminar_state(N, M, K, r)
    u[1, 0, K - 1] = V * r
    u1 = o.run(u, 3)
    assert np.max(np.abs(u1 - u)) <= 1e-13
    # without the moving wall the same state is not steady
    o0 = Oracle(Params(N=N, M=M, K=K, alpha=1.25, Re=500.0, dt=0.01))
    assert np.max(np.abs(o0.run(u, 3) - u)) > 1e-4


def test_spin_up_follows_the_bessel_modes():
    """From u_theta = V r - A1 J1(j_1 r) - A2 J1(j_2 r) (smooth, meeting the
    moving wall) each Bessel mode decays at its own rate j^2 / Re."""
    N, M, K, V, Re, dt, n = 32, 2, 2, 0.5, 100.0, 0.01, 300
    o = Oracle(Params(N=N, M=M, K=K, alpha=1.25, Re=Re, dt=dt, wall=wall_rotation(M, K, V)))
    r = o.g.r
    ja, jb = jn_zeros(1, 2)
    A1, A2 = 0.2, -0.07
    u0 = laminar_state(N, M, K, r)
    u0[1, 0, K - 1] = V * r - A1 * j1(ja * r) - A2 * j1(jb * r)
    u = o.run(u0, n)
    t = n * dt
    expect = V * r - A1 * j1(ja * r) * np.exp(-ja ** 2 * t / Re) - A2 * j1(jb * r) * np.exp(-jb ** 2 * t / Re)
    assert np.max(np.abs(u[1, 0, K - 1].real - expect)) <= 1e-6 * abs(A1)
    assert np.max(np.abs(u[1, 0, K - 1].imag)) == 0.0


def test_general_wall_velocity_is_met():
    N, M, K = 16, 4, 3
    rng = np.random.default_rng(8)
    b = 1e-2 * (rng.standard_normal((3, M, 2 * K - 1)) + 1j * rng.standard_normal((3, M, 2 * K - 1)))
    b[:, 0, :K - 1] = np.conj(b[:, 0, K:][:, ::-1])  # m = 0 of a real field
    b[:, 0, K - 1] = b[:, 0, K - 1].real
    b[0, 0, K - 1] = 0.0                              # no net radial flux through the wall
    o = Oracle(Params(N=N, M=M, K=K, alpha=1.25, Re=500.0, dt=0.01, wall=b))
    u = make_state(N, M, K, 1, 1.25, o.g.r, 1e-2, 3.0, 3.0, 5)
    u1 = o.step(u)
    assert np.max(np.abs(u1[:, :, :, -1] - b)) <= 1e-13
    g, d = o.boundary_and_divergence(u1)
    assert g <= 1e-13
