"""Pins of the oracle's boundary residual, interior divergence and CFL
number against closed forms (laminar flow, rigid rotation, a single mode
with a known wall value and divergence) and against a divergence-free
analytic state."""
import numpy as np

from inputs import laminar_state, make_state
from oracle import Oracle, Params


def oracle(N=16, M=4, K=4, mp=1, alpha=1.25, dt=0.01):
    return Oracle(Params(N=N, M=M, K=K, mp=mp, alpha=alpha, Re=1000.0, dt=dt))


def test_laminar_flow():
    o = oracle()
    r = o.g.r
    u = laminar_state(16, 4, 4, r)
    g, d = o.boundary_and_divergence(u)
    assert g <= 1e-15 and d <= 1e-15
    # u_z = 1 - r^2 peaks at the innermost node; dz = 2 pi / (alpha 3K)
    expect = 0.01 * (1 - r[0] ** 2) * 1.25 * 3 * 4 / (2 * np.pi)
    assert abs(o.cfl(u) - expect) <= 1e-13 * expect


def test_rigid_rotation_and_plug_flow():
    o = oracle(mp=2)
    r = o.g.r
    u = np.zeros((3, 4, 7, 16), dtype=complex)
    u[1, 0, 3] = r  # u_theta = r: |u_theta| / (r dtheta) = 1 / dtheta everywhere
    assert abs(o.cfl(u) - 0.01 * 2 * 12 / (2 * np.pi)) <= 1e-13
    u = np.zeros((3, 4, 7, 16), dtype=complex)
    u[2, 0, 3] = 0.7  # plug flow
    assert abs(o.cfl(u) - 0.01 * 0.7 * 1.25 * 12 / (2 * np.pi)) <= 1e-13


def test_single_mode_wall_value_and_divergence():
    o = oracle()
    r = o.g.r
    K = 4
    c = 0.3 + 0.4j
    u = np.zeros((3, 4, 7, 16), dtype=complex)
    u[2, 1, K - 1 + 2] = c * r  # m = 1, k = 2: u_z = c r (odd in r, as m = 1 requires)
    kap = 1.25 * 2
    g, d = o.boundary_and_divergence(u)
    # g = (0, 0, c, i kappa c) at the wall; div = i kappa c r inside
    assert abs(g - max(1.0, kap) * abs(c)) <= 1e-13
    assert abs(d - kap * abs(c) * r[-2]) <= 1e-13


def test_divergence_free_state():
    o = oracle(N=24, M=6, K=5)
    u = make_state(24, 6, 5, 1, 1.25, o.g.r, 1e-2, 3.0, 3.0, 9, laminar=False)
    g, d = o.boundary_and_divergence(u)
    scale = np.max(np.abs(u))
    assert d <= 1e-5 * scale and g <= 1e-5 * scale
