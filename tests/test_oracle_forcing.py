"""Pins of the oracle's Coriolis force: it does no work (the energy inner
product <u, f(u)> vanishes, since u . (Omega x u) = 0 pointwise and the
dealiased grid holds the product exactly), laminar flow under a transverse
axis gives the closed-form m = 1 force, an axial axis acts mode by mode as
2 Oz (u_theta, -u_r, 0), and the Ekman-number conversion."""
import numpy as np
import pytest

from inputs import laminar_state, make_state
from oracle import Oracle, Params
from oracle.forcing import coriolis, ekman_rotation
from oracle.newton import inner


def test_no_work():
    o = Oracle(Params(N=16, M=5, K=4, alpha=1.25))
    u = make_state(16, 5, 4, 1, 1.25, o.g.r, 5e-2, 3.0, 3.0, 13)
    f = coriolis(u, 1, (0.3, -0.7, 0.4))
    nu, nf = np.sqrt(inner(o, u, u)), np.sqrt(inner(o, f, f))
    assert nf > 0.1 * nu
    assert abs(inner(o, u, f)) <= 1e-14 * nu * nf


def test_laminar_flow_under_transverse_rotation():
    o = Oracle(Params(N=16, M=4, K=3, alpha=1.25))
    r = o.g.r
    u = laminar_state(16, 4, 3, r)
    ox, oy = 0.25, -0.6
    f = coriolis(u, 1, (ox, oy, 0.0))
    uz = 1 - r ** 2
    k0 = 2  # k = 0 at index K - 1
    expect = np.zeros_like(f)
    expect[0, 1, k0] = -uz * (1j * ox + oy)   # f_r = 2 u_z (Ox sin - Oy cos): m = 1 part
    expect[1, 1, k0] = uz * (ox - 1j * oy)    # f_t = 2 u_z (Ox cos + Oy sin)
    assert np.max(np.abs(f - expect)) <= 1e-14


def test_axial_rotation_acts_mode_by_mode():
    o = Oracle(Params(N=16, M=4, K=3, mp=2, alpha=1.25))
    u = make_state(16, 4, 3, 2, 1.25, o.g.r, 5e-2, 3.0, 3.0, 17)
    f = coriolis(u, 2, (0.0, 0.0, 0.35))
    assert np.max(np.abs(f[0] - 0.7 * u[1])) <= 1e-14
    assert np.max(np.abs(f[1] + 0.7 * u[0])) <= 1e-14
    assert np.max(np.abs(f[2])) <= 1e-14
    with pytest.raises(ValueError):
        coriolis(u, 2, (0.1, 0.0, 0.0))


def test_ekman_number():
    # E = nu / (2 Omega D^2) with D = 2 R, nu = U_cl R / Re: Omega = 1 / (8 E Re)
    Re, E = 5300.0, 1.0
    om = ekman_rotation(E, Re)
    nu = 1.0 / Re
    assert nu / (2 * om * 4.0) == pytest.approx(E, rel=1e-15)


def test_step_with_rotation_keeps_energy_budget():
    """dE/dt = I - D holds with the force on (it does no work): the
    centred difference of E over two steps against the mean of I - D."""
    p = Params(N=16, M=4, K=3, alpha=1.25, Re=500.0, dt=0.002, rotation=(0.05, 0.02, 0.0))
    o = Oracle(p)
    u0 = make_state(16, 4, 3, 1, 1.25, o.g.r, 1e-2, 3.0, 3.0, 19)
    u1 = o.step(u0)
    d1 = o.diagnostics(u1)
    u2 = o.step(u1)
    d0, d2 = o.diagnostics(u0), o.diagnostics(u2)
    dE = (d2["E"] - d0["E"]) / (2 * p.dt)
    assert abs(dE - (d1["I"] - d1["D"])) <= 2e-3 * abs(d1["D"])
