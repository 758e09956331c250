"""Pins of the oracle's multiple-shooting residual and Newton iteration:
sections on one trajectory give zero continuity residuals and the last
equals the single-shooting residual; the shift column of the Jacobian
product equals its closed form i alpha k shift(Phi(x_S), -s); the period
column approaches the vector field at the section ends (first order in dt);
free-period, free-shift Newton from a near-laminar guess on two sections
reaches laminar flow."""
from dataclasses import replace

import numpy as np

from inputs import laminar_state, make_state
from oracle import Oracle, Params
from oracle.newton import residual, shift
from oracle.shooting import Shooting, solve_orbit

P = Params(N=12, M=3, K=3, alpha=1.25, Re=400.0, dt=0.04)
T, S_SHIFT, N_SEC = 2.0, 0.1, 25


def sections():
    sh = Shooting(P, 2, N_SEC)
    x = make_state(12, 3, 3, 1, 1.25, Oracle(P).g.r, 1e-3, 3.0, 3.0, 7)
    x2 = sh.oracle(T).run(x, N_SEC)
    return sh, x, x2


def test_residual_on_a_trajectory():
    sh, x, x2 = sections()
    G = sh.unpack(sh.residual(sh.pack([x, x2], T, S_SHIFT)))[0]
    assert np.max(np.abs(G[0])) == 0.0
    single = residual(Oracle(replace(P, dt=T / (2 * N_SEC))), x, T, S_SHIFT)
    assert np.max(np.abs(G[1] - single)) == 0.0


def test_shift_and_period_columns():
    sh, x, x2 = sections()
    X = sh.pack([x, x2], T, S_SHIFT)
    G = sh.residual(X)
    ph = sh.phase_vectors(X)
    o = sh.oracle(T)
    y = [o.run(x, N_SEC), o.run(x2, N_SEC)]
    V = np.zeros_like(X)
    V[-1] = 1.0
    Js = sh.unpack(sh.jvp(X, G, V, ph))[0]
    k = np.arange(-2, 3)
    closed = 1j * 1.25 * k[None, None, :, None] * shift(o, y[1], -S_SHIFT)
    assert np.max(np.abs(Js[0])) <= 1e-9
    assert np.max(np.abs(Js[1] - closed)) <= 1e-5 * np.max(np.abs(closed))
    V = np.zeros_like(X)
    V[-2] = 1.0
    Jt = sh.unpack(sh.jvp(X, G, V, ph))[0]
    dt = o.p.dt
    for i in range(2):  # d/dT Phi_{T/2} = (1/2) d/dt at the section end, vs one step
        f = (o.step(y[i]) - y[i]) / dt / 2
        if i == 1:
            f = shift(o, f, -S_SHIFT)
        assert np.max(np.abs(Jt[i] - f)) <= 0.08 * np.max(np.abs(f))


def test_two_sections_reach_laminar_flow():
    p = Params(N=12, M=2, K=2, alpha=1.25, Re=50.0, dt=0.08)
    sh = Shooting(p, 2, 25)
    x = make_state(12, 2, 2, 1, 1.25, Oracle(p).g.r, 1e-3, 3.0, 3.0, 7)
    x2 = sh.oracle(4.0).run(x, 25)
    out, T1, s1, hist, info = solve_orbit(p, [x, x2], 4.0, 0.1, 25, tol=1e-8, m=20, gmres_tol=1e-3)
    assert hist[-1] <= 1e-8 and not info["stalled"]
    lam = laminar_state(12, 2, 2, Oracle(p).g.r)
    assert all(np.max(np.abs(z - lam)) <= 1e-7 for z in out)
    assert np.isfinite(T1) and np.isfinite(s1)
