"""Pins of the oracle's radial solves, influence-matrix correction and time step.

What fixes the answer without any implementation to compare against:
  * Section 2 (influence matrix): the boundary-condition vector g is at
    machine-epsilon level after every solve;
  * laminar Hagen-Poiseuille flow is an exact fixed point of the discrete step
    (all its profiles are polynomials of degree <= 4; 9-point stencils are
    exact to degree 8);
  * linear Stokes modes decay at the Bessel-function rates of
    tests/golden/stokes_modes.txt (Crank-Nicolson maps a rate lambda to the
    step factor (1 - lambda dt/2) / (1 + lambda dt/2));
  * (0,0)-only states evolve linearly even with the nonlinear term on;
  * disturbances of laminar flow at Re = 2400 decay and travel downstream with
    phase speeds between 0 and the centre-line speed;
  * the energy budget dE/dt = I - D, shift / rotation equivariance and
    second-order accuracy in time.
"""
import os

import numpy as np
import pytest

from inputs import laminar_state, make_state
from oracle import Params, Oracle
from oracle.spectral import to_pm

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def stokes_table():
    rows = []
    with open(os.path.join(GOLDEN, "stokes_modes.txt")) as f:
        for line in f:
            if line.startswith("#"):
                continue
            fam, m, kap, n, mu, lam = line.split()
            rows.append((fam, int(m), float(kap), int(n), float(mu), float(lam)))
    return rows


def mode_map(o, mi, k, base=None, eps=1.0):
    """3N x 3N matrix of the step restricted to mode (mi, k): column j is the
    response (minus the response of `base`) to a unit change of unknown j."""
    N, K = o.N, o.K
    ki = k + K - 1
    if base is None:
        base = np.zeros((3, o.M, o.nk, N), dtype=np.complex128)
    s0 = o.step(base)
    S = np.zeros((3 * N, 3 * N), dtype=np.complex128)
    for j in range(3 * N):
        u = base.copy()
        u[j // N, mi, ki, j % N] += eps
        S[:, j] = (o.step(u) - s0)[:, mi, ki, :].reshape(-1) / eps
    return S


def cn_rates(S, dt):
    sig = np.linalg.eigvals(S)
    sig = sig[np.abs(sig) > 1e-8]
    lam = (2.0 / dt) * (1.0 - sig) / (1.0 + sig)
    return np.sort(lam.real)


def test_boundary_conditions_at_machine_epsilon():
    p = Params(N=24, M=6, K=5, mp=2, Re=1000.0, dt=0.01)
    o = Oracle(p)
    rng = np.random.default_rng(3)
    R = rng.standard_normal((3, p.M, o.nk, p.N)) + 1j * rng.standard_normal((3, p.M, o.nk, p.N))
    u = o.solve(R)
    v = to_pm(u)
    scale = np.max(np.abs(u))
    assert np.max(np.abs(u[:, :, :, -1])) <= 100 * np.finfo(float).eps * scale
    for mi in range(p.M):
        m = p.mp * mi
        g = o.gvec(m, o.kap, v[:, mi])
        d1max = np.max(np.abs(o.g.D1[0][-1]))
        assert np.max(np.abs(g[:, 3])) <= 100 * np.finfo(float).eps * d1max * scale


@pytest.mark.parametrize("mp,alpha,Re", [(1, 1.25, 2400.0), (2, 0.5, 5300.0)])
def test_laminar_is_fixed_point(mp, alpha, Re):
    p = Params(N=24, M=4, K=4, mp=mp, alpha=alpha, Re=Re, dt=0.005)
    o = Oracle(p)
    u = laminar_state(p.N, p.M, p.K, o.g.r)
    v = o.run(u, 3)
    assert np.max(np.abs(v - u)) <= 1e-13
    d = o.diagnostics(v)
    lam = o.laminar_values()
    assert abs(d["E"] / lam["E"] - 1) < 1e-13
    assert abs(d["I"] / lam["I"] - 1) < 1e-11
    assert abs(d["D"] / lam["D"] - 1) < 1e-13
    assert abs(d["tau_w"] - 2.0) < 1e-12


@pytest.mark.parametrize("family,mi,k,fixed_flux", [
    ("swirl", 0, 0, True), ("axial_flux", 0, 0, True), ("axial_dpdz", 0, 0, False),
    ("meridional", 0, 1, True), ("general", 1, 1, True), ("general", 2, 1, True)])
def test_stokes_modes_decay_at_bessel_rates(family, mi, k, fixed_flux):
    p = Params(N=24, M=3, K=2, Re=100.0, dt=0.01, alpha=1.25, nonlinear=False,
               fixed_flux=fixed_flux)
    o = Oracle(p)
    rates = cn_rates(mode_map(o, mi, k), p.dt) * p.Re
    want = [lam for fam, m, kap, n, mu, lam in stokes_table() if fam == family and m == mi]
    for lam in want[:2]:
        err = np.min(np.abs(rates - lam)) / lam
        assert err < 1e-6, (family, lam, rates[:6])


def test_axisymmetric_swirl_evolves_linearly_with_nonlinear_term():
    """For a (0,0)-only state u x omega is a radial field balanced by pressure,
    so the nonlinear step equals the Stokes step."""
    from scipy.special import jv, jn_zeros
    kw = dict(N=24, M=3, K=3, Re=500.0, dt=0.01)
    a = Oracle(Params(**kw))
    b = Oracle(Params(nonlinear=False, **kw))
    r = a.g.r
    u = laminar_state(24, 3, 3, r)
    u[1, 0, 2] = 0.7 * jv(1, jn_zeros(1, 1)[0] * r)
    u[2, 0, 2] += 0.3 * (jv(0, jn_zeros(2, 1)[0] * r) - jv(0, jn_zeros(2, 1)[0]))
    ua, ub = a.run(u, 5), b.run(u, 5)
    assert np.max(np.abs(ua - ub)) < 1e-13
    assert np.max(np.abs(ua[:, 1:])) == 0.0 and np.max(np.abs(ua[:, :, :2])) == 0.0


def test_disturbances_of_laminar_flow_travel_downstream_and_decay():
    p = Params(N=32, M=3, K=3, Re=2400.0, dt=0.01, alpha=1.25)
    o = Oracle(p)
    base = laminar_state(p.N, p.M, p.K, o.g.r)
    sig = np.linalg.eigvals(mode_map(o, 1, 1, base=base, eps=1e-7))
    sig = sig[np.argsort(-np.abs(sig))][:10]
    growth = np.log(np.abs(sig)) / p.dt
    speed = -np.angle(sig) / (p.alpha * 1 * p.dt)
    assert np.all(growth < 0)
    assert np.all((speed > 0) & (speed < 1)), speed


def _tiny_state(o, energy=1e-2, seed=7):
    p = o.p
    return make_state(p.N, p.M, p.K, p.mp, p.alpha, o.g.r, energy, 4.0, 4.0, seed)


def test_energy_budget():
    """dE/dt = I - D (Section 3.2's E, I, D).  Over one step, with the
    time-centred input of the fixed-flux forcing and the trapezoidal
    dissipation, (E^{n+1} - E^n)/dt - (I^{n+1/2} - (D^n + D^{n+1})/2) -> 0 as
    dt -> 0 (down to the finite-difference floor, which shrinks with N).
    The first step is skipped: it projects the synthetic state onto the
    discrete divergence constraint, a jump in E that does not scale with dt."""
    errs = []
    for dt in (0.02, 0.01, 0.005):
        o = Oracle(Params(N=48, M=6, K=6, Re=1000.0, dt=dt, alpha=1.25))
        u = o.run(_tiny_state(o), 1 + int(round(0.04 / dt)))
        d0 = o.diagnostics(u)
        u = o.step(u)
        d1 = o.diagnostics(u)  # its beta is that of the step just taken
        err = (d1["E"] - d0["E"]) / dt - (d1["I"] - 0.5 * (d0["D"] + d1["D"]))
        errs.append(abs(err) / d1["D"])
    assert errs[0] / errs[1] > 3.5 and errs[1] / errs[2] > 3.5, errs
    assert errs[2] < 1e-5, errs


def test_shift_and_rotation_equivariance():
    p = Params(N=24, M=6, K=5, mp=1, Re=1000.0, dt=0.01, alpha=1.1)
    o = Oracle(p)
    u = _tiny_state(o, 1e-2, 9)
    s, phi = 0.37, 0.61
    ks = np.arange(-(p.K - 1), p.K)
    ms = np.arange(p.M)
    shift = np.exp(1j * p.alpha * ks * s)[None, None, :, None]
    rot = np.exp(1j * p.mp * ms * phi)[None, :, None, None]
    ref = o.step(u)
    assert np.max(np.abs(o.step(u * shift) - ref * shift)) < 1e-13
    assert np.max(np.abs(o.step(u * rot) - ref * rot)) < 1e-13


def test_second_order_in_time():
    T = 0.16
    res = []
    for dt in (0.04, 0.02, 0.01):
        o = Oracle(Params(N=24, M=6, K=6, Re=1000.0, dt=dt, alpha=1.25))
        res.append(o.run(_tiny_state(o, 2e-2, 5), int(round(T / dt))))
    e1 = np.max(np.abs(res[0] - res[1]))
    e2 = np.max(np.abs(res[1] - res[2]))
    assert 3.6 < e1 / e2 < 4.4, (e1, e2)


def test_interior_divergence_small_and_converging():
    errs = []
    for N in (24, 48):
        o = Oracle(Params(N=N, M=4, K=4, Re=1000.0, dt=0.01, alpha=1.25))
        u = o.run(_tiny_state(o, 1e-2, 13), 2)
        v = to_pm(u)
        d = max(np.max(np.abs(o.div_pm(o.p.mp * mi, o.kap, v[0, mi], v[1, mi], v[2, mi])))
                for mi in range(o.M))
        errs.append(d / np.max(np.abs(u[:, :, :, :])))
    assert errs[0] < 1e-3 and errs[1] < errs[0] / 10, errs
