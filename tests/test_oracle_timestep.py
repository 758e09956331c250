"""Pins of the oracle's automatic time-step control: the last correction of
a step vanishes for axisymmetric streamwise-invariant flow (u x omega is
then a radial gradient, which the pressure absorbs) and scales as dt^2
otherwise; the control rule on hand-computed cases; laminar flow settles at
the closed-form Courant step and stays laminar."""
from dataclasses import replace

import numpy as np
import pytest

from inputs import laminar_state, make_state
from oracle import Oracle, Params
from oracle.timestep import DtControl, next_dt, pc_difference, run_adaptive


def params(**kw):
    base = dict(N=16, M=4, K=4, alpha=1.25, Re=2400.0, dt=0.01)
    base.update(kw)
    return Params(**base)


def test_correction_vanishes_for_axisymmetric_state():
    o = Oracle(params())
    r = o.g.r
    u = laminar_state(16, 4, 4, r)
    u[1, 0, 3] = 0.3 * r * (1 - r ** 2)              # swirl, odd in r
    u[2, 0, 3] += 0.2 * (1 - r ** 2) ** 2             # axial profile, even in r
    u1, up = o.step_pc(u)
    assert pc_difference(o, u1, up) <= 1e-14 * o.energy_norm(u)
    # the swirl decays, so the step itself is not trivial
    assert o.energy_norm(u1 - u) > 1e-6
    # and a 3D perturbation gives a correction well above rounding
    v = make_state(16, 4, 4, 1, 1.25, r, 1e-2, 3.0, 3.0, 11, laminar=True)
    v1, vp = o.step_pc(v)
    assert pc_difference(o, v1, vp) > 1e-7


def test_correction_is_second_order_in_dt():
    p = params()
    u = make_state(16, 4, 4, 1, 1.25, Oracle(p).g.r, 1e-2, 3.0, 3.0, 11, laminar=True)
    d = []
    for dt in (0.01, 0.005):
        o = Oracle(replace(p, dt=dt))
        u1, up = o.step_pc(u)
        d.append(pc_difference(o, u1, up))
    assert 3.7 <= d[0] / d[1] <= 4.3


def test_control_rule_cases():
    ctl = DtControl(courant=0.5, pc_tol=0.0, dt_min=1e-5, dt_max=0.02, grow=0.1)
    # Courant limit 0.5 / 80 below dt: shrink with headroom
    assert next_dt(0.01, 0.8, 0.0, ctl) == pytest.approx(0.00625 / 1.1, rel=1e-15)
    # far below the limit: grow, capped at dt_max
    assert next_dt(0.001, 0.01, 0.0, ctl) == 0.02
    # limit 0.0111 above dt but 0.0111/1.1 < 1.1 dt: keep
    assert next_dt(0.01, 0.45, 0.0, ctl) == 0.01
    # reaching dt_max is allowed by less than the factor 1 + h
    assert next_dt(0.019, 0.01, 0.0, ctl) == 0.02
    # corrector limit: delta = 4 tau halves the step
    tight = replace(ctl, pc_tol=1e-6)
    assert next_dt(0.01, 0.1, 4e-6, tight) == pytest.approx(0.005 / 1.1, rel=1e-15)
    with pytest.raises(ValueError):
        next_dt(0.01, 1000.0, 0.0, ctl)


def test_laminar_flow_settles_at_the_courant_step():
    N, M, K, alpha = 16, 4, 4, 1.25
    p = params(dt=0.001)
    ctl = DtControl(courant=0.5, pc_tol=1e-8, dt_max=1.0, grow=0.1, check_every=2)
    u0 = laminar_state(N, M, K, Oracle(p).g.r)
    u, dts, info = run_adaptive(p, u0, 8, ctl)
    # u_z = 1 - r^2 peaks at the innermost node r_0 = cos(pi (N-1) / (2N-1))
    r0 = np.cos(np.pi * (N - 1) / (2 * N - 1))
    dz = 2 * np.pi / (alpha * 3 * K)
    star = 0.5 * dz / ((1 - r0 ** 2) * 1.1)
    assert dts[:2] == [0.001, 0.001]
    assert np.allclose(dts[2:], star, rtol=1e-13, atol=0)
    assert info["changes"] == 1
    assert np.max(np.abs(u - u0)) <= 1e-13
