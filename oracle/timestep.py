"""Automatic time-step control of the predictor-corrector scheme (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section 2 says the predictor-corrector scheme runs with automatic time-step
control but gives no rule.  The rule used here (one reading):

  * Courant limit.  With the CFL number of Oracle.cfl, which is dt times
    U = max over the dealiased grid of |u_r|/dr + |u_theta|/(r dtheta) +
    |u_z|/dz, the largest step with CFL number C is dt_c = C / U.
  * Corrector limit.  The last correction, delta = ||u^{n+1} - u^p|| (energy
    norm of Oracle.energy_norm; u^p the iterate before the last corrector),
    is O(dt^2): the predictor treats u x omega by the explicit Euler rule and
    the corrector by the trapezoidal rule, and the two differ by
    c dt (N(u^p) - N(u^n)) = O(dt^2).  A tolerance tau then allows
    dt_e = dt sqrt(tau / delta).
  * Every `check_every` steps, after the step: lim = min(dt_c, dt_e),
    new = min(dt_max, lim / (1 + h)).  The step shrinks to `new` when
    dt > lim, and grows to `new` when new > dt and either
    new >= (1 + h) dt or new == dt_max; otherwise dt is kept.  A `new` below
    dt_min is an error.  The factor 1 + h leaves headroom after a change and
    keeps dt from changing at every check, since every change rebuilds the
    implicit operators H = 1/dt - (c/Re) L.
  * No step is repeated: a new dt applies from the next step on.
"""
from dataclasses import dataclass, replace

import numpy as np

from .solver import Oracle


@dataclass
class DtControl:
    courant: float = 0.5      # C
    pc_tol: float = 0.0       # tau; 0 switches the corrector limit off
    dt_min: float = 1e-6
    dt_max: float = 0.05
    grow: float = 0.1         # h
    check_every: int = 10


def pc_difference(o, u_next, u_pred):
    """delta = ||u^{n+1} - u^p|| in the energy norm."""
    return float(o.energy_norm(u_next - u_pred))


def next_dt(dt, cfl, delta, ctl):
    """The step size after a check, from the CFL number and the last
    correction of the step just taken with size dt."""
    U = cfl / dt
    dt_c = ctl.courant / U if U > 0 else np.inf
    dt_e = dt * np.sqrt(ctl.pc_tol / delta) if ctl.pc_tol > 0 and delta > 0 else np.inf
    lim = min(dt_c, dt_e)
    new = min(ctl.dt_max, lim / (1.0 + ctl.grow))
    if new < ctl.dt_min:
        raise ValueError(f"time step {new} below dt_min {ctl.dt_min}")
    if dt > lim:
        return new
    if new > dt and (new >= (1.0 + ctl.grow) * dt or new == ctl.dt_max):
        return new
    return dt


def run_adaptive(p, u, nsteps, ctl):
    """nsteps steps from u with the control above, starting at p.dt.
    Returns (u, dts, info): dts[j] is the step size of step j, info holds the
    last CFL number, the last correction, the number of changes and the
    simulated time."""
    o = Oracle(p)
    dts, changes, t = [], 0, 0.0
    cfl = delta = 0.0
    for j in range(1, nsteps + 1):
        dts.append(o.p.dt)
        t += o.p.dt
        u, up = o.step_pc(u)
        if j % ctl.check_every == 0:
            cfl = o.cfl(u)
            delta = pc_difference(o, u, up)
            new = next_dt(o.p.dt, cfl, delta, ctl)
            if new != o.p.dt:
                beta = o.beta
                o = Oracle(replace(o.p, dt=new))
                o.beta = beta
                changes += 1
    return u, dts, dict(cfl=cfl, delta=delta, changes=changes, t=t, dt=o.p.dt)
