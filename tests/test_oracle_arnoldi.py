"""Pins of the oracle's Arnoldi iteration: with the nonlinear term off, the
time-T map is affine and its eigenvalues are the Crank-Nicolson images of
the Stokes decay rates of the pipe, whose Bessel-function values are in
tests/golden/stokes_modes.txt (m = 1 at kappa = 1.25, the m = 0 swirl) plus
the swirl at kappa = 1.25, j_{1,1}^2 + kappa^2 in units of 1/Re."""
import os

import numpy as np

from inputs import laminar_state, make_state
from oracle import Oracle, Params
from oracle.arnoldi import arnoldi, order

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "stokes_modes.txt")


def golden_rate(family, m, kappa):
    with open(GOLDEN) as f:
        for line in f:
            if line.startswith("#"):
                continue
            fam, mm, ka, n, mu, lre = line.split()
            if fam == family and int(mm) == m and abs(float(ka) - kappa) < 1e-9 and int(n) == 1:
                return float(lre), float(mu)
    raise KeyError(family)


def test_order_of_ritz_values():
    ev = order(np.array([0.5, 0.6 - 0.8j, 0.6 + 0.8j, -0.9, 0.1]))
    assert list(ev) == [0.6 + 0.8j, 0.6 - 0.8j, -0.9, 0.5, 0.1]


def test_stokes_spectrum_of_the_time_map():
    Re, dt, T, alpha = 50.0, 0.01, 2.0, 1.25
    o = Oracle(Params(N=24, M=3, K=2, alpha=alpha, Re=Re, dt=dt, nonlinear=False))
    x = laminar_state(24, 3, 2, o.g.r)
    v0 = make_state(24, 3, 2, 1, alpha, o.g.r, 1e-2, 3.0, 3.0, 21, laminar=False)
    ev, k, conv = arnoldi(o, x, T, 0.0, v0, 40, 3, tol=1e-8, check_every=5)
    assert conv and k <= 40
    n = int(round(T / dt))

    def mult(lre):  # one Crank-Nicolson step per dt at rate lambda = lre / Re
        lam = lre / Re
        return ((1 - 0.5 * lam * dt) / (1 + 0.5 * lam * dt)) ** n

    gen, _ = golden_rate("general", 1, 1.25)
    swirl, j11 = golden_rate("swirl", 0, 0.0)
    expect = [mult(gen), mult(swirl), mult(j11 ** 2 + alpha ** 2)]
    assert np.allclose(ev.real, expect, rtol=1e-8, atol=0)
    assert np.all(np.abs(ev.imag) <= 1e-10)
