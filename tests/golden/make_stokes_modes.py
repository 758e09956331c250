"""Write stokes_modes.txt: decay rates of linear Stokes modes in a pipe.

For du/dt = -grad p + Re^-1 lap u, div u = 0, u(1) = 0, a mode
exp(i(m theta + kappa z) - lambda t) has lambda Re = mu^2 + kappa^2 where mu
solves (textbook separation of variables; p ~ I_m(kappa r), homogeneous
velocity ~ J_{m+-1}(mu r), J_m(mu r)):

  m = 0 swirl:               J_1(mu) = 0
  m = 0 meridional, k != 0:  kappa I_0(kappa) J_1(mu) - mu I_1(kappa) J_0(mu) = 0
  general m, kappa != 0:     mu/2 [I_{m-1} J_{m+1} J_m - I_{m+1} J_{m-1} J_m]
                             + kappa I_m J_{m-1} J_{m+1} = 0
                             (I at kappa, J at mu)
  (0,0) axial, fixed flux:   J_2(mu) = 0     (the flux constraint removes J_0)
  (0,0) axial, fixed dp/dz:  J_0(mu) = 0

Uses scipy only.  Run: python tests/golden/make_stokes_modes.py
"""
import os

import numpy as np
from scipy import optimize, special


def roots(f, lo, hi, n, *args):
    xs = np.linspace(lo, hi, 4000)
    v = [f(x, *args) for x in xs]
    out = [optimize.brentq(f, xs[i], xs[i + 1], args=args, xtol=1e-15)
           for i in range(len(xs) - 1) if v[i] * v[i + 1] < 0]
    return out[:n]


def general(mu, m, kap):
    I = lambda n: special.iv(n, kap)  # noqa: E731
    J = lambda n: special.jv(n, mu)   # noqa: E731
    return 0.5 * mu * (I(m - 1) * J(m + 1) * J(m) - I(m + 1) * J(m - 1) * J(m)) \
        + kap * I(m) * J(m - 1) * J(m + 1)


def meridional0(mu, kap):
    return kap * special.iv(0, kap) * special.jv(1, mu) - mu * special.iv(1, kap) * special.jv(0, mu)


def main():
    rows = []
    for n, mu in enumerate(special.jn_zeros(1, 3), 1):
        rows.append(("swirl", 0, 0.0, n, mu))
    for n, mu in enumerate(special.jn_zeros(2, 3), 1):
        rows.append(("axial_flux", 0, 0.0, n, mu))
    for n, mu in enumerate(special.jn_zeros(0, 3), 1):
        rows.append(("axial_dpdz", 0, 0.0, n, mu))
    for n, mu in enumerate(roots(meridional0, 0.5, 12.0, 3, 1.25), 1):
        rows.append(("meridional", 0, 1.25, n, mu))
    for m in (1, 2):
        for n, mu in enumerate(roots(general, 0.5, 12.0, 3, m, 1.25), 1):
            rows.append(("general", m, 1.25, n, mu))
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "stokes_modes.txt")
    with open(path, "w") as f:
        f.write("# Linear Stokes decay rates in a pipe of radius 1: lambda*Re = mu^2 + kappa^2.\n")
        f.write("# Written by make_stokes_modes.py (scipy Bessel functions; see its docstring).\n")
        f.write("# family m kappa n mu lambda_Re\n")
        for fam, m, kap, n, mu in rows:
            f.write(f"{fam} {m} {kap:.4f} {n} {mu:.15f} {mu * mu + kap * kap:.15f}\n")


if __name__ == "__main__":
    main()
