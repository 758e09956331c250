"""Coriolis force added to the nonlinear term (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section 3.1: the effect of the Earth's rotation is modelled by a function
called at the point of the step where the nonlinear terms have just been
evaluated, which adds the Coriolis force to them; the paper's example has the
rotation axis perpendicular to the pipe axis, at Ekman number
E = nu / (2 Omega D^2).  In units of the pipe radius and the laminar
centre-line speed the force per unit mass is -2 Omega x u, and
2 |Omega| = 1 / (4 E Re) (D = 2, Re = U_cl R / nu).

Omega = (Ox, Oy, Oz) in Cartesian components, z the pipe axis and theta
measured from x; at angle theta its cylindrical components are
O_r = Ox cos + Oy sin, O_t = -Ox sin + Oy cos, O_z = Oz.  The force is formed
pointwise on the dealiased grid (it is linear in u, so that grid holds it
exactly) and truncated to |m| < M, |k| < K like u x omega.  A transverse
axis couples m to m +- 1 and needs mp = 1.
"""
import numpy as np

from .spectral import to_physical, to_spectral


def ekman_rotation(E, Re):
    """|Omega| (units U_cl / R) of Ekman number E = nu / (2 Omega D^2)."""
    return 1.0 / (8.0 * E * Re)


def coriolis(u, mp, rotation):
    """-2 Omega x u in spectral (r, theta, z) form."""
    ox, oy, oz = rotation
    M, nk = u.shape[1], u.shape[2]
    K = (nk + 1) // 2
    if (ox != 0.0 or oy != 0.0) and mp != 1:
        raise ValueError("a transverse rotation axis needs mp = 1")
    ur, ut, uz = (to_physical(u[c], M, K) for c in range(3))
    th = (2.0 * np.pi * np.arange(3 * M) / (3 * M * mp))[None, :, None]
    o_r = ox * np.cos(th) + oy * np.sin(th)
    o_t = -ox * np.sin(th) + oy * np.cos(th)
    fr = -2.0 * (o_t * uz - oz * ut)
    ft = -2.0 * (oz * ur - o_r * uz)
    fz = -2.0 * (o_r * ut - o_t * ur)
    return np.stack([to_spectral(f, M, K) for f in (fr, ft, fz)])
