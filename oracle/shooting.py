"""Relative periodic orbits by multiple shooting (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section 2: the Newton solver for invariant solutions has a multiple-shooting
option, in which an orbit is split into sections.  The reading used here:

  * Unknowns X = (x_1 .. x_S, T, s): S states, the period T and the axial
    shift s of a relative periodic orbit (a travelling wave when only s
    matters).  Each section runs T/S with dt = T / (S n) for a fixed number n
    of steps per section, so the discrete map depends smoothly on T.
  * Residual: G_i = Phi_{T/S}(x_i) - x_{i+1} for i < S and
    G_S = shift(Phi_{T/S}(x_S), -s) - x_1 (S = 1 gives the travelling-wave
    residual of newton.py with dt = T / n).
  * Free T and s add the phase conditions <xdot_1, dx_1> = 0 and
    <d_z x_1, dx_1> = 0 on the update (xdot_1 = (Phi_dt(x_1) - x_1) / dt,
    d_z the spectral axial derivative i alpha k); their residuals are 0.
  * The Jacobian product is the forward difference of the whole residual in
    all unknowns, eps = 1e-7 max(||X||, 1) / ||dX||, plus the phase rows.
  * Inner product: the energy inner product summed over the sections, plus
    the products of the T and s entries; the Newton iteration is the
    hookstep of hookstep.py on these extended vectors.
"""
from dataclasses import replace

import numpy as np

from .hookstep import newton_hook
from .newton import inner, shift
from .solver import Oracle


class Shooting:
    """Extended vectors are flat complex arrays: S fields, then T and s."""

    def __init__(self, p, S, n, free_T=True, free_s=True):
        self.p, self.S, self.n = p, S, n
        self.free_T, self.free_s = free_T, free_s
        self.shape = (3, p.M, 2 * p.K - 1, p.N)
        self.size = int(np.prod(self.shape))
        self._o = {}
        self._inner = Oracle(p)  # quadrature weights only

    def oracle(self, T):
        dt = T / (self.S * self.n)
        if dt not in self._o:
            self._o = {dt: Oracle(replace(self.p, dt=dt))}
        return self._o[dt]

    def pack(self, xs, T, s):
        return np.concatenate([np.ravel(x) for x in xs] + [np.array([T, s], dtype=complex)])

    def unpack(self, X):
        xs = [X[i * self.size:(i + 1) * self.size].reshape(self.shape) for i in range(self.S)]
        return xs, X[-2].real, X[-1].real

    def dot(self, A, B):
        o = self._inner
        a, Ta, sa = self.unpack(A)
        b, Tb, sb = self.unpack(B)
        return sum(inner(o, x, y) for x, y in zip(a, b)) + Ta * Tb + sa * sb

    def residual(self, X):
        xs, T, s = self.unpack(X)
        o = self.oracle(T)
        ends = [o.run(x, self.n) for x in xs]
        G = [ends[i] - xs[i + 1] for i in range(self.S - 1)]
        G.append(shift(o, ends[-1], -s) - xs[0])
        return self.pack(G, 0.0, 0.0)

    def phase_vectors(self, X):
        """xdot_1 and d_z x_1 (zero when that unknown is fixed)."""
        xs, T, s = self.unpack(X)
        o = self.oracle(T)
        x1 = xs[0]
        xdot = (o.step(x1) - x1) / o.p.dt if self.free_T else np.zeros_like(x1)
        k = np.arange(-(self.p.K - 1), self.p.K)
        dz = 1j * self.p.alpha * k[None, None, :, None] * x1 if self.free_s else np.zeros_like(x1)
        return xdot, dz

    def jvp(self, X, G0, V, phases, eps_rel=1e-7):
        V = V.copy()
        if not self.free_T:
            V[-2] = 0.0
        if not self.free_s:
            V[-1] = 0.0
        nv = np.sqrt(max(self.dot(V, V), 0.0))
        if nv == 0.0:
            return np.zeros_like(X)
        eps = eps_rel * max(np.sqrt(self.dot(X, X)), 1.0) / nv
        out = (self.residual(X + eps * V) - G0) / eps
        o = self._inner
        v1 = self.unpack(V)[0][0]
        out[-2] = inner(o, phases[0], v1) if self.free_T else 0.0
        out[-1] = inner(o, phases[1], v1) if self.free_s else 0.0
        return out


def solve_orbit(p, xs, T, s, n, free_T=True, free_s=True, **kw):
    """Hookstep Newton on the multiple-shooting system; returns
    (sections, T, s, history of ||G|| / ||X||, info)."""
    sh = Shooting(p, len(xs), n, free_T, free_s)
    cache = {}

    def jv(X, G0, V):
        if cache.get("X") is not X:  # phase vectors once per Newton step
            cache["X"], cache["ph"] = X, sh.phase_vectors(X)
        return sh.jvp(X, G0, V, cache["ph"])

    X, hist, info = newton_hook(sh.residual, jv, sh.dot, sh.pack(xs, T, s), **kw)
    out, T1, s1 = sh.unpack(X)
    return out, T1, s1, hist, info
