"""Radial solves, influence-matrix correction and predictor-corrector step (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Equations, in units of the pipe radius R and the laminar centre-line speed U_cl
(Re = U_cl R / nu, which equals the paper's bulk-velocity / diameter Re):

  du/dt = u x omega - grad P + Re^-1 lap u + (4/Re)(1 + beta) z^,  div u = 0,
  u(r=1) = 0,  with beta set so that the flux int_0^1 u_z,00 r dr = 1/4.

Per Fourier mode (m, k), m = mp*m_index, kappa = alpha*k, the radial operator
L_{mu,kappa} f = f'' + f'/r - (mu^2/r^2 + kappa^2) f acts on u_+ (mu = m+1),
u_- (mu = m-1), u_z and P (mu = m); its radial derivatives are the
finite-difference matrices of the parity (-1)^mu.

Time scheme (Section 2, second-order predictor-corrector; implicitness c = 1/2,
one corrector):
  R0 = [1/dt + (1-c) L / Re] u^n + N(u^n) + f,   u^p = S(R0)
  R1 = [1/dt + (1-c) L / Re] u^n + c N(u^p) + (1-c) N(u^n) + f,  u^{n+1} = S(R1)
where S is the substep solve (Section 2: pressure-Poisson equation with an
influence-matrix enforcement of the boundary conditions, the viscous terms
implicit with H_mu = 1/dt - (c/Re) L_mu):
  1. L_m P_b = div R, P_b(1) = 0
  2. H_{m+-1} u+-_b = R+- - (grad P_b)+-,  H_m u_z,b = R_z - i kappa P_b,  u_b(1) = 0
  3. homogeneous solutions: h1 (L P1 = 0, P1(1) = 1, H u = -grad P1, u(1) = 0),
     h2, h3, h4 (H u = 0 with unit wall value of u_+, u_-, u_z respectively)
  4. g(v) = (v_+(1), v_-(1), v_z(1), div v(1)); A = [g(h1) .. g(h4)];
     solve A a = -g(u_b);  u = u_b + sum_j a_j h_j  (so g(u) = 0).
Mode (0,0): u_r = 0; H_1 u_theta = R_theta; H_0 u_z = R_z + gamma with u_z(1) = 0
and gamma fixed by the flux (beta = gamma Re / 4).  m = 0 is made Hermitian:
the k < 0 solution is the conjugate of the k > 0 one, (0,0) is real.
"""
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

from .grid import radial_nodes, fd_matrices, quadrature_weights
from .spectral import to_pm, from_pm, vorticity, nonlinear, to_physical
from .forcing import coriolis


@dataclass
class Params:
    N: int
    M: int
    K: int
    mp: int = 1
    alpha: float = 1.25
    Re: float = 2400.0
    dt: float = 0.01
    c: float = 0.5
    n_corr: int = 1
    fixed_flux: bool = True
    nonlinear: bool = True
    stencil: int = 9
    rotation: tuple = (0.0, 0.0, 0.0)   # Omega of the Coriolis force -2 Omega x u (forcing.py)
    # wall velocity per mode, [3][M][2K-1] complex (r, theta, z) components at
    # r = 1, or None for no slip; (0,0) takes theta and z only, m = 0 uses k >= 0
    wall: Optional[np.ndarray] = field(default=None, repr=False)
    r: Optional[np.ndarray] = field(default=None, repr=False)


class Grid:
    def __init__(self, p: Params):
        self.r = radial_nodes(p.N) if p.r is None else np.asarray(p.r, dtype=np.float64)
        self.N = len(self.r)
        even = fd_matrices(self.r, +1, p.stencil)
        odd = fd_matrices(self.r, -1, p.stencil)
        self.D1 = (even[0], odd[0])   # index = parity bit: 0 even, 1 odd
        self.D2 = (even[1], odd[1])
        self.w = quadrature_weights(self.r, p.stencil)
        self.mp = p.mp
        self.alpha = p.alpha


def _bsolve(A, b):
    """Batched dense solve A x = b; A [..., N, N], b [..., N] (complex ok)."""
    return np.linalg.solve(A, b[..., None])[..., 0]


class Oracle:
    """Plain CPU FP64 implementation of the pipe-flow time step."""

    def __init__(self, p: Params):
        self.p = p
        self.g = Grid(p)
        self.N, self.M, self.K = self.g.N, p.M, p.K
        self.nk = 2 * p.K - 1
        self.kap = p.alpha * np.arange(-(p.K - 1), p.K, dtype=np.float64)
        self.beta = 0.0
        self._hom = {}

    # ---- operators ------------------------------------------------------
    def lap(self, mu, kap):
        """L_{mu,kappa} as dense matrices, shape [len(kap), N, N]."""
        g = self.g
        q = abs(mu) % 2
        base = g.D2[q] + g.D1[q] / g.r[:, None] - np.diag(mu * mu / g.r ** 2)
        return base[None, :, :] - (np.asarray(kap) ** 2)[:, None, None] * np.eye(self.N)[None]

    def helm(self, mu, kap):
        """H_{mu,kappa} = 1/dt - (c/Re) L_{mu,kappa}, last row replaced by the wall value."""
        p = self.p
        H = np.eye(self.N)[None] / p.dt - (p.c / p.Re) * self.lap(mu, kap)
        H[:, -1, :] = 0.0
        H[:, -1, -1] = 1.0
        return H

    def ppe(self, m, kap):
        """L_{m,kappa} with the bulk condition P(1) = 0 in the last row."""
        A = self.lap(m, kap)
        A[:, -1, :] = 0.0
        A[:, -1, -1] = 1.0
        return A

    def d1(self, mu, f):
        return f @ self.g.D1[abs(mu) % 2].T

    def div_pm(self, m, kap, vp, vm, vz):
        """div v for v in (+,-,z) form (rows of radial values)."""
        r = self.g.r
        return (0.5 * (self.d1(m + 1, vp) + (1 + m) * vp / r)
                + 0.5 * (self.d1(m - 1, vm) + (1 - m) * vm / r)
                + 1j * kap[:, None] * vz)

    def grad_pm(self, m, kap, P):
        r = self.g.r
        dP = self.d1(m, P)
        return dP - m * P / r, dP + m * P / r, 1j * kap[:, None] * P

    # ---- homogeneous solutions and influence matrix --------------------
    def homogeneous(self, mi):
        """h1..h4 for all k at m index mi: arrays [4][3][nk][N] (+,-,z), P1
        [nk][N], and the influence matrices A [nk][4][4]."""
        if mi in self._hom:
            return self._hom[mi]
        m = self.p.mp * mi
        kap = self.kap
        nk, N = self.nk, self.N
        e = np.zeros((nk, N))
        e[:, -1] = 1.0
        P1 = _bsolve(self.ppe(m, kap), e.astype(np.complex128))
        gp, gm, gz = self.grad_pm(m, kap, P1)
        h = np.zeros((4, 3, nk, N), dtype=np.complex128)
        for c, (mu, rhs) in enumerate([(m + 1, -gp), (m - 1, -gm), (m, -gz)]):
            rhs = rhs.copy()
            rhs[:, -1] = 0.0
            h[0, c] = _bsolve(self.helm(mu, kap), rhs)
        for j, mu in enumerate([m + 1, m - 1, m]):
            h[1 + j, j] = _bsolve(self.helm(mu, kap), e.astype(np.complex128))
        A = np.zeros((nk, 4, 4), dtype=np.complex128)
        for j in range(4):
            A[:, :, j] = self.gvec(m, kap, h[j])
        self._hom[mi] = (h, P1, A)
        return self._hom[mi]

    def gvec(self, m, kap, v):
        """Boundary-condition vector g(v) = (v_+(1), v_-(1), v_z(1), div v(1))."""
        dv = self.div_pm(m, kap, v[0], v[1], v[2])
        return np.stack([v[0][:, -1], v[1][:, -1], v[2][:, -1], dv[:, -1]], axis=-1)

    # ---- right-hand side and substep solve ----------------------------
    def explicit(self, u):
        """[1/dt + (1-c) L / Re] u^n + f, in (+,-,z) form."""
        p = self.p
        v = to_pm(u)
        out = np.empty_like(v)
        for mi in range(self.M):
            m = p.mp * mi
            for c, mu in enumerate([m + 1, m - 1, m]):
                Lv = np.einsum("kij,kj->ki", self.lap(mu, self.kap), v[c, mi])
                out[c, mi] = v[c, mi] / p.dt + (1.0 - p.c) / p.Re * Lv
        out[2, 0, self.K - 1] += 4.0 / p.Re
        return out

    def solve(self, R, want_pressure=False):
        """Substep solve S(R): R in (+,-,z) form -> u in (r,theta,z) form."""
        p, g = self.p, self.g
        M, nk, N, K = self.M, self.nk, self.N, self.K
        v = np.zeros((3, M, nk, N), dtype=np.complex128)
        Pout = np.zeros((M, nk, N), dtype=np.complex128)
        for mi in range(M):
            m = p.mp * mi
            ks = np.arange(nk) if mi > 0 else np.arange(K - 1, nk)  # m=0: k >= 0
            if mi == 0:
                ks = ks[1:]  # (0,0) handled below
            kap = self.kap[ks]
            Rp, Rm, Rz = R[0, mi, ks], R[1, mi, ks], R[2, mi, ks]
            rhs = self.div_pm(m, kap, Rp, Rm, Rz)
            rhs[:, -1] = 0.0
            P = _bsolve(self.ppe(m, kap), rhs)
            gp, gm, gz = self.grad_pm(m, kap, P)
            ub = []
            for mu, b in [(m + 1, Rp - gp), (m - 1, Rm - gm), (m, Rz - gz)]:
                b = b.copy()
                b[:, -1] = 0.0
                ub.append(_bsolve(self.helm(mu, kap), b))
            ub = np.stack(ub)
            h, P1, A = self.homogeneous(mi)
            gv = self.gvec(m, kap, ub)
            if p.wall is not None:  # drive g to the wall values instead of 0
                br, bt, bz = p.wall[0, mi, ks], p.wall[1, mi, ks], p.wall[2, mi, ks]
                gv = gv - np.stack([br + 1j * bt, br - 1j * bt, bz, np.zeros_like(bz)], axis=-1)
            a = _bsolve(A[ks], -gv)
            for j in range(4):
                ub += a[None, :, j, None] * h[j][:, ks]
            P = P + a[:, 0, None] * P1[ks]
            v[:, mi, ks] = ub
            Pout[mi, ks] = P
        u = from_pm(v)
        # mode (0,0): u_r = 0, swirl and axial flow, fixed flux
        k0 = K - 1
        Rth = ((R[0, 0, k0] - R[1, 0, k0]) / 2j).real
        b = Rth.copy()
        b[-1] = p.wall[1, 0, k0].real if p.wall is not None else 0.0
        u[:, 0, k0] = 0.0
        u[1, 0, k0] = np.linalg.solve(self.helm(1, [0.0])[0], b)
        b = R[2, 0, k0].real.copy()
        b[-1] = p.wall[2, 0, k0].real if p.wall is not None else 0.0
        H0 = self.helm(0, [0.0])[0]
        ua = np.linalg.solve(H0, b)
        if p.fixed_flux:
            one = np.ones(N)
            one[-1] = 0.0
            uG = np.linalg.solve(H0, one)
            gamma = (0.25 - g.w @ ua) / (g.w @ uG)
            ua = ua + gamma * uG
            self.beta = gamma * p.Re / 4.0
        u[2, 0, k0] = ua
        # Hermitian m = 0
        for k in range(1, K):
            u[:, 0, k0 - k] = np.conj(u[:, 0, k0 + k])
            Pout[0, k0 - k] = np.conj(Pout[0, k0 + k])
        if want_pressure:
            return u, Pout
        return u

    # ---- nonlinear term and the step ----------------------------------
    def vorticity(self, u):
        return vorticity(u, self.g)

    def nonlinear(self, u):
        """u x omega, plus the Coriolis force when a rotation is set."""
        if not self.p.nonlinear:
            return np.zeros_like(u)
        n = nonlinear(u, self.g)
        if any(o != 0.0 for o in self.p.rotation):
            n = n + coriolis(u, self.p.mp, self.p.rotation)
        return n

    def step(self, u):
        """One predictor-corrector step u^n -> u^{n+1} (r,theta,z spectral)."""
        return self.step_pc(u)[0]

    def step_pc(self, u):
        """One step, returning (u^{n+1}, the iterate before the last
        corrector): with one corrector the second value is the predicted
        state u^p."""
        p = self.p
        N0 = to_pm(self.nonlinear(u))
        Rlin = self.explicit(u)
        u1 = self.solve(Rlin + N0)
        prev = u1
        for _ in range(p.n_corr):
            prev = u1
            N1 = to_pm(self.nonlinear(u1))
            u1 = self.solve(Rlin + p.c * N1 + (1.0 - p.c) * N0)
        return u1, prev

    def run(self, u, nsteps):
        for _ in range(nsteps):
            u = self.step(u)
        return u

    # ---- diagnostics (Section 3.2: E, I, D normalised by laminar) ------
    def laminar_values(self):
        p = self.p
        lz = 2.0 * np.pi / p.alpha
        return dict(E=np.pi * lz / (6.0 * p.mp),
                    I=2.0 * np.pi * lz / (p.mp * p.Re),
                    D=2.0 * np.pi * lz / (p.mp * p.Re))

    def mode_integrals(self, f):
        """sum over m >= 0 (weight 2 for m > 0), k of int |f_mk|^2 r dr."""
        cm = np.full(self.M, 2.0)
        cm[0] = 1.0
        per = np.sum(np.abs(f) ** 2 * self.g.w, axis=-1)  # [..., M, nk]
        return float(np.sum(cm[:, None] * per.reshape(-1, self.M, self.nk).sum(0)))

    def diagnostics(self, u):
        p, g = self.p, self.g
        vol = 2.0 * np.pi * (2.0 * np.pi / p.alpha) / p.mp
        k0 = self.K - 1
        E = 0.5 * vol * self.mode_integrals(u)
        w = self.vorticity(u)
        D = vol * self.mode_integrals(w) / p.Re
        flux = float(g.w @ u[2, 0, k0].real)
        I = (4.0 / p.Re) * (1.0 + self.beta) * vol * flux
        tau = -float((g.D1[0] @ u[2, 0, k0].real)[-1])
        return dict(E=E, I=I, D=D, tau_w=tau, flux=flux, beta=self.beta)

    def boundary_and_divergence(self, u):
        """Largest boundary-condition residual over the modes,
        max_mk max(|u_+(1) - b_+|, |u_-(1) - b_-|, |u_z(1) - b_z|, |div u(1)|)
        (the vector g of Section 2, b the wall velocity, zero for no slip), and
        the largest interior divergence max_mk max_{n<N-1} |div u_mk(r_n)|,
        with div u = (1/r) d(r u_r)/dr + (i m/r) u_theta + i kappa u_z written
        in the (+,-,z) form."""
        v = to_pm(u)
        b = np.zeros(v.shape[:3], dtype=complex) if self.p.wall is None else to_pm(self.p.wall[..., None])[..., 0]
        gmax = dmax = 0.0
        for mi in range(self.M):
            m = self.p.mp * mi
            dv = self.div_pm(m, self.kap, v[0, mi], v[1, mi], v[2, mi])
            bc = np.stack([v[0, mi][:, -1] - b[0, mi], v[1, mi][:, -1] - b[1, mi], v[2, mi][:, -1] - b[2, mi],
                           dv[:, -1]])
            gmax = max(gmax, float(np.max(np.abs(bc))))
            dmax = max(dmax, float(np.max(np.abs(dv[:, :-1]))))
        return gmax, dmax

    def cfl(self, u):
        """dt max over the dealiased physical grid (N x 3M x 3K) of
        |u_r|/dr_n + |u_theta|/(r_n dtheta) + |u_z|/dz, with dtheta = 2 pi/(mp 3M),
        dz = 2 pi/(alpha 3K) and dr_n the distance from r_n to its nearer
        radial neighbour (the axis mirror -r_0 counts as the neighbour of r_0)."""
        p, r = self.p, self.g.r
        ur, ut, uz = (to_physical(u[c], self.M, self.K) for c in range(3))
        left = np.concatenate([[2.0 * r[0]], np.diff(r)])
        right = np.concatenate([np.diff(r), [np.inf]])
        dr = np.minimum(left, right)
        dth = 2.0 * np.pi / (p.mp * 3 * self.M)
        dz = 2.0 * np.pi / (p.alpha * 3 * self.K)
        loc = (np.abs(ur) / dr[:, None, None] + np.abs(ut) / (r[:, None, None] * dth) + np.abs(uz) / dz)
        return float(p.dt * np.max(loc))

    def energy_norm(self, u):
        """||u||^2 = sum_k sum_{m>=0} c_m sum_n w_n |u_mk(r_n)|^2."""
        return np.sqrt(self.mode_integrals(u))
