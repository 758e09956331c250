"""Newton-Krylov pieces for travelling waves (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section 2: a Newton solver for invariant solutions calls the time integrator
as a black box; Section 3.2: a travelling wave is an equilibrium in a frame
moving with its phase speed.  With Phi_T the time-T map (T/dt steps) and
shift(A, s)_k = A_k exp(-i alpha k s), which moves a pattern downstream by s,
a travelling wave of speed c_w satisfies
    F(x) = shift(Phi_T(x), -c_w T) - x = 0.
Vectors are spectral states; the inner product is the energy one,
<a, b> = sum_k sum_{m>=0} c_m sum_n w_n Re(a_mk(r_n) conj(b_mk(r_n))),
c_0 = 1, c_m = 2 (Parseval for real fields).
Linear systems J dx = -F are solved by restarted GMRES (Saad & Schultz 1986):
Arnoldi with modified Gram-Schmidt and Givens rotations on the Hessenberg
matrix; J v is the forward difference (F(x + eps v) - F(x)) / eps.
"""
import numpy as np


def shift(o, u, s):
    """shift(A, s)_k = A_k exp(-i alpha k s)."""
    K = o.K
    k = np.arange(-(K - 1), K)
    return u * np.exp(-1j * o.p.alpha * k * s)[None, None, :, None]


def inner(o, a, b):
    cm = np.full(o.M, 2.0)
    cm[0] = 1.0
    per = np.sum((a * np.conj(b)).real * o.g.w, axis=-1)  # [3][M][nk]
    return float(np.sum(cm[None, :, None] * per))


def norm(o, a):
    return np.sqrt(max(inner(o, a, a), 0.0))


def residual(o, x, T, s):
    nsteps = int(round(T / o.p.dt))
    return shift(o, o.run(x, nsteps), -s) - x


def jvp(o, x, v, T, s, F0=None, eps_rel=1e-7):
    if F0 is None:
        F0 = residual(o, x, T, s)
    nv = norm(o, v)
    if nv == 0.0:
        return np.zeros_like(x)
    eps = eps_rel * max(norm(o, x), 1.0) / nv
    return (residual(o, x + eps * v, T, s) - F0) / eps


def gmres(apply, b, dot, m=40, tol=1e-10, maxit=400, x0=None):
    """Restarted GMRES(m) for A x = b with inner product `dot`.  Returns
    (x, history of residual-norm estimates, number of products with A)."""
    def nrm(v):
        return np.sqrt(max(dot(v, v), 0.0))

    x = np.zeros_like(b) if x0 is None else x0.copy()
    bn = nrm(b)
    hist = []
    total = 0
    if bn == 0.0:
        return x, [0.0], 0
    while True:
        if x0 is None and total == 0:
            r = b.copy()
        else:
            r = b - apply(x)
            total += 1
        beta = nrm(r)
        hist.append(beta)
        if beta <= tol * bn or total >= maxit:
            return x, hist, total
        V = [r / beta]
        H = np.zeros((m + 1, m))
        cs, sn = np.zeros(m), np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        k = 0
        for j in range(m):
            w = apply(V[j])
            total += 1
            for i in range(j + 1):  # modified Gram-Schmidt
                H[i, j] = dot(w, V[i])
                w = w - H[i, j] * V[i]
            hn = nrm(w)
            H[j + 1, j] = hn
            for i in range(j):  # previous Givens rotations
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            d = np.hypot(H[j, j], H[j + 1, j])
            cs[j], sn[j] = (1.0, 0.0) if d == 0.0 else (H[j, j] / d, H[j + 1, j] / d)
            H[j, j] = d
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            k = j + 1
            hist.append(abs(g[k]))
            if abs(g[k]) <= tol * bn or hn == 0.0 or total >= maxit:
                break
            V.append(w / hn)
        y = np.linalg.solve(np.triu(H[:k, :k]), g[:k])
        for i in range(k):
            x = x + y[i] * V[i]
        if abs(g[k]) <= tol * bn or total >= maxit:
            return x, hist, total


def newton(o, x, T, s, tol=1e-8, m=40, max_newton=20, gmres_tol=1e-3):
    """Newton iteration for F(x) = 0 at a fixed shift s (phase speed s / T)
    with GMRES(m) for J dx = -F and a backtracking line search on ||F||."""
    F = residual(o, x, T, s)
    hist = [norm(o, F) / norm(o, x)]
    for _ in range(max_newton):
        if hist[-1] <= tol:
            break
        F0 = F

        def apply(v):
            return jvp(o, x, v, T, s, F0=F0)

        dx, _, _ = gmres(apply, -F, lambda a, b: inner(o, a, b), m=m, tol=gmres_tol)
        lam = 1.0
        while True:
            xn = x + lam * dx
            Fn = residual(o, xn, T, s)
            if norm(o, Fn) < norm(o, F) or lam < 1e-3:
                break
            lam *= 0.5
        x, F = xn, Fn
        hist.append(norm(o, F) / norm(o, x))
    return x, hist


# ---- travelling waves with a free phase speed ---------------------------
# Section 3.2: a travelling wave is an equilibrium in a frame moving with its
# phase speed c_w, which is not known in advance.  The unknowns become
# X = (x, c_w) with the residual F(x, c_w) = shift(Phi_T(x), -c_w T) - x and
# one more equation, the phase condition <d_z x, dx> = 0 on the update (it
# removes the axial-shift direction, along which every shifted copy of a
# travelling wave is another one).  d_z is the spectral axial derivative
# i alpha k.  Extended vectors are flat complex arrays: the field, then
# c_w; their inner product is the energy inner product plus the product of
# the speed entries.  The derivative of F in c_w is T d_z shift(Phi_T(x),
# -c_w T), which the forward difference reproduces.  Where ||d_z x|| /
# ||x|| < freeze (laminar flow is a travelling wave of every speed, so the
# speed direction is null there) the step keeps c_w and solves for x alone.

def ddz(o, u):
    """Axial derivative d_z of a spectral field: i alpha k A_k."""
    k = np.arange(-(o.K - 1), o.K)
    return 1j * o.p.alpha * k[None, None, :, None] * u


class TravellingWave:
    """Residual, inner product and Jacobian product of the free-speed
    travelling-wave system for a time-T map `phi` (by default T/dt steps
    of the oracle's predictor-corrector)."""

    def __init__(self, o, T, phi=None, freeze=1e-6, eps_rel=1e-7):
        self.o, self.T = o, T
        n = int(round(T / o.p.dt))
        self.phi = phi if phi is not None else (lambda x: o.run(x, n))
        self.freeze, self.eps_rel = freeze, eps_rel
        self.shape = (3, o.M, o.nk, o.N)
        self.size = int(np.prod(self.shape))

    def pack(self, x, c):
        return np.concatenate([np.ravel(x), np.array([c], dtype=complex)])

    def unpack(self, X):
        return X[:self.size].reshape(self.shape), float(X[-1].real)

    def dot(self, A, B):
        a, ca = self.unpack(A)
        b, cb = self.unpack(B)
        return inner(self.o, a, b) + ca * cb

    def residual(self, X):
        x, c = self.unpack(X)
        return self.pack(shift(self.o, self.phi(x), -c * self.T) - x, 0.0)

    def speed_active(self, X):
        """False where the state is (nearly) invariant under axial shifts."""
        x, _ = self.unpack(X)
        return norm(self.o, ddz(self.o, x)) > self.freeze * norm(self.o, x)

    def jvp(self, X, F0, V, active):
        """Forward difference of the residual in (x, c_w) plus the phase
        row <d_z x, v>; with active False the speed is held fixed."""
        V = V.copy()
        if not active:
            V[-1] = 0.0
        nv = np.sqrt(max(self.dot(V, V), 0.0))
        if nv == 0.0:
            return np.zeros_like(X)
        eps = self.eps_rel * max(np.sqrt(self.dot(X, X)), 1.0) / nv
        out = (self.residual(X + eps * V) - F0) / eps
        x, _ = self.unpack(X)
        v, _ = self.unpack(V)
        out[-1] = inner(self.o, ddz(self.o, x), v) if active else 0.0
        return out


def newton_tw(o, x, T, c, tol=1e-8, m=40, max_newton=20, gmres_tol=1e-3, phi=None, freeze=1e-6):
    """Newton iteration for a travelling wave with a free phase speed:
    GMRES(m) on the extended system [J_x, dF/dc; <d_z x, .>, 0] (dx, dc)
    = (-F, 0) and a backtracking line search on ||F||, as newton() does for a
    fixed shift.  Returns (x, c_w, history of ||F|| / ||x||, info) with
    info['frozen'] the Newton steps taken at fixed speed."""
    tw = TravellingWave(o, T, phi, freeze)
    X = tw.pack(x, c)
    F = tw.residual(X)

    def fnorm(Fv):
        return np.sqrt(max(tw.dot(Fv, Fv), 0.0))

    hist = [fnorm(F) / norm(o, tw.unpack(X)[0])]
    info = {"frozen": 0, "steps": []}
    for _ in range(max_newton):
        if hist[-1] <= tol:
            break
        active = tw.speed_active(X)
        info["frozen"] += 0 if active else 1
        F0 = F
        dX, _, _ = gmres(lambda v: tw.jvp(X, F0, v, active), -F, tw.dot, m=m, tol=gmres_tol)
        info["steps"].append(dX)
        lam = 1.0
        while True:
            Xn = X + lam * dX
            Fn = tw.residual(Xn)
            if fnorm(Fn) < fnorm(F) or lam < 1e-3:
                break
            lam *= 0.5
        X, F = Xn, Fn
        hist.append(fnorm(F) / norm(o, tw.unpack(X)[0]))
    xs, cs = tw.unpack(X)
    return xs, cs, hist, info
