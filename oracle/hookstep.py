"""Newton iteration with a Krylov trust-region step, the hookstep (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section 2: the Newton solver for invariant solutions calls a method that
combines Krylov subspaces with a trust region (Viswanath 2007).  The reading
used here:

  * Arnoldi without restart from v_1 = -F / beta, beta = ||F||, gives an
    orthonormal basis V_k and the (k+1) x k Hessenberg matrix Hb with
    J V_k = V_{k+1} Hb.  It stops when the least-squares residual
    min_y ||beta e_1 - Hb y|| falls to gmres_tol * beta, at breakdown, or
    after m products.
  * Hookstep: y minimises ||beta e_1 - Hb y|| subject to ||y|| <= Delta, and
    dx = V_k y (so ||dx|| = ||y||).  Its solution is
    y(mu) = (Hb^T Hb + mu I)^{-1} Hb^T beta e_1 with mu = 0 when the
    minimum-norm least-squares solution fits, else the mu > 0 with
    ||y(mu)|| = Delta.
  * Trust region: rho = (||F||^2 - ||F(x + dx)||^2) / (||F||^2 - r^2), with
    r = ||beta e_1 - Hb y|| the linear model's residual.  rho < 0.1 rejects
    the step, halves Delta to ||dx|| / 2 and solves the subproblem again on
    the same basis (at most max_hook tries).  An accepted step doubles Delta
    (up to delta_max) when rho > 0.75 and the step reached the boundary, and
    sets Delta = ||dx|| / 2 when rho < 0.25.  The first Delta is delta0, or
    the length of the first unconstrained step when delta0 <= 0.

Here the subproblem is solved as a damped least-squares problem with a
bracketing root finder for mu; the library solves it through an SVD of Hb.
"""
import numpy as np
from scipy.optimize import brentq


def hook_subproblem(Hb, beta, delta):
    """(y, mu, r): the hookstep coefficients, the multiplier and the model
    residual ||beta e_1 - Hb y||."""
    Hb = np.asarray(Hb, dtype=np.float64)
    k = Hb.shape[1]
    b = np.zeros(Hb.shape[0])
    b[0] = beta
    y, *_ = np.linalg.lstsq(Hb, b, rcond=None)
    mu = 0.0
    if np.linalg.norm(y) > delta:
        # y(mu) solves the damped least-squares problem
        # min ||[Hb; sqrt(mu) I] y - [b; 0]||, whose normal equations are
        # (Hb^T Hb + mu I) y = Hb^T b (solved by QR, not squaring cond(Hb))
        zeros = np.zeros(k)

        def y_of(m):
            return np.linalg.lstsq(np.vstack([Hb, np.sqrt(m) * np.eye(k)]), np.concatenate([b, zeros]),
                                   rcond=None)[0]

        def excess(m):
            return np.linalg.norm(y_of(m)) - delta

        hi = max(np.linalg.norm(Hb.T @ b) / delta, 1e-300)
        while excess(hi) > 0:
            hi *= 2.0
        mu = brentq(excess, 0.0, hi, xtol=1e-300, rtol=4 * np.finfo(float).eps, maxiter=500)
        y = y_of(mu)
    return y, mu, float(np.linalg.norm(b - Hb @ y))


def arnoldi(jv, dot, F, m, gmres_tol):
    """Basis V (list), Hessenberg Hb [(k+1) x k], beta and the products used."""
    def nrm(v):
        return np.sqrt(max(dot(v, v), 0.0))

    beta = nrm(F)
    V = [-F / beta]
    Hb = np.zeros((m + 1, m))
    k = 0
    for j in range(m):
        w = jv(V[j])
        for i in range(j + 1):  # modified Gram-Schmidt
            Hb[i, j] = dot(w, V[i])
            w = w - Hb[i, j] * V[i]
        hn = nrm(w)
        Hb[j + 1, j] = hn
        k = j + 1
        b = np.zeros(k + 1)
        b[0] = beta
        y, *_ = np.linalg.lstsq(Hb[:k + 1, :k], b, rcond=None)
        res = np.linalg.norm(b - Hb[:k + 1, :k] @ y)
        if res <= gmres_tol * beta or hn == 0.0:
            break
        V.append(w / hn)
    return V[:k], Hb[:k + 1, :k], beta, k


def newton_hook(resid, jv, dot, x, tol=1e-8, m=40, max_newton=20, gmres_tol=1e-3, delta0=0.0,
                delta_max=np.inf, max_hook=12):
    """Newton-Krylov-hookstep for resid(x) = 0.  jv(x, F, v) is the Jacobian
    product at x (F = resid(x)).  Returns (x, history of ||F|| / ||x||, info)."""
    def nrm(v):
        return np.sqrt(max(dot(v, v), 0.0))

    F = resid(x)
    fn = nrm(F)
    hist = [fn / nrm(x)]
    delta = delta0
    info = dict(products=0, residuals=1, trials=0, stalled=False, deltas=[], fnorms=[fn], mus=[])
    for _ in range(max_newton):
        if hist[-1] <= tol:
            break
        V, Hb, beta, k = arnoldi(lambda v: jv(x, F, v), dot, F, m, gmres_tol)
        info["products"] += k
        if delta <= 0.0:
            delta = np.linalg.norm(hook_subproblem(Hb, beta, np.inf)[0])
        accepted = False
        for _ in range(max_hook):
            y, mu, r = hook_subproblem(Hb, beta, delta)
            dx = sum(yi * vi for yi, vi in zip(y, V))
            dn = np.linalg.norm(y)
            xn = x + dx
            Fn = resid(xn)
            info["residuals"] += 1
            info["trials"] += 1
            fnn = nrm(Fn)
            den = fn * fn - r * r
            rho = (fn * fn - fnn * fnn) / den if den > 0 else -np.inf
            if rho >= 0.1:
                accepted = True
                info["mus"].append(mu)
                if rho > 0.75 and dn >= 0.99 * delta:
                    delta = min(2.0 * delta, delta_max)
                elif rho < 0.25:
                    delta = 0.5 * dn
                break
            delta = 0.5 * dn
        info["deltas"].append(delta)
        if not accepted:
            info["stalled"] = True
            break
        x, F, fn = xn, Fn, fnn
        hist.append(fn / nrm(x))
        info["fnorms"].append(fn)
    return x, hist, info


def newton_hook_pipe(o, x, T, s, **kw):
    """The hookstep iteration on the travelling-wave residual of newton.py."""
    from .newton import inner, jvp, residual
    return newton_hook(lambda v: residual(o, v, T, s), lambda xx, F, v: jvp(o, xx, v, T, s, F0=F),
                       lambda a, b: inner(o, a, b), x, **kw)
