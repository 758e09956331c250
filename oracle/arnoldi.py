"""Arnoldi iteration for the leading eigenvalues of the linearised time-T map
(oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Stability of an invariant solution x (the paper's Section 3 example: the
leading eigenvalue of a travelling wave) is given by the eigenvalues mu of
J = d shift(Phi_T(x), -s) / dx, the Floquet multipliers; the growth rate of
an eigenmode is log|mu| / T.  The reading used here:

  * J v is the forward difference (P(x + eps v) - P(x)) / eps with
    P(x) = shift(Phi_T(x), -s), eps = 1e-7 max(||x||, 1) / ||v|| (P = F + x
    for the Newton residual F);
  * Arnoldi with modified Gram-Schmidt in the energy inner product, from a
    given start vector, without restart;
  * every `check_every` products, and at breakdown or after m products, the
    Ritz values (eigenvalues of the leading k x k block of the Hessenberg
    matrix) are ordered by decreasing modulus, and for equal modulus by
    decreasing imaginary part; the iteration stops when the leading nev of
    them moved by at most tol |mu_1| since the previous check.
"""
import numpy as np

from .newton import inner, residual


def order(ev):
    return np.array(sorted(ev, key=lambda z: (-abs(z), -z.imag)))


def arnoldi(o, x, T, s, v0, m, nev, tol=1e-8, check_every=5, eps_rel=1e-7):
    """Returns (leading nev Ritz values, products used, converged flag)."""
    def nrm(v):
        return np.sqrt(max(inner(o, v, v), 0.0))

    P0 = residual(o, x, T, s) + x
    xn = max(nrm(x), 1.0)

    def apply(v):
        eps = eps_rel * xn / nrm(v)
        xe = x + eps * v
        return (residual(o, xe, T, s) + xe - P0) / eps

    V = [v0 / nrm(v0)]
    H = np.zeros((m + 1, m))
    prev, ev, k = None, None, 0
    for j in range(m):
        w = apply(V[j])
        for i in range(j + 1):
            H[i, j] = inner(o, w, V[i])
            w = w - H[i, j] * V[i]
        hn = nrm(w)
        H[j + 1, j] = hn
        k = j + 1
        if k % check_every == 0 or k == m or hn == 0.0:
            ev = order(np.linalg.eigvals(H[:k, :k]))[:nev]
            if hn == 0.0:
                return ev, k, True
            if prev is not None and len(prev) == len(ev) and np.max(np.abs(ev - prev)) <= tol * abs(ev[0]):
                return ev, k, True
            prev = ev
        V.append(w / hn)
    return ev, k, False
