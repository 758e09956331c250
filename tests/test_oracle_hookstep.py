"""Pins of the oracle's hookstep Newton iteration: the trust-region
subproblem against a QR least-squares solve, the closed form of a
diagonal Hessenberg matrix, the secular equation written through an SVD, a
brute-force search over the circle and its optimality conditions; the
iteration on a coupled arctan system (where plain Newton diverges) and on a
linear system (one exact step)."""
import numpy as np
import pytest

from oracle.hookstep import hook_subproblem, newton_hook


def rng_hb(k, seed):
    r = np.random.default_rng(seed)
    Hb = np.triu(r.standard_normal((k + 1, k)), -1)  # upper Hessenberg
    return Hb


def test_unconstrained_is_least_squares():
    Hb = rng_hb(6, 1)
    b = np.zeros(7)
    b[0] = 2.5
    Q, R = np.linalg.qr(Hb)
    ls = np.linalg.solve(R, Q.T @ b)
    y, mu, r = hook_subproblem(Hb, 2.5, 1e6)
    assert mu == 0.0
    assert np.allclose(y, ls, rtol=1e-12, atol=1e-12)
    assert abs(r - np.linalg.norm(b - Hb @ ls)) <= 1e-12


def test_diagonal_closed_form():
    sig = np.array([3.0, 0.5, 0.2])
    Hb = np.vstack([np.diag(sig), np.zeros((1, 3))])
    beta, delta = 2.0, 0.1
    y, mu, r = hook_subproblem(Hb, beta, delta)
    # only the first direction sees b = beta e_1: y_1 = beta s_1 / (s_1^2 + mu) = delta
    assert mu == pytest.approx(beta * sig[0] / delta - sig[0] ** 2, rel=1e-12)
    assert np.allclose(y, [delta, 0.0, 0.0], atol=1e-15)
    assert r == pytest.approx(np.hypot(beta - sig[0] * delta, 0.0), rel=1e-12)


def test_secular_equation_through_svd():
    Hb = rng_hb(8, 2)
    beta, delta = 1.7, 0.05
    U, s, Wt = np.linalg.svd(Hb, full_matrices=False)
    p = beta * U[0]

    def length(mu):
        return np.linalg.norm(p * s / (s ** 2 + mu))

    lo, hi = 0.0, 1.0
    while length(hi) > delta:
        hi *= 2
    for _ in range(200):  # plain bisection
        mid = 0.5 * (lo + hi)
        lo, hi = (mid, hi) if length(mid) > delta else (lo, mid)
    mu_ref = 0.5 * (lo + hi)
    y_ref = Wt.T @ (p * s / (s ** 2 + mu_ref))
    y, mu, _ = hook_subproblem(Hb, beta, delta)
    assert mu == pytest.approx(mu_ref, rel=1e-10)
    assert np.allclose(y, y_ref, rtol=1e-9, atol=1e-14)


def test_brute_force_on_the_circle_and_optimality():
    Hb = rng_hb(2, 3)
    beta, delta = 1.0, 0.3
    b = np.array([beta, 0.0, 0.0])
    y, mu, r = hook_subproblem(Hb, beta, delta)
    th = np.linspace(0, 2 * np.pi, 400001)
    pts = delta * np.stack([np.cos(th), np.sin(th)], 1)
    best = np.min(np.linalg.norm(b[None] - pts @ Hb.T, axis=1))
    assert mu > 0 and abs(np.linalg.norm(y) - delta) <= 1e-12
    assert abs(r - best) <= 1e-9
    # KKT: (Hb^T Hb + mu I) y = Hb^T b
    assert np.allclose((Hb.T @ Hb + mu * np.eye(2)) @ y, Hb.T @ b, atol=1e-12)


def coupled_arctan(n=5, seed=4):
    r = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(r.standard_normal((n, n)))
    xs = np.ones(n)

    def F(x):
        return Q @ np.arctan(Q.T @ (x - xs))

    def jv(x, _F, v):
        t = Q.T @ (x - xs)
        return Q @ ((Q.T @ v) / (1 + t * t))

    return Q, xs, F, jv


def test_hookstep_converges_where_newton_diverges():
    Q, xs, F, jv = coupled_arctan()
    x0 = xs + Q @ np.array([2.0, 1.5, -3.0, 0.5, 2.5])
    # a full Newton step from x0 increases the residual
    t0 = Q.T @ (x0 - xs)
    xn = x0 - Q @ (np.arctan(t0) * (1 + t0 * t0))
    assert np.linalg.norm(F(xn)) > np.linalg.norm(F(x0))
    x, hist, info = newton_hook(F, jv, np.dot, x0, tol=1e-12, m=5, max_newton=40, gmres_tol=1e-12)
    assert hist[-1] <= 1e-12 and np.linalg.norm(x - xs) <= 1e-10
    assert info["trials"] > len(hist) - 1  # some steps were rejected and shortened
    fns = info["fnorms"]
    assert all(f1 < f0 for f0, f1 in zip(fns, fns[1:]))  # accepted steps reduce ||F||


def test_linear_system_one_step():
    r = np.random.default_rng(6)
    A = r.standard_normal((6, 6)) + 4 * np.eye(6)
    bb = r.standard_normal(6)
    x, hist, info = newton_hook(lambda x: A @ x - bb, lambda x, F, v: A @ v, np.dot, np.ones(6), tol=1e-12,
                                m=6, gmres_tol=1e-14)
    assert len(hist) == 2 and hist[-1] <= 1e-12
    assert np.allclose(x, np.linalg.solve(A, bb), rtol=1e-12)


def test_pipe_residual_converges_to_laminar_flow():
    """Near-laminar guess (N=12, |m|, |k| < 3, Re 400, T = 2, shift 0.1): the
    hookstep iteration reaches laminar flow, a solution for every shift."""
    from inputs import laminar_state, make_state
    from oracle import Oracle, Params
    from oracle.hookstep import newton_hook_pipe
    o = Oracle(Params(N=12, M=3, K=3, alpha=1.25, Re=400.0, dt=0.04))
    x = make_state(12, 3, 3, 1, 1.25, o.g.r, 1e-3, 3.0, 3.0, 7)
    xh, hist, info = newton_hook_pipe(o, x, 2.0, 0.1, tol=1e-8, m=12, gmres_tol=1e-3, delta0=0.01)
    assert hist[-1] <= 1e-8 and not info["stalled"]
    assert np.max(np.abs(xh - laminar_state(12, 3, 3, o.g.r))) <= 1e-7
    assert info["mus"][0] > 0  # the radius 0.01 holds the first step below the Newton step
