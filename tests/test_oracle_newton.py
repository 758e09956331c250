"""Pins of the oracle's travelling-wave residual, JVP and GMRES.

Section 2 (Newton-Krylov for invariant solutions; Section 3.2: a travelling
wave is an equilibrium in a frame moving with its phase speed).  Pins:
laminar flow is a travelling wave of every speed (F = 0 for any T, s); a
shift by one pipe length is the identity and shifts compose; the
finite-difference JVP agrees with a two-sided difference; GMRES matches a
dense least-squares / direct solve on small explicit systems, under a
non-Euclidean inner product too.
"""
import numpy as np

from inputs import laminar_state, make_state
from oracle import Oracle, Params
from oracle.newton import gmres, inner, jvp, newton, norm, residual, shift


def small():
    return Oracle(Params(N=16, M=3, K=3, mp=2, alpha=1.25, Re=2400.0, dt=0.01))


def test_laminar_is_a_travelling_wave_of_any_speed():
    o = small()
    x = laminar_state(16, 3, 3, o.g.r)
    for T, s in [(0.05, 0.0), (0.05, 0.3), (0.1, -1.7)]:
        assert norm(o, residual(o, x, T, s)) / norm(o, x) < 1e-13


def test_shift_period_and_composition():
    o = small()
    u = make_state(16, 3, 3, 2, 1.25, o.g.r, 1e-2, 4.0, 4.0, 3)
    lz = 2 * np.pi / 1.25
    assert np.max(np.abs(shift(o, u, lz) - u)) < 1e-13
    assert np.max(np.abs(shift(o, shift(o, u, 0.3), 0.4) - shift(o, u, 0.7))) < 1e-14
    # energy inner product is Parseval: shift preserves the norm
    assert abs(norm(o, shift(o, u, 0.9)) - norm(o, u)) < 1e-14


def test_jvp_matches_central_difference():
    o = small()
    x = make_state(16, 3, 3, 2, 1.25, o.g.r, 1e-2, 4.0, 4.0, 4)
    v = make_state(16, 3, 3, 2, 1.25, o.g.r, 1e-2, 4.0, 4.0, 5, laminar=False)
    T, s = 0.03, 0.02
    a = jvp(o, x, v, T, s)
    h = 1e-5 * norm(o, x) / norm(o, v)
    c = (residual(o, x + h * v, T, s) - residual(o, x - h * v, T, s)) / (2 * h)
    assert norm(o, a - c) / norm(o, c) < 1e-6


def test_gmres_matches_dense_solve():
    rng = np.random.default_rng(0)
    n = 30
    A = np.eye(n) * 3 + rng.standard_normal((n, n)) * 0.3
    b = rng.standard_normal(n)
    W = np.diag(rng.uniform(0.5, 2.0, n))     # non-Euclidean inner product
    dot = lambda p, q: float(p @ W @ q)        # noqa: E731
    x, hist, nmv = gmres(lambda v: A @ v, b, dot, m=40, tol=1e-12)
    assert np.max(np.abs(x - np.linalg.solve(A, b))) < 1e-10
    assert hist[-1] <= 1e-12 * np.sqrt(dot(b, b)) * 1.01
    # restarted: GMRES(5) still converges on this well-conditioned system
    x5, _, _ = gmres(lambda v: A @ v, b, dot, m=5, tol=1e-12, maxit=400)
    assert np.max(np.abs(x5 - np.linalg.solve(A, b))) < 1e-9
    # rectangular least squares on the Krylov space equals the minimum-residual update
    x1, _, _ = gmres(lambda v: A @ v, b, dot, m=3, tol=0.0, maxit=3)
    K = np.stack([b, A @ b, A @ A @ b], axis=1)
    Wh = np.sqrt(W)  # W is diagonal
    y, *_ = np.linalg.lstsq(Wh @ (A @ K), Wh @ b, rcond=None)
    assert np.max(np.abs(x1 - K @ y)) < 1e-10


def test_newton_converges_to_laminar_from_near_laminar_guess():
    """Near laminar flow the only travelling wave is laminar flow itself;
    T is long against the slowest Stokes decay time (Re = 100) so that the
    Jacobian Phi_T' - 1 is well conditioned."""
    o = Oracle(Params(N=12, M=2, K=2, mp=2, alpha=1.25, Re=100.0, dt=0.05))
    x = make_state(12, 2, 2, 2, 1.25, o.g.r, 1e-4, 4.0, 4.0, 6)
    xs, hist = newton(o, x, 1.0, 0.0, tol=1e-10, gmres_tol=1e-6)
    assert hist[-1] <= 1e-10, hist
    lam = laminar_state(12, 2, 2, o.g.r)
    assert norm(o, xs - lam) / norm(o, lam) < 1e-8
