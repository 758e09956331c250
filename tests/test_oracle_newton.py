"""Pins of the oracle's travelling-wave residual, JVP and GMRES.

Section 2 (Newton-Krylov for invariant solutions; Section 3.2: a travelling
wave is an equilibrium in a frame moving with its phase speed).  Pins:
laminar flow is a travelling wave of every speed (F = 0 for any T, s); a
shift by one pipe length is the identity and shifts compose; the
finite-difference JVP agrees with a two-sided difference; GMRES matches a
dense least-squares / direct solve on small explicit systems, under a
non-Euclidean inner product too.  Free phase speed: the extended iteration
finds the speed of a model map with one isolated travelling wave, the speed
column equals its closed form T d_z shift(Phi_T(x), -c T), and near laminar
flow the iteration converges with the speed frozen.
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


# ---- free phase speed (Section 3.2: equilibrium in a moving frame) --------

def test_free_speed_finds_the_speed_of_a_model_travelling_wave():
    """A shift-equivariant model map with one isolated travelling wave (up
    to axial shifts): Phi_T(x) = shift(0.5 x' + g x_11, c* T), with x_11 the
    (m index 1, k = 1) part of x, x' the rest and g = 1 + (1 - |x_11|^2 /
    a^2) / 2, so |x_11| relaxes to a while the pattern moves at speed c*.
    Its travelling waves with axial structure are x = x_11, |x_11| = a, of
    speed c* only.  From c_w = c* + 0.04, c* - 0.2 and c* + 0.3 the extended
    Newton iteration must return c* to round-off with x' = 0 and |x_11| = a.
    (Measured on this test: a sign error in the speed column leaves c_w at
    0.17-0.89 with ||F|| / ||x|| >= 0.07 after 40 steps, and without the phase
    row c_w never moves.)"""
    from oracle.newton import newton_tw
    o = small()
    x = make_state(16, 3, 3, 2, 1.25, o.g.r, 1e-2, 4.0, 4.0, 8, laminar=False)

    def part(v):
        p = np.zeros_like(v)
        p[:, 1, 3] = v[:, 1, 3]
        return p

    a = 0.8 * norm(o, part(x))
    T, cstar = 0.7, 0.43

    def phi(v):
        p = part(v)
        g = 1.0 + 0.5 * (1.0 - norm(o, p) ** 2 / a ** 2)
        return shift(o, 0.5 * (v - p) + g * p, cstar * T)

    for c0 in (cstar + 0.04, cstar - 0.2, cstar + 0.3):
        xs, cs, hist, info = newton_tw(o, x, T, c0, tol=1e-12, gmres_tol=1e-10, phi=phi, max_newton=40)
        assert abs(cs - cstar) <= 1e-10, (c0, cs, hist)
        assert hist[-1] <= 1e-12 and info["frozen"] == 0
        assert norm(o, xs - part(xs)) <= 1e-12 * a
        assert abs(norm(o, part(xs)) / a - 1.0) <= 1e-11


def test_speed_column_is_T_dz_of_the_shifted_map():
    """dF/dc_w = T d_z shift(Phi_T(x), -c_w T): the forward-difference
    product with the unit speed direction against that closed form."""
    from oracle.newton import TravellingWave, ddz
    o = small()
    x = make_state(16, 3, 3, 2, 1.25, o.g.r, 1e-2, 4.0, 4.0, 9)
    T, c = 0.05, 0.6
    tw = TravellingWave(o, T)
    X = tw.pack(x, c)
    F0 = tw.residual(X)
    V = np.zeros_like(X)
    V[-1] = 1.0
    got, gc = tw.unpack(tw.jvp(X, F0, V, True))
    closed = T * ddz(o, shift(o, o.run(x, 5), -c * T))
    assert norm(o, got - closed) <= 1e-5 * norm(o, closed)
    assert gc == 0.0  # the phase row sees only the field part
    # the phase row of a field direction: <d_z x, v>, zero for an axially
    # uniform v (k = 0 only) and positive for v = d_z x
    v0 = np.zeros_like(x)
    v0[:, :, 2] = x[:, :, 2]
    assert abs(tw.unpack(tw.jvp(X, F0, tw.pack(v0, 0.0), True))[1]) <= 1e-14 * norm(o, x) ** 2
    assert tw.unpack(tw.jvp(X, F0, tw.pack(ddz(o, x), 0.0), True))[1] > 0.0


def test_free_speed_newton_reaches_laminar_flow_and_freezes_the_speed():
    """Near laminar flow the only travelling wave is laminar flow, which has
    every speed: the extended iteration converges there and takes its last
    steps at fixed speed, once ||d_z x|| / ||x|| < 1e-6."""
    from oracle.newton import newton_tw
    o = Oracle(Params(N=12, M=2, K=2, mp=2, alpha=1.25, Re=100.0, dt=0.05))
    x = make_state(12, 2, 2, 2, 1.25, o.g.r, 1e-4, 4.0, 4.0, 6)
    xs, cs, hist, info = newton_tw(o, x, 1.0, 0.3, tol=1e-10, gmres_tol=1e-6)
    assert hist[-1] <= 1e-10, hist
    lam = laminar_state(12, 2, 2, o.g.r)
    assert norm(o, xs - lam) / norm(o, lam) < 1e-8
    assert info["frozen"] >= 1 and np.isfinite(cs)
