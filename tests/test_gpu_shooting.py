"""GPU parity of the multiple-shooting orbit solver (opf_shoot_solve) against
the oracle's solve_orbit: two sections of 25 steps, free period and shift,
near-laminar guess (N=12, |m|, |k| < 2, Re 50, T = 4, shift 0.1).

Tolerance: as for the hookstep (forward-difference products carry the
~1e-13 residual difference divided by eps ~ 1e-7), so the first step
agrees to 1e-4 of its length and the period and shift updates to 1e-4
relative; counts must be equal."""
import numpy as np
import pytest

from inputs import laminar_state, make_state
from gpu_support import make_ensemble, make_solver, oracle_nodes  # noqa: F401

pytestmark = pytest.mark.gpu

KW = dict(N=12, M=2, K=2, mp=1, alpha=1.25, Re=50.0, dt=0.08)
T, SHIFT, N_SEC = 4.0, 0.1, 25


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def setup():
    import torch

    import paper_1705_03838_amd as opf
    from oracle import Oracle, Params
    from oracle.shooting import Shooting
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    s = make_solver(**KW)
    p = Params(**KW)
    x = make_state(12, 2, 2, 1, 1.25, s.nodes(), 1e-3, 3.0, 3.0, 7)
    x2 = Shooting(p, 2, N_SEC).oracle(T).run(x, N_SEC)
    return torch, s, p, np.stack([x, x2])


def test_first_step_matches_oracle(setup):
    from oracle.shooting import solve_orbit
    torch, s, p, xs = setup
    say("shooting first step")
    g, Tg, sg, rep = s.shoot_solve(torch.from_numpy(xs), T, SHIFT, N_SEC, gmres_m=20, max_newton=1, tol=1e-12,
                                   gmres_tol=1e-3)
    out, To, so, hist, info = solve_orbit(p, list(xs), T, SHIFT, N_SEC, tol=1e-12, m=20, gmres_tol=1e-3,
                                          max_newton=1)
    say("  ", rep, To, so)
    assert rep["products"] == info["products"] and rep["hook_trials"] == info["trials"]
    step = np.sqrt(sum(np.sum(np.abs(a - b) ** 2) for a, b in zip(out, xs)))
    err = np.sqrt(sum(np.sum(np.abs(a - b) ** 2) for a, b in zip(g.cpu().numpy(), out)))
    assert err <= 1e-4 * step
    assert abs((Tg - T) - (To - T)) <= 1e-4 * abs(To - T) + 1e-12
    assert abs((sg - SHIFT) - (so - SHIFT)) <= 1e-4 * abs(so - SHIFT) + 1e-12
    assert abs(rep["history"][1] - hist[1]) <= 1e-4 * hist[1]


def test_orbit_search_reaches_laminar_flow(setup):
    torch, s, p, xs = setup
    say("shooting to laminar")
    g, Tg, sg, rep = s.shoot_solve(torch.from_numpy(xs), T, SHIFT, N_SEC, gmres_m=20, tol=1e-8, gmres_tol=1e-3)
    say("  ", rep, Tg, sg)
    assert rep["converged"] and not rep["stalled"]
    lam = laminar_state(12, 2, 2, s.nodes())
    for z in g.cpu().numpy():
        assert np.max(np.abs(z - lam)) <= 1e-7
    assert np.isfinite(Tg) and np.isfinite(sg)


def test_fixed_period_single_section_is_the_travelling_wave_search(setup):
    """S = 1 with T and s fixed and n = T/dt solves the same residual as
    opf_nk_solve's hookstep; both reach laminar flow."""
    torch, s, p, xs = setup
    g, Tg, sg, rep = s.shoot_solve(torch.from_numpy(xs[:1]), T, SHIFT, 50, free_T=False, free_s=False, gmres_m=20,
                                   tol=1e-8, gmres_tol=1e-3)
    assert Tg == T and sg == SHIFT and rep["converged"]
    xn, nrep = s.nk_solve(torch.from_numpy(xs[0]), T, SHIFT / T, gmres_m=20, tol=1e-8, gmres_tol=1e-3, hookstep=True)
    assert nrep["converged"]
    assert np.max(np.abs(g.cpu().numpy()[0] - xn.cpu().numpy())) <= 1e-7
