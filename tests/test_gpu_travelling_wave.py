"""GPU parity of the travelling-wave search with a free phase speed
(Section 3.2: a travelling wave is an equilibrium in a frame moving with its
phase speed; Section 2: the Newton solver), and the plain-GMRES fallback of
the preconditioned search.

Tolerances: the first extended Newton step is compared with the oracle's
newton_tw to 1e-4 of the step length, as for the hookstep (forward-difference
products with eps = 1e-7 ||X|| turn ~1e-13 rounding differences of the time
stepper into ~1e-6 relative differences of each product; GMRES to 1e-3 then
amplifies them by at most the conditioning of the small Hessenberg system).
"""
import numpy as np
import pytest

from inputs import laminar_state, make_state
from gpu_support import make_solver, oracle_nodes

pytestmark = pytest.mark.gpu

KW = dict(N=12, M=3, K=3, mp=1, alpha=1.25, Re=400.0, dt=0.04)
T, SPEED = 2.0, 0.5


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def test_first_free_speed_step_matches_oracle(torch_cuda):
    from oracle import Oracle, Params
    from oracle.newton import inner, newton_tw
    say("free-speed Newton step", KW, "T", T, "c_w", SPEED)
    s = make_solver(**KW)
    o = Oracle(Params(**KW))
    x = make_state(12, 3, 3, 1, 1.25, oracle_nodes(12), 1e-3, 3.0, 3.0, 7)
    xg, rep = s.nk_solve(torch_cuda.from_numpy(x), T, SPEED, free_speed=True, gmres_m=12, max_newton=1,
                         tol=1e-12, gmres_tol=1e-3)
    xo, co, hist, info = newton_tw(o, x, T, SPEED, tol=1e-12, m=12, max_newton=1, gmres_tol=1e-3)
    say("  gpu", rep)
    say("  oracle c_w", co, "history", hist)
    assert rep["newton_iterations"] == 1 and rep["frozen_steps"] == 0 and info["frozen"] == 0
    dxo = xo - x
    step = np.sqrt(inner(o, dxo, dxo) + (co - SPEED) ** 2)
    d = xg.cpu().numpy() - xo
    err = np.sqrt(inner(o, d, d) + (rep["speed"] - co) ** 2)
    say(f"  step length {step:.3e}, speed change {co - SPEED:.3e}, gpu-oracle {err:.3e}")
    assert abs(co - SPEED) > 1e-6  # the speed really moved
    assert err <= 1e-4 * step
    assert abs(rep["history"][1] - hist[1]) <= 1e-3 * hist[1]


def test_free_speed_search_reaches_laminar_flow(torch_cuda):
    """Near laminar flow the extended search converges to laminar flow and
    takes its last steps at fixed speed, as the oracle's does."""
    kw = dict(N=12, M=2, K=2, mp=2, alpha=1.25, Re=100.0, dt=0.05)
    say("free-speed search to laminar flow", kw)
    s = make_solver(**kw)
    x = make_state(12, 2, 2, 2, 1.25, oracle_nodes(12), 1e-4, 4.0, 4.0, 6)
    xs, rep = s.nk_solve(torch_cuda.from_numpy(x), 1.0, 0.3, free_speed=True, tol=1e-10, gmres_tol=1e-6)
    say("  ", rep)
    assert rep["converged"] and rep["residual"] <= 1e-10
    assert rep["frozen_steps"] >= 1 and np.isfinite(rep["speed"])
    d = xs.cpu().numpy() - laminar_state(12, 2, 2, oracle_nodes(12))
    assert np.sqrt(s.vec_dot(torch_cuda.from_numpy(d), torch_cuda.from_numpy(d))) < 1e-8


def test_untrained_network_falls_back_to_plain_gmres(torch_cuda):
    """A network with random weights is a poor preconditioner: its flexible
    GMRES cycle misses the tolerance, the step is solved again by plain
    GMRES, and the search still converges to 1e-8."""
    import paper_1705_03838_amd as opf
    from oracle.mlp import flatten, init_params
    kw = dict(N=12, M=4, K=4, mp=2, alpha=1.25, Re=200.0, dt=0.05)
    say("untrained network fallback", kw)
    s = make_solver(**kw)
    net = opf.Mlp(s, width=64, layers=2, rank=4)
    p = init_params(net.din, 64, 2, net.dout, seed=31)
    p["W_out"] *= 40.0
    net.set_params(flatten(p, 2).astype(np.float32))
    x = torch_cuda.from_numpy(make_state(12, 4, 4, 2, 1.25, oracle_nodes(12), 1e-4, 4.0, 4.0, 17))
    xp, rp = s.nk_solve(x, 2.0, 0.0, tol=1e-8, gmres_tol=1e-3)
    xs, rep = s.nk_solve(x, 2.0, 0.0, tol=1e-8, gmres_tol=1e-3, precond=net, gmres_m=20)
    say("  plain", rp, "\n  untrained", rep)
    assert rp["converged"] and rep["converged"] and rep["residual"] <= 1e-8
    assert rep["fallbacks"] >= 1
    d = (xs - xp).cpu().numpy()
    assert np.sqrt(s.vec_dot(torch_cuda.from_numpy(d), torch_cuda.from_numpy(d))) < 1e-7
