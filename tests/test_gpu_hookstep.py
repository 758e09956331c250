"""GPU parity of the Newton-Krylov hookstep (opf_nk_solve with hookstep)
against the oracle's newton_hook_pipe on the same near-laminar guess
(N=12, |m|, |k| < 3, Re 400, dt 0.04, T = 2, shift 0.1).

Tolerance: Jacobian products are forward differences with step
eps = 1e-7 max(||x||, 1), so the ~1e-13 relative difference between the
device and oracle residuals becomes ~1e-6 in each product and, through the
small least-squares problem, up to ~1e-5 in the step; 1e-4 relative to the
step length covers it.  Counts (products, tries) must be equal."""
import numpy as np
import pytest

from inputs import laminar_state, make_state
from gpu_support import make_ensemble, make_solver, oracle_nodes  # noqa: F401

pytestmark = pytest.mark.gpu

KW = dict(N=12, M=3, K=3, mp=1, alpha=1.25, Re=400.0, dt=0.04)
T, SHIFT = 2.0, 0.1


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def setup():
    import torch

    import paper_1705_03838_amd as opf
    from oracle import Oracle, Params
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    s = make_solver(**KW)
    o = Oracle(Params(**KW))
    x = make_state(12, 3, 3, 1, 1.25, s.nodes(), 1e-3, 3.0, 3.0, 7)
    return torch, opf, s, o, x


def test_first_hookstep_matches_oracle(setup):
    from oracle.hookstep import newton_hook_pipe
    torch, opf, s, o, x = setup
    say("first hookstep", KW)
    xg, rep = s.nk_solve(torch.from_numpy(x), T, SHIFT / T, gmres_m=12, max_newton=1, tol=1e-12, gmres_tol=1e-3,
                         hookstep=True, tr_delta0=0.01)
    xo, hist, info = newton_hook_pipe(o, x, T, SHIFT, tol=1e-12, m=12, max_newton=1, gmres_tol=1e-3,
                                      delta0=0.01)
    say("  ", rep)
    assert info["mus"][0] > 0  # the radius binds
    assert rep["gmres_iterations"] == info["products"] and rep["hook_trials"] == info["trials"]
    step = np.linalg.norm(xo - x)
    assert np.linalg.norm(xg.cpu().numpy() - xo) <= 1e-4 * step
    assert abs(rep["history"][1] - hist[1]) <= 1e-4 * hist[1]
    assert abs(rep["tr_delta"] - info["deltas"][0]) <= 1e-4 * info["deltas"][0]


def test_hookstep_reaches_laminar_flow(setup):
    from oracle.hookstep import newton_hook_pipe
    torch, opf, s, o, x = setup
    say("hookstep to laminar", KW)
    xg, rep = s.nk_solve(torch.from_numpy(x), T, SHIFT / T, gmres_m=12, tol=1e-8, gmres_tol=1e-3, hookstep=True,
                         tr_delta0=0.01)
    say("  ", rep)
    _, hist, info = newton_hook_pipe(o, x, T, SHIFT, tol=1e-8, m=12, gmres_tol=1e-3, delta0=0.01)
    assert rep["converged"] and not rep["stalled"]
    assert abs(rep["newton_iterations"] - (len(hist) - 1)) <= 1
    lam = laminar_state(12, 3, 3, s.nodes())
    assert np.max(np.abs(xg.cpu().numpy() - lam)) <= 1e-7
    assert rep["residual_evals"] == 1 + rep["hook_trials"]


def test_hookstep_not_combined_with_preconditioner(setup):
    torch, opf, s, o, x = setup
    net = opf.Mlp(s, width=32, layers=1, rank=1, seed=1)
    with pytest.raises(opf.OpfError):
        s.nk_solve(torch.from_numpy(x), T, SHIFT / T, gmres_m=4, max_newton=1, precond=net, hookstep=True)
    net.close()
