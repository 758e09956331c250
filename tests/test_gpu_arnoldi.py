"""GPU parity of the Arnoldi stability solver (opf_arnoldi) against the
oracle's arnoldi on the same state and start vector.

Linear (Stokes) case: the time map is affine, so forward-difference
products differ from the oracle's only by rounding amplified by 1/eps
(~1e-9); the Hessenberg matrices agree to 1e-7 and the Ritz values to the
Bessel-derived multipliers to 1e-8.  Nonlinear case (laminar state at Re
1000): the products carry the ~1e-13 residual difference divided by eps,
~1e-6, so the leading Ritz values are held to 1e-5."""
import os

import numpy as np
import pytest

from inputs import laminar_state, make_state
from gpu_support import make_ensemble, make_solver, oracle_nodes  # noqa: F401

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "stokes_modes.txt")


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def golden(family, m, kappa):
    with open(GOLDEN) as f:
        for line in f:
            if line.startswith("#"):
                continue
            fam, mm, ka, n, mu, lre = line.split()
            if fam == family and int(mm) == m and abs(float(ka) - kappa) < 1e-9 and int(n) == 1:
                return float(lre), float(mu)
    raise KeyError(family)


def test_stokes_multipliers(torch_cuda):
    import paper_1705_03838_amd as opf
    from oracle import Oracle, Params
    from oracle.arnoldi import arnoldi
    Re, dt, T, alpha = 50.0, 0.01, 2.0, 1.25
    kw = dict(N=24, M=3, K=2, alpha=alpha, Re=Re, dt=dt, nonlinear=0)
    say("arnoldi stokes", kw)
    s = make_solver(**kw)
    x = laminar_state(24, 3, 2, s.nodes())
    v0 = make_state(24, 3, 2, 1, alpha, s.nodes(), 1e-2, 3.0, 3.0, 21, laminar=False)
    ev, rep = s.arnoldi(torch_cuda.from_numpy(x), T, 0.0, torch_cuda.from_numpy(v0), m=40, nev=3, tol=1e-8)
    say("  ", ev, rep["products"])
    n = int(round(T / dt))

    def mult(lre):
        lam = lre / Re
        return ((1 - 0.5 * lam * dt) / (1 + 0.5 * lam * dt)) ** n

    gen, _ = golden("general", 1, 1.25)
    swirl, j11 = golden("swirl", 0, 0.0)
    assert rep["converged"]
    assert np.allclose(ev.real, [mult(gen), mult(swirl), mult(j11 ** 2 + alpha ** 2)], rtol=1e-8, atol=0)
    o = Oracle(Params(N=24, M=3, K=2, alpha=alpha, Re=Re, dt=dt, nonlinear=False))
    evo, k, conv = arnoldi(o, x, T, 0.0, v0, 40, 3, tol=1e-8, check_every=5)
    assert k == rep["products"]
    assert np.allclose(ev, evo, rtol=1e-9, atol=0)


def test_nonlinear_multipliers_match_oracle(torch_cuda):
    import paper_1705_03838_amd as opf
    from oracle import Oracle, Params
    from oracle.arnoldi import arnoldi
    kw = dict(N=16, M=4, K=4, alpha=1.25, Re=1000.0, dt=0.02)
    T, shift = 1.0, 0.3
    say("arnoldi nonlinear", kw)
    s = make_solver(**kw)
    x = laminar_state(16, 4, 4, s.nodes())
    v0 = make_state(16, 4, 4, 1, 1.25, s.nodes(), 1e-2, 3.0, 3.0, 22, laminar=False)
    ev, rep = s.arnoldi(torch_cuda.from_numpy(x), T, shift, torch_cuda.from_numpy(v0), m=30, nev=4, tol=1e-6,
                        check_every=5)
    o = Oracle(Params(**kw))
    evo, k, conv = arnoldi(o, x, T, shift, v0, 30, 4, tol=1e-6, check_every=5)
    say("  gpu", ev, rep["products"], "oracle", evo, k)
    Hg = rep["hessenberg"]
    assert Hg.shape[1] >= 5
    assert np.all(np.abs(ev) < 1.0)  # laminar flow at Re 1000 is linearly stable
    assert np.allclose(ev[:2], evo[:2], rtol=1e-5, atol=0)
