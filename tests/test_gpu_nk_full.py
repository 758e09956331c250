"""The travelling-wave residual F(x) = shift(Phi_T(x), -s) - x and the energy
inner product at the full Newton-Krylov grid of the benchmark (N=48,
|m| < 24 with mp = 2, |k| < 32, Re 2400, alpha 1.25, dt 0.01) against the
oracle, with a short period (T = 0.05, five steps) so the oracle finishes in
seconds; same tolerances as the small cases (1e-10, 1e-13)."""
import numpy as np
import pytest

from inputs import WORKLOADS, workload_state
from gpu_support import make_ensemble, make_solver, oracle_nodes  # noqa: F401

pytestmark = pytest.mark.gpu


def test_nk_grid_residual_matches_oracle():
    import torch

    import paper_1705_03838_amd as opf
    from oracle import Oracle, Params
    from oracle.newton import inner, residual
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    w = WORKLOADS["nk"]
    kw = {k: w[k] for k in ("N", "M", "K", "mp", "alpha", "Re", "dt")}
    s = make_solver(**kw)
    o = Oracle(Params(**kw))
    x = workload_state(w, s.nodes())
    x2 = workload_state(dict(w, seed=w["seed"] + 7, energy_frac=1e-2), s.nodes())
    d = s.vec_dot(torch.from_numpy(x), torch.from_numpy(x2))
    assert abs(d - inner(o, x, x2)) <= 1e-13 * inner(o, x, x)
    T, sh = 0.05, 0.3
    F, nrm = s.newton_residual(torch.from_numpy(x2), T, sh)
    ref = residual(o, x2, T, sh)
    err = np.max(np.abs(F.cpu().numpy() - ref)) / np.max(np.abs(ref))
    print("nk grid residual rel err", err, flush=True)
    assert err < 1e-10
    assert abs(nrm - np.sqrt(inner(o, ref, ref))) <= 1e-9 * nrm
