"""GPU parity of the prescribed wall velocity (opf_set_wall_velocity): the
rotating-pipe steady state and Bessel-mode spin-up (closed forms), general
wall motion against the oracle (tiny, ragged with mp = 2, full-size pipe64)
and the boundary residual g_norm measured against the wall velocity.

Tolerances as for the no-slip path: 1e-11 relative per step in FP64 (5e-11
over 5 steps), 1e-5 in mixed precision."""
import numpy as np
import pytest
from scipy.special import j1, jn_zeros

from inputs import WORKLOADS, laminar_state, make_state, workload_state
from gpu_support import make_ensemble, make_solver, oracle_nodes  # noqa: F401

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def rotation_wall(M, K, V):
    b = np.zeros((3, M, 2 * K - 1), dtype=complex)
    b[1, 0, K - 1] = V
    return b


def random_wall(M, K, seed, scale=1e-3):
    """Tangential wall motion of size `scale` per mode and wall-normal
    (blowing / suction) a tenth of it: larger wall-normal velocities next to
    the fine wall spacing exceed the explicit advection limit (CFL > 1)."""
    rng = np.random.default_rng(seed)
    b = scale * (rng.standard_normal((3, M, 2 * K - 1)) + 1j * rng.standard_normal((3, M, 2 * K - 1)))
    b[:, 0, :K - 1] = np.conj(b[:, 0, K:][:, ::-1])
    b[:, 0, K - 1] = b[:, 0, K - 1].real
    b[0] *= 0.1
    b[0, 0, K - 1] = 0.0
    return b


def test_rotating_pipe_steady_and_spin_up(torch_cuda):
    import paper_1705_03838_amd as opf
    N, M, K, V = 32, 2, 2, 0.5
    kw = dict(N=N, M=M, K=K, alpha=1.25, Re=100.0, dt=0.01)
    say("rotating pipe", kw)
    s = make_solver(**kw)
    s.set_wall_velocity(rotation_wall(M, K, V))
    r = s.nodes()
    u = laminar_state(N, M, K, r)
    u[1, 0, K - 1] = V * r
    s.set_state(torch_cuda.from_numpy(u))
    s.step(5)
    assert np.max(np.abs(s.get_state().cpu().numpy() - u)) <= 1e-13
    ja, jb = jn_zeros(1, 2)
    u[1, 0, K - 1] = V * r - 0.2 * j1(ja * r) + 0.07 * j1(jb * r)
    s.set_state(torch_cuda.from_numpy(u))
    s.step(300)
    t = 3.0
    expect = V * r - 0.2 * j1(ja * r) * np.exp(-ja ** 2 * t / 100.0) + 0.07 * j1(jb * r) * np.exp(-jb ** 2 * t / 100.0)
    got = s.get_state().cpu().numpy()[1, 0, K - 1]
    assert np.max(np.abs(got.real - expect)) <= 2e-7
    d = s.diagnostics()
    assert d["g_norm"] <= 1e-14


@pytest.mark.parametrize("case", ["tiny", "ragged"])
def test_general_wall_motion_matches_oracle(torch_cuda, case):
    import paper_1705_03838_amd as opf
    from oracle import Oracle, Params
    kw = {"tiny": dict(N=24, M=8, K=8, mp=1, alpha=1.25, Re=2400.0, dt=0.01),
          "ragged": dict(N=21, M=6, K=4, mp=2, alpha=0.9, Re=1500.0, dt=0.007)}[case]
    say("wall motion", case, kw)
    b = random_wall(kw["M"], kw["K"], 9)
    s = make_solver(**kw)
    s.set_wall_velocity(b)
    o = Oracle(Params(wall=b, **kw))
    u = make_state(kw["N"], kw["M"], kw["K"], kw["mp"], kw["alpha"], s.nodes(), 1e-2, 4.0, 4.0, 43)
    s.set_state(torch_cuda.from_numpy(u))
    s.step(5)
    ref = o.run(u, 5)
    got = s.get_state().cpu().numpy()
    assert np.max(np.abs(ref)) < 2.0 and o.cfl(ref) < 1.0  # a stable run
    assert rel(got, ref) < 5e-11
    assert np.max(np.abs(got[:, :, :, -1] - b)) <= 1e-13
    d = s.diagnostics()
    g, dm = o.boundary_and_divergence(ref)
    assert d["g_norm"] <= 1e-13 and g <= 1e-13
    assert abs(d["div_max"] - dm) <= 1e-9 * max(dm, 1e-12)
    m = make_solver(precision=opf.OPF_MIXED, **kw)
    m.set_wall_velocity(b)
    m.set_state(torch_cuda.from_numpy(u))
    m.step(5)
    assert rel(m.get_state().cpu().numpy(), ref) < 1e-5


def test_pipe64_step_with_moving_wall(torch_cuda):
    """Full-size grid (N=64, |m| < 48, |k| < 64), bench launch configuration."""
    import paper_1705_03838_amd as opf
    from oracle import Oracle, Params
    w = WORKLOADS["pipe64"]
    kw = {k: w[k] for k in ("N", "M", "K", "mp", "alpha", "Re", "dt")}
    b = random_wall(w["M"], w["K"], 10, scale=1e-3)
    b[1, 0, w["K"] - 1] = 0.05
    say("pipe64 wall step")
    s = make_solver(**kw)
    s.set_wall_velocity(b)
    o = Oracle(Params(wall=b, **kw))
    u = workload_state(w, s.nodes())
    s.set_state(torch_cuda.from_numpy(u))
    s.step(1)
    assert rel(s.get_state().cpu().numpy(), o.step(u)) < 1e-11


def test_wall_arguments(torch_cuda):
    import paper_1705_03838_amd as opf
    kw = dict(N=16, M=3, K=3, alpha=1.25, Re=500.0, dt=0.01)
    s = make_solver(**kw)
    b = np.zeros((3, 3, 5), dtype=complex)
    b[0, 0, 2] = 0.1  # net radial flux through the wall
    with pytest.raises(opf.OpfError):
        s.set_wall_velocity(b)
    s.set_wall_velocity(rotation_wall(3, 3, 0.3))
    s.set_wall_velocity(None)  # back to no slip: laminar flow is steady again
    lam = laminar_state(16, 3, 3, s.nodes())
    s.set_state(torch_cuda.from_numpy(lam))
    s.step(3)
    assert np.max(np.abs(s.get_state().cpu().numpy() - lam)) <= 1e-13
