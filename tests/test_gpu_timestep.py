"""GPU parity of automatic time-step control: opf_set_dt against a context
created at the new dt (bitwise), the last correction ||u^{n+1} - u^p||
against the oracle (tiny, ragged and full pipe64 sizes), and whole adaptive
runs against the oracle's run_adaptive (same step-size sequence, same state).

Tolerances: the correction is a difference of two states that agree to
O(dt^2), so the ~1e-13 rounding of each enters relative to delta; 1e-6
relative covers it.  Step sizes come from delta and the CFL number in FP64 on
both sides and agree to 1e-10 relative; states after runs to 1e-10."""
import numpy as np
import pytest

from inputs import WORKLOADS, laminar_state, make_state, workload_state
from gpu_support import make_ensemble, make_solver, oracle_nodes  # noqa: F401

pytestmark = pytest.mark.gpu

CASES = {
    "small": dict(N=16, M=4, K=4, mp=1, alpha=1.25, Re=2400.0, dt=0.01),
    "ragged": dict(N=21, M=6, K=4, mp=2, alpha=0.9, Re=1500.0, dt=0.007),
}


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def solver(**kw):
    import paper_1705_03838_amd as opf
    return make_solver(**kw)


def oracle_for(s, **kw):
    from oracle import Oracle, Params
    return Oracle(Params(**kw))


def state_for(kw, r, energy=1e-2, seed=11):
    return make_state(kw["N"], kw["M"], kw["K"], kw["mp"], kw["alpha"], r, energy, 3.0, 3.0, seed)


def test_set_dt_equals_fresh_context(torch_cuda):
    """Step counts above 8 run through the captured 8-step graph as well as
    single-step graphs: a dt change must drop both."""
    kw = CASES["ragged"]
    say("set_dt vs fresh context", kw)
    a = solver(**kw)
    u = state_for(kw, a.nodes())
    a.set_state(torch_cuda.from_numpy(u))
    a.step(11)
    a.set_dt(0.004)
    a.step(12)
    got = a.get_state().cpu().numpy()
    b = solver(**kw)
    b.set_state(torch_cuda.from_numpy(u))
    b.step(11)
    c = solver(**dict(kw, dt=0.004))
    c.set_state(b.get_state())
    c.step(12)
    assert np.array_equal(got, c.get_state().cpu().numpy())
    # and back: the original tables are rebuilt bit for bit
    a.set_dt(kw["dt"])
    a.set_state(torch_cuda.from_numpy(u))
    a.step(10)
    b.set_state(torch_cuda.from_numpy(u))
    b.step(10)
    assert np.array_equal(a.get_state().cpu().numpy(), b.get_state().cpu().numpy())


@pytest.mark.parametrize("case", list(CASES))
def test_pc_difference_matches_oracle(torch_cuda, case):
    import paper_1705_03838_amd as opf
    from oracle.timestep import pc_difference
    kw = CASES[case]
    say("pc difference", case, kw)
    s = solver(**kw)
    o = oracle_for(s, **kw)
    u = state_for(kw, s.nodes())
    s.set_state(torch_cuda.from_numpy(u))
    with pytest.raises(opf.OpfError):
        s.pc_difference()  # no step since the state was set
    s.step(1)
    d = s.pc_difference()
    u1, up = o.step_pc(u)
    ref = pc_difference(o, u1, up)
    say(f"  delta {d:.6e} oracle {ref:.6e}")
    assert abs(d - ref) <= 1e-6 * ref
    # mixed precision: the FP32 predictor adds its rounding to delta
    m = solver(precision=opf.OPF_MIXED, **kw)
    m.set_state(torch_cuda.from_numpy(u))
    m.step(1)
    assert abs(m.pc_difference() - ref) <= 5e-2 * ref


def test_pc_difference_vanishes_for_axisymmetric_state(torch_cuda):
    kw = CASES["small"]
    s = solver(**kw)
    r = s.nodes()
    u = laminar_state(16, 4, 4, r)
    u[1, 0, 3] = 0.3 * r * (1 - r ** 2)
    u[2, 0, 3] += 0.2 * (1 - r ** 2) ** 2
    s.set_state(torch_cuda.from_numpy(u))
    s.step(1)
    assert s.pc_difference() <= 1e-14


def test_pipe64_pc_difference(torch_cuda):
    """Full-size workload (N=64, |m| < 48, |k| < 64) in the benchmark's
    launch configuration: delta of one graph step against the oracle's."""
    from oracle.timestep import pc_difference
    w = WORKLOADS["pipe64"]
    kw = {k: w[k] for k in ("N", "M", "K", "mp", "alpha", "Re", "dt")}
    say("pipe64 pc difference", kw)
    s = solver(**kw)
    o = oracle_for(s, **kw)
    u = workload_state(w, s.nodes())
    s.set_state(torch_cuda.from_numpy(u))
    s.step(1)
    d = s.pc_difference()
    u1, up = o.step_pc(u)
    ref = pc_difference(o, u1, up)
    say(f"  delta {d:.6e} oracle {ref:.6e}")
    assert abs(d - ref) <= 1e-6 * ref


@pytest.mark.parametrize("case", list(CASES))
def test_adaptive_run_matches_oracle(torch_cuda, case):
    from dataclasses import replace
    from oracle import Params
    from oracle.timestep import DtControl, run_adaptive
    kw = CASES[case]
    s = solver(**kw)
    u = state_for(kw, s.nodes())
    # corrector limit below the first step's delta, so dt shrinks once
    s.set_state(torch_cuda.from_numpy(u))
    s.step(1)
    tol = 0.2 * s.pc_difference()
    ctl = DtControl(courant=0.5, pc_tol=tol, dt_min=1e-5, dt_max=0.05, grow=0.1, check_every=3)
    say("adaptive run", case, kw, "tol", tol)
    s.set_state(torch_cuda.from_numpy(u))
    rep = s.step_adaptive(12, courant=ctl.courant, pc_tol=ctl.pc_tol, dt_min=ctl.dt_min, dt_max=ctl.dt_max,
                          grow=ctl.grow, check_every=ctl.check_every, trace=True)
    ref_u, dts, info = run_adaptive(Params(**kw), u, 12, ctl)
    say(f"  dts {rep['dts']}")
    assert rep["changes"] == info["changes"] >= 1
    assert np.allclose(rep["dts"], dts, rtol=1e-10, atol=0)
    assert abs(rep["t"] - info["t"]) <= 1e-10 * info["t"]
    assert abs(rep["pc_diff"] - info["delta"]) <= 1e-6 * info["delta"]
    assert abs(rep["cfl"] - info["cfl"]) <= 1e-10 * info["cfl"]
    got = s.get_state().cpu().numpy()
    assert np.max(np.abs(got - ref_u)) <= 1e-10 * np.max(np.abs(ref_u))


def test_laminar_flow_settles_at_courant_step(torch_cuda):
    kw = dict(CASES["small"], dt=0.001)
    s = solver(**kw)
    r = s.nodes()
    u = laminar_state(16, 4, 4, r)
    s.set_state(torch_cuda.from_numpy(u))
    rep = s.step_adaptive(8, courant=0.5, pc_tol=1e-8, dt_max=1.0, grow=0.1, check_every=2, trace=True)
    star = 0.5 * (2 * np.pi / (1.25 * 12)) / ((1 - r[0] ** 2) * 1.1)
    assert rep["dts"][:2] == [0.001, 0.001]
    assert np.allclose(rep["dts"][2:], star, rtol=1e-12, atol=0)
    assert rep["changes"] == 1
    assert np.max(np.abs(s.get_state().cpu().numpy() - u)) <= 1e-13


def test_control_arguments_checked(torch_cuda):
    import paper_1705_03838_amd as opf
    kw = CASES["small"]
    s = solver(**kw)
    s.set_state(torch_cuda.from_numpy(state_for(kw, s.nodes())))
    for bad in (dict(courant=0.0), dict(pc_tol=-1.0), dict(dt_min=0.0), dict(dt_max=1e-7, dt_min=1e-6),
                dict(grow=-0.1), dict(check_every=0), dict(dt_max=0.005)):
        with pytest.raises(opf.OpfError):
            s.step_adaptive(2, **bad)
    with pytest.raises(opf.OpfError):
        s.set_dt(0.0)
    # a limit the step cannot meet is a numeric error, with the state advanced
    with pytest.raises(opf.OpfError):
        s.step_adaptive(2, courant=1e-9, dt_min=1e-6, check_every=1)
