"""Properties of the GPU step at the full pipe64 size (N=64, |m|<48, |k|<64),
where the CPU oracle would be slow: the graph-launched step equals the same
kernels launched one by one, the step commutes with axial shifts and
azimuthal rotations (Section 2: Fourier directions z and theta are
homogeneous), the energy budget dE/dt = I - D (Section 3.2's E, I, D) closes
at second order in dt, and a non-finite state is reported, not hidden.

Tolerances: equivariance is exact in exact arithmetic; the shifted and
unshifted states differ in their rounding, which after one step is a few
units of 1e-16 relative to the largest coefficient (laminar u_z ~ 1), so
1e-12 leaves a wide margin.  The energy budget's error (E^{n+1} - E^n)/dt -
(I^{n+1/2} - (D^n + D^{n+1})/2) falls as dt^2 until the finite-difference
floor; halving dt must cut it by more than 3 (4 for a clean second order),
as in the oracle's own pin of the same identity.
"""
import numpy as np
import pytest

from inputs import WORKLOADS, workload_state
from gpu_support import make_solver, oracle_nodes

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def pipe64(**over):
    w = dict(WORKLOADS["pipe64"], **over)
    kw = {k: w[k] for k in ("N", "M", "K", "mp", "alpha", "Re", "dt")}
    return w, kw


@pytest.mark.parametrize("nsteps", [5, 21])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_graph_step_equals_kernel_by_kernel_launches(torch_cuda, precision, nsteps):
    """opf_step replays captured graphs (one of 8 steps, then one step at a
    time: 21 = 2 x 8 + 5 uses both); opf_profile_steps launches the same
    kernels one by one with timing events.  From the same state both must
    give bitwise the same state."""
    import paper_1705_03838_amd as opf
    w, kw = pipe64()
    prec = opf.OPF_MIXED if precision == "mixed" else opf.OPF_FP64
    say("graph vs kernel-by-kernel, pipe64", precision, nsteps, "steps")
    s = make_solver(precision=prec, **kw)
    u = torch_cuda.from_numpy(workload_state(w, oracle_nodes(kw["N"])))
    s.set_state(u)
    s.step(nsteps)
    a = s.get_state().clone()
    s.set_state(u)
    s.profile_steps(nsteps)
    b = s.get_state()
    assert torch_cuda.equal(a, b)
    s.close()


def test_shift_and_rotation_equivariance_pipe64(torch_cuda):
    w, kw = pipe64()
    say("shift / rotation equivariance, pipe64")
    s = make_solver(**kw)
    u = workload_state(w, oracle_nodes(kw["N"]))
    ks = np.arange(-(kw["K"] - 1), kw["K"])
    ms = np.arange(kw["M"])
    shift = np.exp(1j * kw["alpha"] * ks * 0.37)[None, None, :, None]
    rot = np.exp(1j * kw["mp"] * ms * 0.61)[None, :, None, None]

    def step(x, n=2):
        s.set_state(torch_cuda.from_numpy(np.ascontiguousarray(x)))
        s.step(n)
        return s.get_state().cpu().numpy()

    ref = step(u)
    scale = np.max(np.abs(ref))
    es = np.max(np.abs(step(u * shift) - ref * shift)) / scale
    er = np.max(np.abs(step(u * rot) - ref * rot)) / scale
    say(f"  shift {es:.2e}, rotation {er:.2e}")
    assert es < 1e-12 and er < 1e-12
    s.close()


def test_energy_budget_second_order_pipe64(torch_cuda):
    """From the workload state advanced to t = 0.02, one more step at dt,
    dt/2, dt/4 (dt = 0.005): the budget error relative to D falls by more
    than 3 per halving (the first step of each run, which projects the
    synthetic state onto the discrete divergence constraint, is excluded by
    the warm-up)."""
    errs = []
    for dt in (0.005, 0.0025, 0.00125):
        w, kw = pipe64(dt=dt)
        s = make_solver(**kw)
        s.set_state(torch_cuda.from_numpy(workload_state(w, oracle_nodes(kw["N"]))))
        s.step(int(round(0.02 / dt)))
        d0 = s.diagnostics(check=False)
        s.step(1)
        d1 = s.diagnostics(check=False)  # its beta is that of the step just taken
        err = (d1["E"] - d0["E"]) / dt - (d1["I"] - 0.5 * (d0["D"] + d1["D"]))
        errs.append(abs(err) / d1["D"])
        say(f"  dt {dt}: dE/dt {(d1['E'] - d0['E']) / dt:.6e}, I - D {d1['I'] - 0.5 * (d0['D'] + d1['D']):.6e}, "
            f"relative error {errs[-1]:.3e}")
        s.close()
    assert errs[0] / errs[1] > 3.0 and errs[1] / errs[2] > 3.0, errs


def test_non_finite_state_is_reported(torch_cuda):
    """A NaN planted in one coefficient of the state (from the host) spreads
    through the step; diagnostics report it: OPF_E_NUMERIC when checked, the
    status in the dict otherwise."""
    import paper_1705_03838_amd as opf
    w = WORKLOADS["tiny"]
    kw = {k: w[k] for k in ("N", "M", "K", "mp", "alpha", "Re", "dt")}
    s = make_solver(**kw)
    u = workload_state(w, oracle_nodes(kw["N"]))
    u[2, 1, kw["K"], 3] = np.nan
    s.set_state(torch_cuda.from_numpy(u))
    s.step(1)
    d = s.diagnostics(check=False)
    say("  planted NaN: status", d["status"], "E", d["E"])
    assert d["status"] == opf.OPF_E_NUMERIC and not np.isfinite(d["E"])
    with pytest.raises(opf.OpfError) as e:
        s.diagnostics()
    assert e.value.status == opf.OPF_E_NUMERIC
    s.close()
