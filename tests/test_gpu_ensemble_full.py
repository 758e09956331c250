"""The benchmark's ensemble at full size (96 members in three classes:
N=32 |m|<16 |k|<24, N=48 |m|<24 |k|<32, N=64 |m|<32 |k|<48; mixed
precision; autotuned tiles, one graph launch per step): after 3 ensemble
steps, one sampled member of each class against the FP64 oracle.

Tolerance: mixed precision (FP32 transforms and products, FP64 solves)
against the FP64 oracle, 1e-5 relative as for the single-trajectory mixed
path."""
import numpy as np
import pytest

from inputs import ensemble_members, make_state
from gpu_support import make_ensemble, make_solver, oracle_nodes  # noqa: F401

pytestmark = pytest.mark.gpu


def test_bench_ensemble_sampled_members_match_oracle():
    import torch

    import paper_1705_03838_amd as opf
    from oracle import Oracle, Params
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    mem = ensemble_members()
    kws = [dict(N=m["N"], M=m["M"], K=m["K"], mp=m["mp"], alpha=m["alpha"], Re=m["Re"], dt=m["dt"],
                precision=opf.OPF_MIXED) for m in mem]
    e = make_ensemble(kws)
    states = [make_state(m["N"], m["M"], m["K"], m["mp"], m["alpha"], oracle_nodes(m["N"]), m["energy_frac"],
                         m["decay_m"], m["decay_k"], m["seed"], axis_power=1) for i, m in enumerate(mem)]
    for i, st in enumerate(states):
        e.members[i].set_state(torch.from_numpy(st))
    e.tune(2)
    for i, st in enumerate(states):
        e.members[i].set_state(torch.from_numpy(st))
    e.step(3)
    for i in (5, 40, 95):  # one member of each class
        m = mem[i]
        print("member", i, m["N"], m["M"], m["K"], flush=True)
        o = Oracle(Params(N=m["N"], M=m["M"], K=m["K"], mp=m["mp"], alpha=m["alpha"], Re=m["Re"], dt=m["dt"]))
        ref = o.run(states[i], 3)
        got = e.members[i].get_state().cpu().numpy()
        err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
        print("  rel err", err, flush=True)
        assert err < 1e-5
    e.close()
