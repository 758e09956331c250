"""Tile shapes of the batched step on the GPU: every admissible transform
and solve tile gives members bitwise equal to single runs (the tiles decide
only the speed); the offline autotuner writes a tile cache that an ensemble
created from it adopts; the ensemble tuner times candidates of all three
tile dimensions."""
import json

import numpy as np
import pytest

from inputs import make_state
from gpu_support import make_ensemble, make_solver, oracle_nodes

pytestmark = pytest.mark.gpu

MEM = [dict(N=24, M=8, K=8, alpha=1.1, Re=1900.0, dt=0.01),
       dict(N=24, M=8, K=8, alpha=1.5, Re=2500.0, dt=0.008),
       dict(N=21, M=6, K=4, mp=2, alpha=0.9, Re=1500.0, dt=0.007, precision=1)]


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def full(kw):
    return dict(dict(mp=1, precision=0), **kw)


@pytest.mark.parametrize("tiles", [(1, 2, 4), (2, 8, 16), (4, 4, 8)])
def test_members_equal_single_runs_for_every_tile(torch_cuda, tmp_path, tiles):
    gm, tz, zt = tiles
    entries = []
    for kw in MEM[::2]:
        f = full(kw)
        entries.append(dict(N=f["N"], M=f["M"], K=f["K"], mp=f["mp"], precision=f["precision"],
                            gm=min(gm, 2 if f["mp"] == 2 else 4), tz=tz, ztile=zt))
    import paper_1705_03838_amd as opf
    path = str(tmp_path / "tiles.json")
    opf.tile_cache_write(entries, path)
    say("tiles", entries)
    e = make_ensemble(MEM, tune_cache=path)
    got = e.tiles()
    for g, want in zip(got, entries):
        assert (g["gm"], g["tz"], g["ztile"]) == (want["gm"], want["tz"], want["ztile"]), (g, want)
    states = []
    for i, kw in enumerate(MEM):
        f = full(kw)
        st = make_state(f["N"], f["M"], f["K"], f["mp"], f["alpha"], oracle_nodes(f["N"]), 1e-2, 4.0, 4.0, 50 + i)
        states.append(st)
        e.members[i].set_state(torch_cuda.from_numpy(st))
    e.step(3)
    for i, kw in enumerate(MEM):
        s = make_solver(**kw)
        s.set_state(torch_cuda.from_numpy(states[i]))
        s.step(3)
        assert np.array_equal(e.members[i].get_state().cpu().numpy(), s.get_state().cpu().numpy()), i
    e.close()


def test_autotune_cache_is_adopted(torch_cuda, tmp_path):
    import paper_1705_03838_amd as opf
    path = str(tmp_path / "auto.json")
    classes = [dict(N=24, M=8, K=8, alpha=1.2, Re=2000.0, dt=0.01),
               dict(N=32, M=16, K=24, alpha=1.0, Re=2200.0, dt=0.01, precision=opf.OPF_MIXED)]
    opf.autotune(classes, path)
    cache = json.load(open(path))
    say(json.dumps(cache)[:600])
    assert len(cache["classes"]) == 2
    dims = set()
    for c in cache["classes"]:
        cands = c["candidates"]
        assert len(cands) >= 5 and min(x["us_per_step"] for x in cands) == pytest.approx(c["us_per_step"], rel=1e-3)
        for x in cands:
            dims.update((("gm", x["gm"]), ("tz", x["tz"]), ("ztile", x["ztile"])))
    assert {("tz", 2), ("tz", 4), ("ztile", 4), ("ztile", 8), ("gm", 1), ("gm", 4)} <= dims
    e = make_ensemble([classes[0], classes[1], classes[0]], tune_cache=path)
    for g, c in zip(e.tiles(), cache["classes"]):
        assert (g["N"], g["gm"], g["tz"], g["ztile"]) == (c["N"], c["gm"], c["tz"], c["ztile"])
    e.close()


def test_ensemble_tune_without_states_leaves_no_state(torch_cuda):
    import paper_1705_03838_amd as opf
    e = make_ensemble(MEM)
    rep = e.tune(2)
    assert len(rep["classes"]) == 2
    for c in rep["classes"]:
        assert all(np.isfinite(x["us_per_step"]) for x in c["candidates"])
    with pytest.raises(opf.OpfError):  # tuning ran on laminar flow; members still need a state
        e.step(1)
    e.close()
