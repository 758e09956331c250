"""Nonlinear term at every supported transform length.

The transform kernels are instantiated per length (L = 3M for theta, L = 3K
for z), each with its own radix split and LDS segment stride.  These grids
reach every length a context accepts: 6 ... 192 in theta (M <= 64) and
6 ... 192 in z (K <= 64).  The nonlinear term is checked against the CPU FP64
oracle in FP64 (1e-13), in mixed precision (FP32 transforms, 1e-5) and with a
transverse Coriolis force.
"""
import numpy as np
import pytest

from inputs import make_state
from gpu_support import make_ensemble, make_solver, oracle_nodes  # noqa: F401

pytestmark = pytest.mark.gpu

# (M, K): theta length 3M, axial length 3K; N = 13 leaves a ragged radial tile
GRIDS = [(2, 12), (12, 2), (18, 36), (36, 18), (48, 3), (3, 64), (4, 16), (16, 4),
         (24, 48), (48, 24), (32, 6), (6, 32), (8, 8), (64, 4)]
AXIAL = {6, 9, 12, 18, 24, 36, 48, 54, 72, 96, 108, 144, 192}
THETA = AXIAL
ROT = (0.3, -0.2, 0.1)


def say(*a):
    print(*a, flush=True)


def rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def test_grids_reach_every_length():
    theta = {3 * m for m, _ in GRIDS}
    axial = {3 * k for _, k in GRIDS}
    assert theta == THETA and axial == AXIAL


@pytest.mark.parametrize("M,K", GRIDS)
def test_nonlinear_every_length(torch_cuda, M, K):
    import paper_1705_03838_amd as opf
    from oracle import Oracle, Params
    kw = dict(N=13, M=M, K=K, mp=1, alpha=1.3, Re=2000.0, dt=0.01)
    say("nonlinear at lengths", 3 * M, 3 * K, kw)
    s = make_solver(**kw)
    r = s.nodes()
    u = make_state(13, M, K, 1, 1.3, r, 5e-2, 4.0, 4.0, 7 + M + K)
    ud = torch_cuda.from_numpy(u)
    ref = Oracle(Params(r=r, **kw)).nonlinear(u)
    assert rel(s.nonlinear(ud).cpu().numpy(), ref) < 1e-13
    m = make_solver(precision=opf.OPF_MIXED, **kw)
    assert rel(m.nonlinear(ud).cpu().numpy(), ref) < 1e-5
    s.set_rotation(*ROT)
    ref_rot = Oracle(Params(r=r, rotation=ROT, **kw)).nonlinear(u)
    assert rel(s.nonlinear(ud).cpu().numpy(), ref_rot) < 1e-13
