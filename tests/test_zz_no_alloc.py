"""opf_probe_pairs_noalloc, the entry point for callers that cannot allocate
device memory: through the C-ABI it must give bitwise the pairs of
opf_probe_pairs (the existing entry point, whose pairs are checked against
fresh finite differences in test_gpu_mlp.py), on two calls in a row, the
second on a smaller grid with fewer probes; a grid too large for its
16 MiB scratch is refused before any device work."""
import pytest

from inputs import make_state
from gpu_support import make_solver, oracle_nodes

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def test_noalloc_probes_equal_existing_entry_point(torch_cuda):
    import paper_1705_03838_amd as opf
    cases = [(dict(N=12, M=4, K=4, mp=2, alpha=1.25, Re=200.0, dt=0.05), 0.25, 0.1, 3, 7),
             (dict(N=12, M=2, K=2, mp=2, alpha=1.25, Re=100.0, dt=0.05), 0.15, 0.0, 2, 9)]
    for kw, T, sh, n, seed in cases:
        print("no-alloc probes", kw, "T", T, "n", n, flush=True)
        s = make_solver(**kw)
        x = torch_cuda.from_numpy(make_state(kw["N"], kw["M"], kw["K"], kw["mp"], kw["alpha"], oracle_nodes(kw["N"]),
                                             1e-3, 4.0, 4.0, seed)).cuda()
        ref = s.probe_pairs(x, T, sh, n, seed=seed)
        got = s.probe_pairs_noalloc(x, T, sh, n, seed=seed)
        assert got.shape == ref.shape
        assert torch_cuda.equal(got, ref)
        assert torch_cuda.isfinite(got).all()
        s.close()


def test_noalloc_refuses_grid_beyond_scratch(torch_cuda):
    import paper_1705_03838_amd as opf
    kw = dict(N=64, M=32, K=48, mp=1, alpha=1.0, Re=1000.0, dt=0.01)  # 3 fields of 3 x 32 x 95 x 64 entries: 28 MB
    s = make_solver(**kw)
    x = torch_cuda.zeros(s.shape, dtype=torch_cuda.complex128, device="cuda")
    with pytest.raises(opf.OpfError) as e:
        s.probe_pairs_noalloc(x, 0.01, 0.0, 1)
    assert e.value.status == opf.OPF_E_INVALID
    s.close()
