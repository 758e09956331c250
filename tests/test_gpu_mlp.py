"""GPU parity of the learned preconditioner (matrix-core GEMMs of the
residual MLP, backward pass, Adam, the pair-loss head and the per-mode
low-rank map) against the oracle, and its effect on Newton-Krylov.

Tolerances.  The device rounds every GEMM operand to bfloat16 exactly as the
oracle's bf16 mode does, but accumulates in FP32 where the oracle uses FP64.
The accumulation differs by about K 2^-24 relative (K <= 1536 here, ~1e-4);
where that moves a value across a bfloat16 rounding boundary before the next
product, one element changes by one bfloat16 ulp (2^-8).  With a few percent
of such flips per layer the norm-wise effect stays below ~3e-3, so outputs
and gradients are held to 1e-2 relative (norm-wise) against the bf16 oracle,
while the same outputs differ from the unrounded FP64 oracle by several times
more (which shows that the device really computes in bfloat16).  Adam runs
in FP32 and is held to FP32 rounding.
"""
import numpy as np
import pytest

from inputs import make_state
from gpu_support import make_ensemble, make_solver, oracle_nodes  # noqa: F401

pytestmark = pytest.mark.gpu

GRID = dict(N=21, M=6, K=4, mp=2, alpha=0.9, Re=1500.0, dt=0.007)  # 42 mode rows: ragged tile
RANK = 2


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def make_net(torch_cuda, width=64, layers=3, max_rows=0, seed=7, rank=RANK, **kw):
    import paper_1705_03838_amd as opf
    from oracle.mlp import flatten, init_params, unflatten
    s = make_solver(**GRID)
    net = opf.Mlp(s, width=width, layers=layers, rank=rank, max_rows=max_rows, **kw)
    p = init_params(net.din, width, layers, net.dout, seed=seed)
    rng = np.random.default_rng(seed)
    for k in p:
        if k.startswith("b_"):
            p[k] = 0.1 * rng.standard_normal(p[k].shape)
    p["W_out"] *= 0.5
    flat = flatten(p, layers).astype(np.float32)
    net.set_params(flat)
    p32 = unflatten(flat.astype(np.float64), net.din, width, layers, net.dout)
    return s, net, p32


def nrel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def rows(rng, n, d):
    return (rng.standard_normal((n, d))).astype(np.float32)


def test_forward_matches_bf16_oracle(torch_cuda):
    from oracle.mlp import forward
    s, net, p = make_net(torch_cuda, max_rows=200)
    rng = np.random.default_rng(1)
    for n in (1, 42, 77, 200):  # single row, ragged tiles, full
        say("mlp forward rows", n)
        x = rows(rng, n, net.din)
        y = net.forward(torch_cuda.from_numpy(x)).cpu().numpy().astype(np.float64)
        yb, _ = forward(p, x.astype(np.float64), 3, bf16=True)
        yf, _ = forward(p, x.astype(np.float64), 3, bf16=False)
        e_b, e_f = nrel(y, yb), nrel(y, yf)
        say("   vs bf16 oracle", e_b, "vs fp64 oracle", e_f)
        assert e_b <= 1e-2
        assert e_b <= 0.3 * e_f


def check_grads(g, gref, layers):
    from oracle.mlp import flatten, param_names
    gflat = flatten(gref, layers)
    o = 0
    for k in param_names(layers):
        sz = gref[k].size
        e = nrel(g[o:o + sz].astype(np.float64), gflat[o:o + sz])
        say("   grad", k, e)
        assert e <= 1e-2, k
        o += sz
    assert o == g.size


def test_gradient_matches_bf16_oracle(torch_cuda):
    from oracle.mlp import backward, forward, loss
    s, net, p = make_net(torch_cuda, max_rows=224)  # batch rows (160 padded) < capacity (224)
    rng = np.random.default_rng(2)
    n = 150
    x, t = rows(rng, n, net.din), rows(rng, n, net.dout)
    w = rng.uniform(0.2, 2.0, n).astype(np.float32)
    say("mlp gradient rows", n)
    lg, g = net.gradient(torch_cuda.from_numpy(x), torch_cuda.from_numpy(t), torch_cuda.from_numpy(w))
    x64, t64, w64 = x.astype(np.float64), t.astype(np.float64), w.astype(np.float64)
    y, cache = forward(p, x64, 3, bf16=True)
    gref = backward(p, cache, y, t64, 3, bf16=True, w=w64)
    assert abs(lg - loss(y, t64, w64)) <= 1e-3 * loss(y, t64, w64)
    check_grads(g, gref, 3)


def test_adam_step_and_weight_copies(torch_cuda):
    from oracle.mlp import adam, forward, unflatten
    s, net, p = make_net(torch_cuda, max_rows=64, lr=1e-2)
    rng = np.random.default_rng(3)
    n = 64
    x, t = rows(rng, n, net.din), rows(rng, n, net.dout)
    p0 = net.get_params().astype(np.float64)
    _, g = net.gradient(torch_cuda.from_numpy(x), torch_cuda.from_numpy(t))
    net.train(torch_cuda.from_numpy(x), torch_cuda.from_numpy(t), batch=n, epochs=1)
    p1 = net.get_params().astype(np.float64)
    ref, _, _ = adam(p0, g.astype(np.float64), np.zeros_like(p0), np.zeros_like(p0), 1, lr=1e-2)
    say("adam step max diff", np.max(np.abs(p1 - ref)))
    assert np.max(np.abs(p1 - ref)) <= 1e-6
    # the bfloat16 weight copies follow the update
    y = net.forward(torch_cuda.from_numpy(x)).cpu().numpy().astype(np.float64)
    q = unflatten(p1, net.din, 64, 3, net.dout)
    yb, _ = forward(q, x.astype(np.float64), 3, bf16=True)
    assert nrel(y, yb) <= 1e-2


def field(s, seed, energy=1e-2):
    v = make_state(GRID["N"], GRID["M"], GRID["K"], GRID["mp"], GRID["alpha"], s.nodes(), energy, 3.0, 3.0,
                   seed, laminar=False)
    K = GRID["K"]
    for kk in range(K - 1):  # exactly the spectrum of a real field at m = 0
        v[:, 0, kk] = np.conj(v[:, 0, 2 * (K - 1) - kk])
    v[:, 0, K - 1] = v[:, 0, K - 1].real
    return v


def test_factors_and_precondition_match_oracle(torch_cuda):
    from oracle.mlp import lowrank_apply, precondition
    s, net, p = make_net(torch_cuda)
    F, singular = net.factors()
    assert singular == 0
    v = field(s, 23)
    say("precondition", v.shape)
    z = net.precondition(torch_cuda.from_numpy(v)).cpu().numpy()
    # the low-rank map itself, from the device's own factors: FP64 rounding only
    zf = lowrank_apply(F.astype(np.float64), v, RANK)
    assert np.max(np.abs(z - zf)) <= 1e-12 * np.max(np.abs(zf))
    # network + Woodbury + map against the bf16 oracle
    zb = precondition(p, 3, v, GRID["mp"], GRID["alpha"], RANK, bf16=True)
    assert nrel(z + v, zb + v) <= 1e-2
    K = GRID["K"]
    for kk in range(K - 1):
        assert np.array_equal(z[:, 0, kk], np.conj(z[:, 0, 2 * (K - 1) - kk]))
    assert np.all(z[:, 0, K - 1].imag == 0)
    # a network with zero output layer models J = -I and gives z = -v exactly
    q = net.get_params()
    q[-(net.dout * 64 + net.dout):] = 0.0
    net.set_params(q)
    z0 = net.precondition(torch_cuda.from_numpy(v)).cpu().numpy()
    assert np.array_equal(z0, -v)


@pytest.mark.parametrize("rank", [RANK, 3])
def test_pair_gradient_matches_oracle(torch_cuda, rank):
    """Rank 2 divides the loss head's 256 threads (each thread keeps one
    column's C and G in registers); rank 3 takes the general path."""
    from oracle.mlp import backprop, feature_rows, forward, head
    s, net, p = make_net(torch_cuda, rank=rank)
    pairs = np.stack([np.stack([field(s, 40 + i), field(s, 50 + i)]) for i in range(5)])
    pairs[2, 1, :, 3, 2] = 0.0  # an empty (J z) profile: that mode-pair is skipped
    idx = np.array([3, 0, 2, 2], dtype=np.int32)
    say("pair gradient", pairs.shape, idx)
    lg, g = net.pair_gradient(torch_cuda.from_numpy(pairs), idx)
    # the head on the device's own model rows: FP32 accumulation of the loss only
    X = feature_rows(GRID["M"], GRID["K"], GRID["mp"], GRID["alpha"])
    Fdev = net.forward(torch_cuda.from_numpy(X.astype(np.float32))).cpu().numpy().astype(np.float64)
    Ldev, _ = head(Fdev, pairs[idx], rank)
    say("   loss", lg, Ldev)
    assert abs(lg - Ldev) <= 1e-5 * Ldev
    F, cache = forward(p, X, 3, bf16=True)
    L, dF = head(F.astype(np.float32).astype(np.float64), pairs[idx], rank)
    assert abs(lg - L) <= 1e-2 * L
    gref = backprop(p, cache, dF, 3, bf16=True)
    check_grads(g, gref, 3)


def test_probe_pairs_are_jacobian_products(torch_cuda):
    import paper_1705_03838_amd as opf
    from inputs import laminar_state
    kw = dict(N=12, M=2, K=2, mp=2, alpha=1.25, Re=100.0, dt=0.05)
    say("probe pairs", kw)
    s = make_solver(**kw)
    x = torch_cuda.from_numpy(make_state(12, 2, 2, 2, 1.25, s.nodes(), 1e-4, 4.0, 4.0, 6)).cuda()
    pairs = s.probe_pairs(x, 1.0, 0.0, 3, seed=5)
    again = s.probe_pairs(x, 1.0, 0.0, 3, seed=5)
    assert torch_cuda.equal(pairs, again)
    # run as ensemble members, two at a time (the second batch has an idle member): the same pairs
    batched = s.probe_pairs(x, 1.0, 0.0, 3, seed=5, batch=2)
    assert torch_cuda.equal(pairs, batched)
    other = s.probe_pairs(x, 1.0, 0.0, 1, seed=6)
    assert not torch_cuda.equal(pairs[0, 0], other[0, 0])
    for i in range(3):
        z, jz = pairs[i, 0], pairs[i, 1]
        assert abs(s.vec_dot(z, z) - 1.0) <= 1e-12
        zn = z.cpu().numpy()
        assert np.array_equal(zn[:, 0, 0], np.conj(zn[:, 0, 2])) and np.all(zn[:, 0, 1].imag == 0)
        F0, _ = s.newton_residual(x, 1.0, 0.0)
        eps = 1e-7 * max(np.sqrt(s.vec_dot(x, x)), 1.0)
        F1, _ = s.newton_residual(x + eps * z, 1.0, 0.0)
        fd = ((F1 - F0) / eps - jz).cpu().numpy()
        assert np.sqrt(s.vec_dot(torch_cuda.from_numpy(fd), torch_cuda.from_numpy(fd))) <= 1e-10 * max(
            1.0, np.sqrt(s.vec_dot(jz, jz)))
    # near laminar flow J z of a unit z has norm of order one, and not J = -I
    lam = torch_cuda.from_numpy(laminar_state(12, 2, 2, s.nodes())).cuda()
    pl = s.probe_pairs(lam, 1.0, 0.0, 1, seed=5)
    d = pl[0, 1] + pl[0, 0]
    assert 1e-3 < np.sqrt(s.vec_dot(d, d)) < 1.0


def test_flexible_gmres_with_minus_identity_matches_plain(torch_cuda):
    """P = -I (zero output layer) makes flexible GMRES plain GMRES on -J:
    same Newton iterations and converged result as the unpreconditioned
    solve, and the recorded pairs are (z, J z) products."""
    import paper_1705_03838_amd as opf
    kw = dict(N=12, M=2, K=2, mp=2, alpha=1.25, Re=100.0, dt=0.05)
    say("fgmres -I", kw)
    s = make_solver(**kw)
    net = opf.Mlp(s, width=32, layers=1, rank=2)
    q = net.get_params()
    q[-(net.dout * 32 + net.dout):] = 0.0
    net.set_params(q)
    x = make_state(12, 2, 2, 2, 1.25, s.nodes(), 1e-4, 4.0, 4.0, 6)
    rec = torch_cuda.zeros((8, 2) + s.shape, dtype=torch_cuda.complex128, device="cuda")
    x1, r1 = s.nk_solve(torch_cuda.from_numpy(x), 1.0, 0.0, tol=1e-10, gmres_tol=1e-6, record=rec)
    x2, r2 = s.nk_solve(torch_cuda.from_numpy(x), 1.0, 0.0, tol=1e-10, gmres_tol=1e-6, precond=net)
    say("  plain", r1, "\n  fgmres", r2)
    assert r1["converged"] and r2["converged"]
    assert r2["newton_iterations"] == r1["newton_iterations"]
    assert abs(r2["jvps"] - r1["jvps"]) <= 2 and r2["precond_applies"] > 0
    d = (x1 - x2).cpu().numpy()
    assert np.sqrt(s.vec_dot(torch_cuda.from_numpy(d), torch_cuda.from_numpy(d))) < 1e-8
    assert r1["recorded"] == min(8, r1["jvps"])
    # a recorded pair reproduces J z by a fresh finite difference
    z, jz = rec[0, 0], rec[0, 1]
    xs = torch_cuda.from_numpy(x).cuda()
    F0, _ = s.newton_residual(xs, 1.0, 0.0)
    zn = np.sqrt(s.vec_dot(z, z))
    eps = 1e-7 * max(np.sqrt(s.vec_dot(xs, xs)), 1.0) / zn
    F1, _ = s.newton_residual(xs + eps * z, 1.0, 0.0)
    fd = ((F1 - F0) / eps - jz).cpu().numpy()
    assert np.sqrt(s.vec_dot(torch_cuda.from_numpy(fd), torch_cuda.from_numpy(fd))) <= 1e-10 * max(
        1.0, np.sqrt(s.vec_dot(jz, jz)))


def test_trained_preconditioner_cuts_krylov_work(torch_cuda):
    """What the learned preconditioner gains: trained on Jacobian probes at
    laminar flow, it must leave the Newton-Krylov search converging to the
    same laminar solution with far fewer Jacobian-vector products than plain
    GMRES on a near-laminar guess of another seed."""
    import paper_1705_03838_amd as opf
    from inputs import laminar_state
    kw = dict(N=12, M=4, K=4, mp=2, alpha=1.25, Re=200.0, dt=0.05)
    T = 2.0
    say("learned preconditioner gain", kw, "T", T)
    s = make_solver(**kw)
    lam = torch_cuda.from_numpy(laminar_state(12, 4, 4, s.nodes())).cuda()
    pairs = s.probe_pairs(lam, T, 0.0, 96, seed=3)  # 3N = 36 complex unknowns per mode
    net = opf.Mlp(s, width=128, layers=4, rank=4, seed=2)
    losses = net.train_pairs(pairs, batch=16, steps=2000, seed=4)
    say("  loss first / last", losses[0], losses[-50:].mean())
    assert losses[-50:].mean() < 0.05 * losses[0]
    _, bad = net.factors()
    assert bad == 0
    x = torch_cuda.from_numpy(make_state(12, 4, 4, 2, 1.25, s.nodes(), 1e-4, 4.0, 4.0, 17))
    x1, r1 = s.nk_solve(x, T, 0.0, tol=1e-10, gmres_tol=1e-4)
    x2, r2 = s.nk_solve(x, T, 0.0, tol=1e-10, gmres_tol=1e-4, precond=net)
    say("  plain", r1, "\n  learned", r2)
    assert r1["converged"] and r2["converged"]
    assert r2["jvps"] <= 0.6 * r1["jvps"]
    for xs in (x1, x2):
        d = xs - lam
        assert np.sqrt(s.vec_dot(d, d)) < 1e-8


def test_full_size_network_matches_oracle(torch_cuda):
    """The configuration the bench trains (nk grid: N=48, |m|<24 with mp=2,
    |k|<32; width 256, 4 layers, rank 16): model rows of sampled modes and
    the preconditioner of a field against the bf16 oracle, and one pair
    gradient against the oracle's head + backprop."""
    import paper_1705_03838_amd as opf
    from inputs import WORKLOADS
    from oracle.mlp import (backprop, flatten, feature_rows, forward, head, init_params, precondition,
                            unflatten)
    w = WORKLOADS["nk"]
    s = make_solver(N=w["N"], M=w["M"], K=w["K"], mp=w["mp"], alpha=w["alpha"], Re=w["Re"], dt=w["dt"])
    net = opf.Mlp(s, width=256, layers=4, rank=16)
    say("full-size network", net.din, net.dout, net.n_params)
    p = init_params(net.din, 256, 4, net.dout, seed=12)
    p["W_out"] *= 0.3
    flat = flatten(p, 4).astype(np.float32)
    net.set_params(flat)
    p = unflatten(flat.astype(np.float64), net.din, 256, 4, net.dout)
    X = feature_rows(w["M"], w["K"], w["mp"], w["alpha"])
    rows_ = [0, 1, 31, 62, 63, 700, 1511]
    Fdev = net.forward(torch_cuda.from_numpy(X.astype(np.float32))).cpu().numpy().astype(np.float64)
    Fb, cache = forward(p, X, 4, bf16=True)
    assert nrel(Fdev[rows_], Fb[rows_]) <= 1e-2
    v = make_state(w["N"], w["M"], w["K"], w["mp"], w["alpha"], s.nodes(), 1e-3, 4.0, 4.0, 77, laminar=False)
    K = w["K"]
    for kk in range(K - 1):
        v[:, 0, kk] = np.conj(v[:, 0, 2 * (K - 1) - kk])
    v[:, 0, K - 1] = v[:, 0, K - 1].real
    z = net.precondition(torch_cuda.from_numpy(v)).cpu().numpy()
    zb = precondition(p, 4, v, w["mp"], w["alpha"], 16, bf16=True)
    say("   precondition rel", nrel(z + v, zb + v))
    assert nrel(z + v, zb + v) <= 2e-2
    g = np.random.default_rng(5)
    pairs = g.standard_normal((3, 2) + s.shape) + 1j * g.standard_normal((3, 2) + s.shape)
    idx = np.array([2, 0], dtype=np.int32)
    lg, grad = net.pair_gradient(torch_cuda.from_numpy(pairs), idx)
    L, dF = head(Fb.astype(np.float32).astype(np.float64), pairs[idx], 16)
    assert abs(lg - L) <= 1e-2 * L
    gref = backprop(p, cache, dF, 4, bf16=True)
    check_grads(grad, gref, 4)
