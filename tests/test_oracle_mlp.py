"""Pins of the oracle MLP (learned-preconditioner network): FP64 backward
against central finite differences; bfloat16 rounding against its definition
(nearest, ties to even, on the top 16 bits of IEEE single)."""
import numpy as np

from oracle.mlp import backward, bf16_round, forward, init_params, loss


def test_bf16_rounding_definition():
    vals = np.array([1.0, 1.00390625, 1.005859375, 1.0078125, -3.14159265, 65504.0, 1e-3])
    got = bf16_round(vals)
    # 1 + 2^-8 is a tie between 1 and 1 + 2^-7 -> even mantissa (1.0)
    assert got[0] == 1.0 and got[1] == 1.0
    assert got[2] == 1.0078125 and got[3] == 1.0078125
    assert abs(got[4] + 3.140625) < 1e-12
    # every result has at most 8 significant bits
    m, _ = np.frexp(got)
    assert np.all(np.abs(m * 256 - np.round(m * 256)) < 1e-9)


def test_backward_matches_finite_differences():
    din, width, layers, dout, B = 12, 16, 3, 10, 7
    p = init_params(din, width, layers, dout, seed=11)
    for k in p:
        if k.startswith("b_"):
            p[k] = np.linspace(-0.1, 0.1, p[k].size)
    rng = np.random.default_rng(2)
    x = rng.standard_normal((B, din))
    t = rng.standard_normal((B, dout))
    y, cache = forward(p, x, layers)
    g = backward(p, cache, y, t, layers)
    h = 1e-6
    for name in ["W_in", "b_in", "W_0", "b_1", "W_2", "W_out", "b_out"]:
        for idx in [(0,), (3,), (-1,)] if p[name].ndim == 1 else [(0, 0), (2, 5), (-1, -1)]:
            pp = {k: v.copy() for k, v in p.items()}
            pm = {k: v.copy() for k, v in p.items()}
            pp[name][idx] += h
            pm[name][idx] -= h
            fd = (loss(forward(pp, x, layers)[0], t) - loss(forward(pm, x, layers)[0], t)) / (2 * h)
            assert abs(fd - g[name][idx]) <= 1e-6 * max(1.0, abs(fd)), (name, idx, fd, g[name][idx])


def test_adam_constant_gradient_closed_form():
    # with a constant gradient the bias-corrected moments are exactly g and
    # g^2, so every step moves by lr g / (|g| + eps)
    from oracle.mlp import adam
    g = np.array([0.3, -2.0, 1e-3, 0.0])
    p = np.array([1.0, 2.0, 3.0, 4.0])
    m = np.zeros(4)
    v = np.zeros(4)
    lr, eps = 1e-2, 1e-8
    for t in range(1, 6):
        p, m, v = adam(p, g, m, v, t, lr=lr, eps=eps)
    expect = np.array([1.0, 2.0, 3.0, 4.0]) - 5 * lr * g / (np.abs(g) + eps)
    assert np.allclose(p, expect, rtol=0, atol=1e-13)


def test_weighted_loss_gradient_finite_differences():
    din, width, layers, dout, B = 8, 16, 2, 6, 5
    p = init_params(din, width, layers, dout, seed=3)
    rng = np.random.default_rng(4)
    x, t = rng.standard_normal((B, din)), rng.standard_normal((B, dout))
    w = rng.uniform(0.1, 3.0, B)
    y, cache = forward(p, x, layers)
    g = backward(p, cache, y, t, layers, w=w)
    h = 1e-6
    for name, idx in [("W_in", (1, 2)), ("b_0", (3,)), ("W_out", (4, 5))]:
        pp = {k: v.copy() for k, v in p.items()}
        pm = {k: v.copy() for k, v in p.items()}
        pp[name][idx] += h
        pm[name][idx] -= h
        fd = (loss(forward(pp, x, layers)[0], t, w) - loss(forward(pm, x, layers)[0], t, w)) / (2 * h)
        assert abs(fd - g[name][idx]) <= 1e-6 * max(1.0, abs(fd))


def _field(seed, M=4, K=3, N=5):
    rng = np.random.default_rng(seed)
    nk = 2 * K - 1
    v = rng.standard_normal((3, M, nk, N)) + 1j * rng.standard_normal((3, M, nk, N))
    for kk in range(K - 1):  # real field: m = 0 Hermitian in k
        v[:, 0, kk] = np.conj(v[:, 0, 2 * (K - 1) - kk])
    v[:, 0, K - 1] = v[:, 0, K - 1].real
    v[:, 2, 1] = 0.0  # an empty mode
    return v


def _net(N, seed=5, layers=2, width=32, zero_out=False):
    from oracle.mlp import dims
    din, dout = dims(N)
    p = init_params(din, width, layers, dout, seed=seed)
    p["b_out"] = np.linspace(-0.2, 0.3, dout)
    if zero_out:
        p["W_out"][:] = 0.0
        p["b_out"][:] = 0.0
    return p


def test_zero_network_is_minus_identity():
    from oracle.mlp import precondition
    v = _field(1)
    z = precondition(_net(5, zero_out=True), 2, v, mp=2, alpha=1.25)
    assert np.array_equal(z, -v) or np.max(np.abs(z + v)) <= 1e-15 * np.max(np.abs(v))


def test_preconditioner_homogeneous_phase_equivariant_hermitian():
    from oracle.mlp import precondition
    v = _field(2)
    p = _net(5)
    K = 3
    z = precondition(p, 2, v, mp=2, alpha=1.25)
    # positive homogeneity
    z2 = precondition(p, 2, 3.7 * v, mp=2, alpha=1.25)
    assert np.max(np.abs(z2 - 3.7 * z)) <= 1e-12 * np.max(np.abs(z2))
    # commutes with a phase rotation of the modes m > 0 (and of (0, k >= 0))
    ph = np.exp(0.83j)
    zr = precondition(p, 2, ph * v, mp=2, alpha=1.25)
    assert np.max(np.abs(zr[:, 1:] - ph * z[:, 1:])) <= 1e-12 * np.max(np.abs(z))
    assert np.max(np.abs(zr[:, 0, K - 1:] - ph * z[:, 0, K - 1:])) <= 1e-12 * np.max(np.abs(z))
    # m = 0 output is Hermitian in k; an empty mode maps to zero
    for kk in range(K - 1):
        assert np.array_equal(z[:, 0, kk], np.conj(z[:, 0, 2 * (K - 1) - kk]))
    assert np.all(z[:, 2, 1] == 0)
    # a nonzero network changes the result
    assert np.max(np.abs(z + v)) > 1e-3


def test_pack_rows_layout_and_features():
    from oracle.mlp import cond_features, dims, pack
    v = _field(3)
    X, T, w, S, E = pack(v, 2, 1.25, z=-v)
    din, p6 = dims(5)
    assert X.shape == (4 * 5, din) and T.shape == (4 * 5, p6)
    q = 1 * 5 + 3  # m = 1, k = +1
    prof = v[:, 1, 3, :].reshape(-1)
    s = np.sqrt(np.mean(np.abs(prof) ** 2))
    assert abs(S[q] - s) <= 1e-15 * s and abs(w[q] - s * s) <= 1e-14 * s * s
    yh = X[q, 0:30:2] + 1j * X[q, 1:30:2]
    assert abs(np.sum(yh).imag) <= 1e-12 and np.sum(yh).real > 0  # phase canonical
    assert abs(np.mean(np.abs(yh) ** 2) - 1) <= 1e-12
    assert np.max(np.abs(T[q])) <= 1e-12  # target of z = -y is zero
    f = cond_features(1, 1, 2, 1.25)
    assert np.array_equal(X[q, p6:], f)
    assert f[0] == 1 and f[9] == 1 and f[24] == 1 and f[31] == 0 and f.sum() > 3
