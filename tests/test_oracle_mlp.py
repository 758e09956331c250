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
    if M > 2:
        v[:, 2, 1] = 0.0  # an empty mode
    return v


def test_zero_factors_give_minus_identity_and_map_is_linear():
    from oracle.mlp import factor_dims, lowrank_apply
    M, K, N, R = 4, 3, 5, 2
    rows = M * (2 * K - 1)
    u, v = _field(1), _field(2)
    assert np.max(np.abs(lowrank_apply(np.zeros((rows, factor_dims(N, R))), v, R) + v)) == 0.0
    F = np.random.default_rng(3).standard_normal((rows, factor_dims(N, R)))
    a, b = 0.7, -2.3
    lhs = lowrank_apply(F, a * u + b * v, R)
    rhs = a * lowrank_apply(F, u, R) + b * lowrank_apply(F, v, R)
    assert np.max(np.abs(lhs - rhs)) <= 1e-12 * np.max(np.abs(rhs))
    z = lowrank_apply(F, v, R)
    for kk in range(K - 1):  # real output field
        assert np.array_equal(z[:, 0, kk], np.conj(z[:, 0, 2 * (K - 1) - kk]))
    assert np.all(z[:, 0, K - 1].imag == 0) and np.all(z[:, 2, 1] == 0)


def test_woodbury_inverts_a_low_rank_jacobian_model():
    # J = -I + U V^H on one mode (rank 2): the preconditioner built from the
    # model rows must return x from J x exactly (up to rounding)
    from oracle.mlp import factor_dims, lowrank_apply, woodbury
    M, K, N, R = 2, 2, 4, 2
    nk, n3 = 2 * K - 1, 3 * N
    rng = np.random.default_rng(8)
    U = rng.standard_normal((n3, R)) + 1j * rng.standard_normal((n3, R))
    V = 0.2 * (rng.standard_normal((n3, R)) + 1j * rng.standard_normal((n3, R)))
    q = 1 * nk + 2  # mode m = 1, k = +1
    F = np.zeros((M * nk, factor_dims(N, R)))
    F[q, 0:2 * n3 * R:2], F[q, 1:2 * n3 * R:2] = U.reshape(-1).real, U.reshape(-1).imag
    F[q, 2 * n3 * R:4 * n3 * R:2], F[q, 2 * n3 * R + 1:4 * n3 * R:2] = V.reshape(-1).real, V.reshape(-1).imag
    x = rng.standard_normal(n3) + 1j * rng.standard_normal(n3)
    jx = -x + U @ (np.conj(V).T @ x)
    v = np.zeros((3, M, nk, N), dtype=complex)
    v[:, 1, 2, :] = jx.reshape(3, N)
    z = lowrank_apply(woodbury(F, N, R), v, R)
    assert np.max(np.abs(z[:, 1, 2, :].reshape(-1) - x)) <= 1e-12 * np.max(np.abs(x))
    # modes with a zero model are left at P = -I
    assert np.all(z[:, 0] == 0) and np.all(z[:, 1, 0] == 0)


def test_head_gradient_matches_finite_differences():
    from oracle.mlp import factor_dims, head
    M, K, N, R = 2, 2, 4, 2
    rows = M * (2 * K - 1)
    rng = np.random.default_rng(9)
    F = 0.3 * rng.standard_normal((rows, factor_dims(N, R)))
    pairs = np.stack([np.stack([_field(20 + i, M, K, N), _field(30 + i, M, K, N)]) for i in range(3)])
    L0, dF = head(F, pairs, R)
    assert L0 > 0
    h = 1e-6
    for idx in [(0, 0), (1, 7), (3, 3 * N * R * 2 + 5), (5, 4 * 3 * N * R - 1)]:
        Fp, Fm = F.copy(), F.copy()
        Fp[idx] += h
        Fm[idx] -= h
        fd = (head(Fp, pairs, R)[0] - head(Fm, pairs, R)[0]) / (2 * h)
        assert abs(fd - dF[idx]) <= 1e-7 * max(1.0, abs(fd)), (idx, fd, dF[idx])


def test_feature_rows():
    from oracle.mlp import cond_features, feature_rows
    X = feature_rows(3, 4, 2, 1.25)
    assert X.shape == (3 * 7, 32)
    f = cond_features(1, 1, 2, 1.25)
    assert np.array_equal(X[1 * 7 + 4], f)
    assert f[0] == 1 and f[9] == 1 and f[24] == 1 and f[31] == 0
    assert abs(f[1] - 2 / 48) < 1e-15 and abs(f[2] - 1.25 / 40) < 1e-15 and f[4] == 1
    g = cond_features(9, -8, 2, 1.25)
    assert g[31] == 1 and np.all(g[8:31] == 0) and g[4] == -1
