"""Residual MLP used as a learned GMRES preconditioner (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Not part of the paper: the network stands in front of the Newton-Krylov
solver of Section 2.  Architecture (shared by the HIP kernels):
    h_0 = W_in x + b_in                         x: DIN features, h: width H
    h_l = h_{l-1} + relu(W_l h_{l-1} + b_l),    l = 1..L
    y   = W_out h_L + b_out                     y: DOUT outputs
Loss of a batch: sum_r w_r sum_j (y_rj - t_rj)^2 / sum_r w_r (w_r = 1 when no
weights are given), minimised by Adam (Kingma & Ba 2015).
Weights are [out][in] row-major.  `bf16=True` rounds every GEMM operand
(weights, x, h, output gradients) to bfloat16 (round to nearest even) as the
device kernels do, accumulating in float64 here (FP32 on the device).
"""
import numpy as np


def bf16_round(a):
    """Round float64 values to bfloat16 (nearest, ties to even) and back."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    u = (u + np.uint64(0x7FFF) + lsb) & np.uint64(0xFFFF0000)
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def init_params(din, width, layers, dout, seed):
    """He-style initialisation from SplitMix64 normals (seeded input data)."""
    from inputs import normals
    g = normals(seed, din * width + layers * width * width + width * dout)
    p, o = {}, 0

    def take(n_out, n_in, scale):
        nonlocal o
        w = g[o:o + n_out * n_in].reshape(n_out, n_in) * scale
        o += n_out * n_in
        return w

    p["W_in"] = take(width, din, np.sqrt(1.0 / din))
    p["b_in"] = np.zeros(width)
    for l in range(layers):
        p[f"W_{l}"] = take(width, width, 0.5 * np.sqrt(2.0 / width))
        p[f"b_{l}"] = np.zeros(width)
    p["W_out"] = take(dout, width, np.sqrt(1.0 / width))
    p["b_out"] = np.zeros(dout)
    return p


def forward(p, x, layers, bf16=False):
    r = bf16_round if bf16 else (lambda a: a)
    cache = {"x": x}
    h = r(x) @ r(p["W_in"]).T + p["b_in"]
    cache["h0"] = h
    for l in range(layers):
        z = r(h) @ r(p[f"W_{l}"]).T + p[f"b_{l}"]
        cache[f"z{l}"] = z
        h = h + np.maximum(z, 0.0)
        cache[f"h{l + 1}"] = h
    y = r(h) @ r(p["W_out"]).T + p["b_out"]
    return y, cache


def loss(y, t, w=None):
    w = np.ones(y.shape[0]) if w is None else np.asarray(w, dtype=np.float64)
    return float(np.sum(w * np.sum((y - t) ** 2, axis=1)) / np.sum(w))


def backward(p, cache, y, t, layers, bf16=False, w=None):
    """Gradients of loss(y, t, w) with respect to every parameter."""
    w = np.ones(y.shape[0]) if w is None else np.asarray(w, dtype=np.float64)
    dy = 2.0 * w[:, None] * (y - t) / np.sum(w)
    return backprop(p, cache, dy, layers, bf16)


def backprop(p, cache, dy, layers, bf16=False):
    """Parameter gradients of a loss whose gradient with respect to the
    network output is dy."""
    r = bf16_round if bf16 else (lambda a: a)
    g = {}
    hL = cache[f"h{layers}"]
    g["W_out"] = r(dy).T @ r(hL)
    g["b_out"] = dy.sum(0)
    dh = r(dy) @ r(p["W_out"])
    for l in reversed(range(layers)):
        z = cache[f"z{l}"]
        hprev = cache[f"h{l}"]
        dz = dh * (z > 0)
        g[f"W_{l}"] = r(dz).T @ r(hprev)
        g[f"b_{l}"] = dz.sum(0)
        dh = dh + r(dz) @ r(p[f"W_{l}"])
    g["W_in"] = r(dh).T @ r(cache["x"])
    g["b_in"] = dh.sum(0)
    return g


def param_names(layers):
    """Order of the flat parameter array (W_in, b_in, W_0, b_0, ..., W_out, b_out)."""
    names = ["W_in", "b_in"]
    for l in range(layers):
        names += [f"W_{l}", f"b_{l}"]
    return names + ["W_out", "b_out"]


def flatten(p, layers):
    return np.concatenate([p[k].ravel() for k in param_names(layers)])


def unflatten(flat, din, width, layers, dout):
    shapes = {"W_in": (width, din), "b_in": (width,), "W_out": (dout, width), "b_out": (dout,)}
    for l in range(layers):
        shapes[f"W_{l}"] = (width, width)
        shapes[f"b_{l}"] = (width,)
    p, o = {}, 0
    for k in param_names(layers):
        n = int(np.prod(shapes[k]))
        p[k] = np.asarray(flat[o:o + n], dtype=np.float64).reshape(shapes[k])
        o += n
    assert o == len(flat)
    return p


def adam(p, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba 2015) on flat arrays; t counts from 1."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


# ---------------------------------------------------------------------------
# The preconditioner built from the network: per-mode low-rank corrections

NCOND = 32


def cond_features(mi, k, mp, alpha):
    """32 conditioning features of mode (m, k): mu = mp m, kappa = alpha k;
    1, mu/48, kappa/40, |kappa|/40, sign kappa, (mu/48)^2, (kappa/40)^2,
    mu |kappa| / 1920, one-hot of m for m < 8, one-hot of k for |k| <= 7,
    and [|k| > 7]."""
    mu, ka = mp * mi, alpha * k
    f = [1.0, mu / 48, ka / 40, abs(ka) / 40, float(np.sign(ka)), (mu / 48) ** 2, (ka / 40) ** 2,
         mu * abs(ka) / 1920]
    f += [1.0 if mi == j else 0.0 for j in range(8)]
    f += [1.0 if k == j else 0.0 for j in range(-7, 8)]
    f += [1.0 if abs(k) > 7 else 0.0]
    assert len(f) == NCOND
    return np.array(f)


def feature_rows(M, K, mp, alpha):
    """Network input: one row per mode (m, k), m-major, k = -(K-1)..K-1."""
    nk = 2 * K - 1
    return np.array([cond_features(mi, kk - (K - 1), mp, alpha) for mi in range(M) for kk in range(nk)])


def factor_dims(N, rank):
    return (12 * N * rank + 31) // 32 * 32


def factors(F, N, rank):
    """Output rows [modes][>= 12 N rank] -> A, B [modes][3N][rank] complex:
    A[e][j] at 2(e rank + j) (+1 imaginary), B the same from 6 N rank on."""
    n = 3 * N * rank
    A = F[:, 0:2 * n:2] + 1j * F[:, 1:2 * n:2]
    B = F[:, 2 * n:4 * n:2] + 1j * F[:, 2 * n + 1:4 * n:2]
    return A.reshape(-1, 3 * N, rank), B.reshape(-1, 3 * N, rank)


def profiles(v):
    """[3][M][nk][N] -> [M nk][3N] (mode rows, component-major profile)."""
    _, M, nk, N = v.shape
    return np.transpose(v, (1, 2, 0, 3)).reshape(M * nk, 3 * N)


def lowrank_apply(F, v, rank):
    """z_mk = -v_mk + A_mk (B_mk^H v_mk) for every mode; (m = 0, k < 0) is the
    conjugate of (0, -k) and (0, 0) keeps its real part."""
    _, M, nk, N = v.shape
    K = (nk + 1) // 2
    A, B = factors(F, N, rank)
    y = profiles(v)
    c = np.einsum("qej,qe->qj", np.conj(B), y)
    z = -y + np.einsum("qej,qj->qe", A, c)
    z = np.transpose(z.reshape(M, nk, 3, N), (2, 0, 1, 3)).copy()
    for kk in range(K - 1):
        z[:, 0, kk] = np.conj(z[:, 0, 2 * (K - 1) - kk])
    z[:, 0, K - 1] = z[:, 0, K - 1].real
    return z


def head(F, pairs, rank):
    """Loss of the Jacobian model J_q ~ -I + U V^H (U, V = factors(F)) on a
    batch of (z, J z) pairs [b][2][3][M][nk][N], and its gradient with
    respect to the output rows.  Per mode and pair: s = RMS of the z profile
    (pairs with s = 0 skip), xhat = z/s, that = (J z)/s,
    r = -xhat + U (V^H xhat) - that; loss = sum |r|^2 / (b M nk); the gradient
    of a real function of complex factors (Re + i Im parts) is
    dU = 2 r c^H with c = V^H xhat, dV = 2 xhat (U^H r)^H per term."""
    b = pairs.shape[0]
    _, M, nk, N = pairs.shape[2:]
    U, V = factors(F, N, rank)
    dU, dV = np.zeros_like(U), np.zeros_like(V)
    total = 0.0
    for p in range(b):
        x, y = profiles(pairs[p, 0]), profiles(pairs[p, 1])
        s = np.sqrt(np.mean(np.abs(x) ** 2, axis=1))
        live = s > 0
        inv = np.where(live, 1.0 / np.where(live, s, 1.0), 0.0)
        xh, th = x * inv[:, None], y * inv[:, None]
        c = np.einsum("qej,qe->qj", np.conj(V), xh)
        r = -xh + np.einsum("qej,qj->qe", U, c) - th
        total += np.sum(np.abs(r) ** 2)
        g = np.einsum("qej,qe->qj", np.conj(U), r)
        dU += 2 * np.einsum("qe,qj->qej", r, np.conj(c))
        dV += 2 * np.einsum("qe,qj->qej", xh, np.conj(g))
    scale = 1.0 / (b * M * nk)
    dF = np.zeros_like(F)
    n = 3 * N * rank
    dU, dV = dU.reshape(-1, n) * scale, dV.reshape(-1, n) * scale
    dF[:, 0:2 * n:2], dF[:, 1:2 * n:2] = dU.real, dU.imag
    dF[:, 2 * n:4 * n:2], dF[:, 2 * n + 1:4 * n:2] = dV.real, dV.imag
    return total * scale, dF


def woodbury(F, N, rank):
    """Preconditioner rows (A, B) from Jacobian-model rows (U, V): the exact
    inverse of -I + U V^H is -(I + U G^{-1} V^H), G = I - V^H U, so A = -U G^{-1},
    B = V (a singular G gives A = 0).  Same row layout as F."""
    U, V = factors(F, N, rank)
    out = np.zeros_like(F)
    n = 3 * N * rank
    for q in range(F.shape[0]):
        G = np.eye(rank) - np.conj(V[q]).T @ U[q]
        try:
            A = -U[q] @ np.linalg.inv(G)
        except np.linalg.LinAlgError:
            A = np.zeros_like(U[q])
        a = A.reshape(-1)
        out[q, 0:2 * n:2], out[q, 1:2 * n:2] = a.real, a.imag
    out[:, 2 * n:4 * n] = F[:, 2 * n:4 * n]
    return out


def precondition(p, layers, v, mp, alpha, rank, bf16=False):
    """The network's preconditioner applied to v: Jacobian-model rows from the
    mode features, Woodbury inverse, then the low-rank map (bf16=True rounds
    as the device does; the device keeps the rows in FP32)."""
    _, M, nk, N = v.shape
    X = feature_rows(M, (nk + 1) // 2, mp, alpha)
    F, _ = forward(p, X, layers, bf16=bf16)
    if bf16:
        F = F.astype(np.float32).astype(np.float64)
    return lowrank_apply(woodbury(F, N, rank), v, rank)
