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
    r = bf16_round if bf16 else (lambda a: a)
    w = np.ones(y.shape[0]) if w is None else np.asarray(w, dtype=np.float64)
    g = {}
    dy = 2.0 * w[:, None] * (y - t) / np.sum(w)
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
# Mode profiles <-> rows (the preconditioner's input and output maps)

NCOND = 32


def dims(N):
    p6 = (6 * N + 31) // 32 * 32
    return p6 + NCOND, p6


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


def pack(y, mp, alpha, z=None):
    """Rows of the modes of one vector field y [3][M][2K-1][N] (complex):
    returns X [M(2K-1)][din], T (targets from z, or None), weights s^2 and
    (s, e) per row.  Row of mode (m, k): yhat = conj(e) y / s with s the RMS
    of the profile and e the phase of its plain sum; target conj(e) z / s + yhat."""
    _, M, nk, N = y.shape
    K = (nk + 1) // 2
    din, p6 = dims(N)
    rows = M * nk
    X = np.zeros((rows, din))
    T = np.zeros((rows, p6)) if z is not None else None
    S = np.zeros(rows)
    E = np.ones(rows, dtype=complex)
    for mi in range(M):
        for kk in range(nk):
            q = mi * nk + kk
            prof = y[:, mi, kk, :].reshape(-1)
            s = np.sqrt(np.sum(np.abs(prof) ** 2) / (3 * N))
            rho = np.sum(prof)
            e = rho / abs(rho) if abs(rho) > 1e-8 * 3 * N * s else 1.0 + 0j
            S[q], E[q] = s, e
            yh = np.conj(e) * prof / s if s > 0 else np.zeros_like(prof)
            X[q, 0:6 * N:2], X[q, 1:6 * N:2] = yh.real, yh.imag
            X[q, p6:] = cond_features(mi, kk - (K - 1), mp, alpha)
            if z is not None:
                zp = z[:, mi, kk, :].reshape(-1)
                th = (np.conj(e) * zp / s if s > 0 else np.zeros_like(zp)) + yh
                T[q, 0:6 * N:2], T[q, 1:6 * N:2] = th.real, th.imag
    return X, T, S ** 2, S, E


def unpack(F, y, S, E):
    """z_mk = s e f - y_mk, f the output row read as a complex profile;
    z(0, k<0) = conj z(0, -k)."""
    _, M, nk, N = y.shape
    K = (nk + 1) // 2
    z = np.zeros_like(y)
    for mi in range(M):
        for kk in range(nk):
            q = mi * nk + kk
            f = (F[q, 0:6 * N:2] + 1j * F[q, 1:6 * N:2]).reshape(3, N)
            z[:, mi, kk, :] = S[q] * E[q] * f - y[:, mi, kk, :]
    for kk in range(K - 1):
        z[:, 0, kk, :] = np.conj(z[:, 0, 2 * (K - 1) - kk, :])
    return z


def precondition(p, layers, y, mp, alpha, bf16=False):
    """Preconditioner applied to a vector field y: pack, network, unpack.
    bf16=True rounds the GEMM operands as the device does; the FP32 rows the
    device feeds its first product are emulated by rounding through float32."""
    X, _, _, S, E = pack(y, mp, alpha)
    if bf16:
        X = X.astype(np.float32).astype(np.float64)
    F, _ = forward(p, X, layers, bf16=bf16)
    if bf16:
        F = F.astype(np.float32).astype(np.float64)
    return unpack(F, y, S, E)
