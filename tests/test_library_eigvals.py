"""The library's Hessenberg eigenvalue routine (host-only C-ABI call,
Francis double-shift QR) against numpy.linalg.eigvals: random upper
Hessenberg matrices of sizes 1-60, matrices with complex pairs, triangular
(already deflated) ones and the ordering of the result."""
import ctypes

import numpy as np
import pytest


def lib_eig(H):
    import paper_1705_03838_amd as opf
    lib = opf.load_library()
    H = np.ascontiguousarray(H, dtype=np.float64)
    k = H.shape[0]
    re, im = np.zeros(k), np.zeros(k)
    dp = ctypes.POINTER(ctypes.c_double)
    st = lib.opf_hessenberg_eigvals(H.ctypes.data_as(dp), k, re.ctypes.data_as(dp), im.ctypes.data_as(dp))
    assert st == 0
    return re + 1j * im


def match(a, b, tol):
    """Every value of a has a distinct partner in b within tol."""
    b = list(b)
    for z in a:
        d = [abs(z - w) for w in b]
        i = int(np.argmin(d))
        assert d[i] <= tol, (z, b[i])
        b.pop(i)


@pytest.mark.parametrize("k", [1, 2, 3, 5, 10, 30, 60])
@pytest.mark.parametrize("seed", [0, 1])
def test_random_hessenberg(k, seed):
    r = np.random.default_rng(seed * 100 + k)
    H = np.triu(r.standard_normal((k, k)), -1)
    ev = lib_eig(H)
    match(ev, np.linalg.eigvals(H), 1e-9 * np.linalg.norm(H))
    mods = np.abs(ev)
    assert np.all(mods[:-1] >= mods[1:] - 1e-12)  # decreasing modulus


def test_complex_pairs_and_order():
    # block diagonal rotations scaled by 0.9 and 0.5, plus a real 0.7
    def rot(a, t):
        return a * np.array([[np.cos(t), -np.sin(t)], [np.sin(t), np.cos(t)]])
    H = np.zeros((5, 5))
    H[0:2, 0:2] = rot(0.9, 0.3)
    H[2, 2] = 0.7
    H[3:5, 3:5] = rot(0.5, 1.1)
    H[0, 2:] = 0.3
    H[2, 3:] = -0.2
    ev = lib_eig(H)
    expect = [0.9 * np.exp(0.3j), 0.9 * np.exp(-0.3j), 0.7, 0.5 * np.exp(1.1j), 0.5 * np.exp(-1.1j)]
    assert np.allclose(ev, expect, atol=1e-13)


def test_triangular_is_its_diagonal():
    r = np.random.default_rng(3)
    H = np.triu(r.standard_normal((8, 8)))
    ev = lib_eig(H)
    match(ev, np.diag(H), 1e-14)
