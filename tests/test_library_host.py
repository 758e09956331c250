"""The C-ABI library without a GPU: it loads, exports every symbol the header
declares, validates parameters, and its create-time radial tables (computed by
its own C++: Fornberg weights, Gauss-Legendre quadrature) equal the oracle's
independently computed ones."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1705_03838_amd as opf
from oracle.grid import fd_matrices, quadrature_weights, radial_nodes

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    with open(os.path.join(ROOT, "include", "opf.h")) as f:
        text = f.read()
    return sorted(set(re.findall(r"\b(opf_[a-z_0-9]+)\s*\(", text)))


def test_exports_every_declared_symbol():
    lib = opf.load_library()
    names = header_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(opf.EXPORTS) == names


def test_parameter_validation_and_workspace():
    lib = opf.load_library()
    p = opf.opf_params()
    assert lib.opf_default_params(ctypes.byref(p)) == 0
    assert (p.N, p.M, p.K, p.stencil) == (24, 8, 8, 9)
    size = ctypes.c_size_t()
    assert lib.opf_workspace_size(ctypes.byref(p), ctypes.byref(size)) == 0
    assert size.value > 0
    for field, bad, code in [("N", 8, opf.OPF_E_INVALID), ("N", 65, opf.OPF_E_UNSUPPORTED),
                             ("M", 5, opf.OPF_E_UNSUPPORTED), ("K", 1, opf.OPF_E_INVALID),
                             ("stencil", 7, opf.OPF_E_INVALID), ("dt", 0.0, opf.OPF_E_INVALID),
                             ("Re", -1.0, opf.OPF_E_INVALID), ("precision", 7, opf.OPF_E_INVALID),
                             ("n_corr", 0, opf.OPF_E_INVALID)]:
        q = opf.make_params()
        setattr(q, field, bad)
        assert lib.opf_workspace_size(ctypes.byref(q), ctypes.byref(size)) == code, field
    # bad explicit nodes
    q = opf.make_params(N=12)
    r = np.linspace(0.1, 0.9, 12)
    q.r_nodes = r.ctypes.data
    assert lib.opf_workspace_size(ctypes.byref(q), ctypes.byref(size)) == opf.OPF_E_INVALID
    assert lib.opf_status_string(opf.OPF_E_STATE) == b"no state set"
    out = ctypes.c_void_p()
    assert lib.opf_create(None, None, 0, None, ctypes.byref(out)) == opf.OPF_E_INVALID
    p = opf.make_params()
    assert lib.opf_create(ctypes.byref(p), None, 0, None, ctypes.byref(out)) == opf.OPF_E_NOMEM


@pytest.mark.parametrize("N", [13, 24, 48, 64])
def test_host_tables_match_oracle(N):
    r, q, d1, d2, s0 = opf.host_tables(N=N)
    assert np.max(np.abs(r - radial_nodes(N))) <= 2e-16
    assert np.max(np.abs(q - quadrature_weights(r))) <= 1e-15
    for par, sign in ((0, +1), (1, -1)):
        D1, D2 = fd_matrices(r, sign)
        A1 = np.zeros((N, N))
        A2 = np.zeros((N, N))
        for n in range(N):
            A1[n, s0[n]:s0[n] + 9] = d1[par, n]
            A2[n, s0[n]:s0[n] + 9] = d2[par, n]
        assert np.max(np.abs(A1 - D1)) <= 1e-12 * np.max(np.abs(D1))
        assert np.max(np.abs(A2 - D2)) <= 1e-12 * np.max(np.abs(D2))
