"""Helpers of the GPU parity tests (not collected by pytest).

The checker owns its inputs: every library context under test is created on
the radial nodes the oracle computes for itself (oracle.grid.radial_nodes),
passed to the library through opf_params.r_nodes, so the oracle never takes
a value from the library under test.  The library's own default nodes are
compared with the oracle's separately, on the CPU (test_library_host.py).
"""
import numpy as np


def oracle_nodes(N):
    from oracle.grid import radial_nodes
    return np.ascontiguousarray(radial_nodes(N), dtype=np.float64)


def make_solver(**kw):
    """opf.Solver on the oracle's radial nodes for kw['N'] (default 24)."""
    import paper_1705_03838_amd as opf
    return opf.Solver(r_nodes=oracle_nodes(kw.get("N", 24)), **kw)


def make_ensemble(members, **kw):
    """opf.Ensemble whose members all use the oracle's radial nodes."""
    import paper_1705_03838_amd as opf
    return opf.Ensemble([dict(m, r_nodes=oracle_nodes(m.get("N", 24))) for m in members], **kw)


def energy_rel(o, got, ref, base):
    """Energy-norm errors of `got` against `ref` relative to the full state
    and to the perturbation ref - base (the workload's laminar flow)."""
    e = o.energy_norm(got - ref)
    return e / o.energy_norm(ref), e / o.energy_norm(ref - base)
