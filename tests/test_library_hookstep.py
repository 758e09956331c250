"""The library's hookstep subproblem (host-only C-ABI call, SVD by one-sided
Jacobi) against the oracle's (normal equations and a bracketing root
finder), on random Hessenberg matrices with constrained and unconstrained
radii, a rank-deficient (breakdown) case and the diagonal closed form."""
import numpy as np
import pytest

from oracle.hookstep import hook_subproblem


def lib_solve(Hb, beta, delta):
    import paper_1705_03838_amd as opf
    return opf.hookstep_solve(Hb, beta, delta)


def hess(k, seed, scale=1.0):
    r = np.random.default_rng(seed)
    return np.triu(r.standard_normal((k + 1, k)), -1) * scale


@pytest.mark.parametrize("k", [1, 2, 5, 13, 40])
@pytest.mark.parametrize("frac", [0.01, 0.3, 0.9, 2.0])
def test_matches_oracle(k, frac):
    Hb = hess(k, 100 + k)
    Hb[np.arange(1, k + 1), np.arange(k)] = np.abs(Hb[np.arange(1, k + 1), np.arange(k)]) + 0.05
    beta = 0.7
    yls, _, _ = hook_subproblem(Hb, beta, np.inf)
    delta = frac * np.linalg.norm(yls)
    y0, mu0, r0 = hook_subproblem(Hb, beta, delta)
    y1, mu1, r1 = lib_solve(Hb, beta, delta)
    assert np.linalg.norm(y1 - y0) <= 1e-9 * np.linalg.norm(y0)
    assert abs(r1 - r0) <= 1e-12 * beta
    if frac < 1:
        assert mu0 > 0 and abs(mu1 - mu0) <= 1e-6 * mu0  # mu ~ sigma_min^2 here is weakly determined
        assert abs(np.linalg.norm(y1) - delta) <= 1e-12 * delta
    else:
        assert mu1 == 0.0


def test_breakdown_column():
    Hb = hess(4, 7)
    Hb[4, 3] = 0.0  # Arnoldi breakdown: the last subdiagonal entry vanishes
    for delta in (np.inf, 0.05):
        y0, mu0, r0 = hook_subproblem(Hb, 1.3, delta)
        y1, mu1, r1 = lib_solve(Hb, 1.3, delta)
        assert np.linalg.norm(y1 - y0) <= 1e-9 * np.linalg.norm(y0)
        assert abs(r1 - r0) <= 1e-12


def test_diagonal_closed_form_and_bad_arguments():
    import paper_1705_03838_amd as opf
    sig = np.array([3.0, 0.5, 0.2])
    Hb = np.vstack([np.diag(sig), np.zeros((1, 3))])
    y, mu, r = lib_solve(Hb, 2.0, 0.1)
    assert mu == pytest.approx(2.0 * 3.0 / 0.1 - 9.0, rel=1e-12)
    assert np.allclose(y, [0.1, 0, 0], atol=1e-15)
    with pytest.raises(opf.OpfError):
        lib_solve(Hb, 2.0, 0.0)
