"""Pins for the oracle's multigrid V-cycle (the spatial preconditioner reading).

The paper does not specify its V-cycle, so these tests pin the oracle's cycle to
an independent dense-matrix construction of the same specification and to the
properties Theorem 3.1 needs (symmetry, positivity, rho_A < 1)."""
import numpy as np
import pytest

import synth
from oracle import fd, mg

from _dense import R1, dense_vcycle as _dense_vcycle, kron_d


@pytest.mark.parametrize("d,n", [(1, 15), (2, 7), (3, 7)])
def test_transfer_operators(d, n):
    rng = np.random.default_rng(0)
    Rd = kron_d(R1(n), d)
    Pd = (2 ** d) * Rd.T
    nc = (n - 1) // 2
    r = rng.standard_normal((n,) * d)
    e = rng.standard_normal((nc,) * d)
    assert np.allclose(mg.restrict(r, d).ravel(), Rd @ r.ravel(), rtol=1e-14)
    assert np.allclose(mg.prolong(e, d).ravel(), Pd @ e.ravel(), rtol=1e-14)
    # prolongation of a coarse hat function is the fine hat function (1, 1/2 neighbours)
    x = np.arange(1, n + 1) / (n + 1)
    xc = np.arange(1, nc + 1) / (nc + 1)
    hat = np.maximum(0, 1 - np.abs(x - xc[1]) * (nc + 1))
    assert np.allclose(mg.prolong(np.eye(nc)[1], 1), hat)
    # kappa restriction keeps constants and positivity
    k = np.full((n + 2,) * d, 2.5)
    assert np.allclose(mg.restrict_kappa(k, d), 2.5)
    kr = rng.uniform(0.1, 3.0, size=(n + 2,) * d)
    assert mg.restrict_kappa(kr, d).min() > 0


@pytest.mark.parametrize("d,n", [(1, 15), (2, 7), (3, 7)])
@pytest.mark.parametrize("sigma", [0.0, 0.7])
def test_vcycle_matches_dense_construction(d, n, sigma):
    prob = synth.small_problem(d, n, 2, seed=11)
    hier = mg.Hierarchy(prob.kfields, n, d)
    c = np.array([0.03, 0.01])
    V, L = _dense_vcycle(hier, sigma, c)
    rng = np.random.default_rng(1)
    b = rng.standard_normal((1,) + (n,) * d)
    x = hier.vcycle(np.array([sigma]), c[None, :], b)
    assert np.allclose(x.ravel(), V @ b.ravel(), rtol=1e-11, atol=1e-13 * np.abs(x).max())
    # symmetric positive definite, convergent: rho_A = spectral radius of I - V L < 1
    assert np.allclose(V, V.T, atol=1e-12 * np.abs(V).max())
    assert np.linalg.eigvalsh(0.5 * (V + V.T)).min() > 0
    rho = np.abs(np.linalg.eigvals(np.eye(L.shape[0]) - V @ L)).max()
    assert rho < 0.6


@pytest.mark.parametrize("d", [2, 3])
def test_vcycle_contraction_mesh_independent(d):
    """Measured rho_A (power iteration on I - V L in the L-norm) stays bounded as h shrinks."""
    rhos = []
    for n in ([15, 31, 63] if d == 2 else [7, 15, 31]):
        prob = synth.small_problem(d, n, 2, seed=12)
        hier = mg.Hierarchy(prob.kfields, n, d)
        sig, c = np.array([0.0]), np.array([[1.0, 0.5]])
        rng = np.random.default_rng(2)
        e = rng.standard_normal((1,) + (n,) * d)
        rate = 0
        for _ in range(30):
            e_new = e - hier.vcycle(sig, c, hier.apply_op(sig, c, e))
            rate = np.sqrt(np.sum(e_new * hier.apply_op(sig, c, e_new)) / np.sum(e * hier.apply_op(sig, c, e)))
            e = e_new / np.linalg.norm(e_new)
        rhos.append(rate)
    assert max(rhos) < 0.5
    assert max(rhos) - min(rhos) < 0.15


def test_hierarchy_requires_odd_levels():
    with pytest.raises(ValueError):
        mg.Hierarchy(np.ones((1, 12, 12)), 10, 2)


@pytest.mark.parametrize("nu", [2, 3])
def test_nu_cycles_iterate_the_error_propagator(nu):
    """nu cycles, each on the residual the earlier ones leave, give
    x = (I - (I - V L)^nu) L^{-1} b with V the dense single cycle."""
    d, n, sigma = 2, 7, 0.4
    prob = synth.small_problem(d, n, 2, seed=13)
    hier = mg.Hierarchy(prob.kfields, n, d)
    c = np.array([0.05, 0.02])
    V, L = _dense_vcycle(hier, sigma, c)
    E = np.eye(L.shape[0]) - V @ L
    b = np.random.default_rng(nu).standard_normal((1,) + (n,) * d)
    want = (np.eye(L.shape[0]) - np.linalg.matrix_power(E, nu)) @ np.linalg.solve(L, b.ravel())
    got = hier.vcycles(np.array([sigma]), c[None, :], b, nu)
    assert np.allclose(got.ravel(), want, rtol=1e-10, atol=1e-12 * np.abs(want).max())
