"""Pins for the oracle's finite-difference operator (spatial A_n of Section 2)."""
import numpy as np
import pytest

from oracle import fd


def _nodes(n):
    return np.arange(n + 2) / (n + 1)


@pytest.mark.parametrize("d,n", [(1, 9), (2, 5), (3, 3)])
def test_three_routes_agree(d, n):
    rng = np.random.default_rng(d)
    kap = rng.uniform(0.5, 2.0, size=(n + 2,) * d)
    h = 1.0 / (n + 1)
    A1 = fd.assemble_loops(kap, n, d, h).toarray()
    A2 = fd.assemble(kap, n, d, h).toarray()
    # column by column through the matrix-free operator
    eye = np.eye(n ** d).reshape((n ** d,) + (n,) * d)
    A3 = fd.apply(kap, eye, h, d).reshape(n ** d, n ** d).T
    assert np.allclose(A1, A2, rtol=1e-14, atol=0)
    assert np.allclose(A1, A3, rtol=1e-13, atol=1e-9)
    assert np.allclose(A1, A1.T)
    assert np.linalg.eigvalsh(A1).min() > 0


@pytest.mark.parametrize("d", [1, 2, 3])
def test_exact_on_quadratic_with_linear_kappa(d):
    """For kappa affine and u = prod x(1-x), the scheme with arithmetic-mean faces
    reproduces -div(kappa grad u) exactly at the nodes (closed form)."""
    n = 7
    h = 1.0 / (n + 1)
    x = _nodes(n)
    grids = np.meshgrid(*([x] * d), indexing="ij")   # grids[a] varies along axis a
    coef = [0.7, -0.3, 0.4][:d]
    kap = 1.3 + sum(c * g for c, g in zip(coef, grids))
    ui = [g[(slice(1, n + 1),) * d] for g in grids]
    q = [xi * (1 - xi) for xi in ui]
    u = np.prod(q, axis=0)
    k_in = kap[(slice(1, n + 1),) * d]
    exact = np.zeros_like(u)
    for a in range(d):
        other = np.prod([q[b] for b in range(d) if b != a], axis=0) if d > 1 else 1.0
        # -d/dx_a (kappa * d/dx_a q_a) * other,  q_a = x(1-x): q' = 1-2x, q'' = -2
        exact += -(coef[a] * (1 - 2 * ui[a]) + k_in * (-2.0)) * other
    got = fd.apply(kap, u, h, d)
    assert np.allclose(got, exact, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("d,n", [(1, 15), (2, 7), (3, 7)])
def test_sine_modes_are_eigenvectors(d, n):
    h = 1.0 / (n + 1)
    x = np.arange(1, n + 1) * h
    kap = np.full((n + 2,) * d, 1.0)
    ks = [1, 3, 2][:d]
    mode = 1.0
    for a, k in enumerate(ks):
        shape = [1] * d
        shape[a] = n
        mode = mode * np.sin(k * np.pi * x).reshape(shape)
    lam = fd.laplace_eigenvalue(ks, h)
    assert np.allclose(fd.apply(kap, mode, h, d), lam * mode, rtol=1e-12, atol=1e-10)


def test_batched_apply_and_diagonal():
    rng = np.random.default_rng(5)
    n, d = 7, 2
    h = 1.0 / (n + 1)
    kap = rng.uniform(0.5, 2.0, size=(3,) + (n + 2,) * d)
    u = rng.standard_normal((3,) + (n,) * d)
    out = fd.apply(kap, u, h, d)
    for s in range(3):
        A = fd.assemble(kap[s], n, d, h)
        assert np.allclose(out[s].ravel(), A @ u[s].ravel(), rtol=1e-13, atol=1e-10)
        assert np.allclose(fd.diagonal(kap, h, d)[s].ravel(), A.diagonal(), rtol=1e-14)
