"""Pins for the time transforms of Section 4 (eqs. (4.2), (4.3), (4.5), (7.5))."""
import numpy as np
import pytest
import scipy.fft as sfft

from oracle import dst


@pytest.mark.parametrize("N", [1, 2, 3, 7, 16, 64, 100])
def test_discrete_orthogonality(N):
    """Lemma 7.3: sum_n w_n phi_k^n phi_j^n = (N/2) delta_kj and
    sum_n (phi_k^n - phi_k^{n-1})(phi_j^n - phi_j^{n-1}) = (N/2) mu_k^2 delta_kj."""
    S = dst.sine_matrix(N)
    w = dst.weights(N)
    G = S.T @ (w[:, None] * S)
    assert np.allclose(G, (N / 2) * np.eye(N), atol=1e-12 * N)
    Sp = np.vstack([np.zeros((1, N)), S])
    D = np.diff(Sp, axis=0)
    assert np.allclose(D.T @ D, (N / 2) * np.diag(dst.mu(N) ** 2), atol=1e-12 * N)


@pytest.mark.parametrize("N", [1, 5, 64, 257])
def test_inverse_pair(N):
    rng = np.random.default_rng(N)
    u = rng.standard_normal((N, 3))
    assert np.allclose(dst.inverse(dst.forward(u)), u, atol=1e-12)
    assert np.allclose(dst.forward(dst.inverse(u)), u, atol=1e-12)


@pytest.mark.parametrize("N", [1, 2, 5, 64, 1021])
def test_library_dst_mapping(N):
    """Reduction to scipy's unnormalised DST types II/III:
    Phi^{-T} r = dst3(r with r_N doubled)/2,  Phi^{-1} y = dst2(y)/2,  Phi r = dst3(r)/N."""
    rng = np.random.default_rng(N + 1)
    r = rng.standard_normal(N)
    r2 = r.copy()
    r2[-1] *= 2
    tol = 1e-13 * N
    assert np.allclose(dst.inverse_transpose(r), 0.5 * sfft.dst(r2, type=3), atol=tol)
    assert np.allclose(dst.inverse(r), 0.5 * sfft.dst(r, type=2), atol=tol)
    assert np.allclose(dst.forward(r), sfft.dst(r, type=3) / N, atol=tol)


@pytest.mark.parametrize("N", [4097, 8192])
def test_large_N_route_equals_definition(N):
    """Above DENSE_MAX_N the oracle evaluates the maps through the library DST;
    compare with the dense sums (sine matrix built here) on a few columns."""
    assert N > dst.DENSE_MAX_N
    rng = np.random.default_rng(N)
    r = rng.standard_normal((N, 2))
    S = dst.sine_matrix(N)
    tol = 1e-13 * N
    assert np.allclose(dst.inverse(r), S @ r, atol=tol)
    assert np.allclose(dst.inverse_transpose(r), S.T @ r, atol=tol)
    assert np.allclose(dst.forward(r), (2.0 / N) * S.T @ (dst.weights(N)[:, None] * r), atol=tol)


def test_mu_positive_and_bounded():
    for N in [1, 4, 1000]:
        m = dst.mu(N)
        assert (m > 0).all() and (m < 2).all()
        assert np.all(np.diff(m) > 0)
