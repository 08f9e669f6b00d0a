"""Pins for the oracle's two preconditioners against dense assembly.

* H-tilde^{-1} (eq. (4.6)): the matrix-free Phi^{-1} Hhat_approx^{-1} Phi^{-T}
  of ``Preconditioners.Hinv`` against a dense solve with
  H-tilde = Phi^T (N/2tau) diag(H~_k A^{-1} H~_k) Phi assembled from its
  definition, with exact H_k = mu_k I + tau A_ref (eq. (4.5)) and with H~_k the
  inverse of the dense V-cycle matrix (built independently in ``_dense``);
  time-varying coefficients and graded steps.
* A-tilde^{-1} (eq. (3.2)): block-diagonal dense solves with tau_n A_n or the
  dense V-cycle matrices of tau_n A_n."""
import numpy as np
import pytest
import scipy.linalg as sla

import synth
from oracle import spacetime as st
from oracle.precond import Preconditioners

from _dense import dense_vcycles


def _problem(d, n, N, graded, R=2, seed=21):
    steps = synth.graded_steps(N, ratio=6.0, jitter=0.3, seed=seed) if graded else None
    return synth.small_problem(d, n, N, seed=seed, R=R, steps=steps)


CASES = [(1, 15, 8, False), (2, 7, 8, False), (2, 7, 6, True), (3, 3, 4, False), (3, 3, 5, True)]


@pytest.mark.parametrize("d,n,N,graded", CASES)
def test_Hinv_exact_equals_dense_solve(d, n, N, graded):
    prob = _problem(d, n, N, graded)
    M, _, _, Aref = st.fd_dense_pieces(prob)
    H = st.dense_H(M, Aref, prob.tau, N)
    r = np.random.default_rng(3).standard_normal((N,) + (n,) * d)
    want = np.linalg.solve(H, r.ravel())
    got = Preconditioners(prob, spatial="exact").Hinv(r)
    assert np.allclose(got.ravel(), want, rtol=1e-10, atol=1e-12 * np.abs(want).max())


@pytest.mark.parametrize("d,n,N,graded", CASES)
@pytest.mark.parametrize("nu", [1, 2])
def test_Hinv_multigrid_equals_dense_solve(d, n, N, graded, nu):
    prob = _problem(d, n, N, graded)
    pc = Preconditioners(prob, spatial="mg", nu_H=nu)
    M, _, _, Aref = st.fd_dense_pieces(prob)
    mu = 2.0 * np.sin((2 * np.arange(1, N + 1) - 1) * np.pi / (4 * N))    # eq. (4.5)
    cH = prob.tau * st.kref_coef(prob)
    Hk = [np.linalg.inv(dense_vcycles(pc.hier, mu[k], cH, nu)) for k in range(N)]
    H = st.dense_H(M, Aref, prob.tau, N, Hk_list=Hk)
    r = np.random.default_rng(4).standard_normal((N,) + (n,) * d)
    want = np.linalg.solve(H, r.ravel())
    got = pc.Hinv(r)
    assert np.allclose(got.ravel(), want, rtol=1e-9, atol=1e-11 * np.abs(want).max())
    # H~ is symmetric positive definite (Theorem 3.1's assumption)
    assert np.allclose(H, H.T, atol=1e-10 * np.abs(H).max())
    assert np.linalg.eigvalsh(0.5 * (H + H.T)).min() > 0


@pytest.mark.parametrize("d,n,N,graded", CASES)
@pytest.mark.parametrize("spatial,nu", [("exact", 1), ("mg", 1), ("mg", 2)])
def test_Ainv_equals_block_dense_solve(d, n, N, graded, spatial, nu):
    prob = _problem(d, n, N, graded)
    pc = Preconditioners(prob, spatial=spatial, nu_A=nu)
    _, A_list, taus, _ = st.fd_dense_pieces(prob)
    if spatial == "exact":
        blocks = [np.linalg.inv(taus[i] * A_list[i]) for i in range(N)]
    else:
        blocks = [dense_vcycles(pc.hier, 0.0, taus[i] * prob.tcoef[:, i], nu) for i in range(N)]
    r = np.random.default_rng(5).standard_normal((N,) + (n,) * d)
    want = sla.block_diag(*blocks) @ r.ravel()
    got = pc.Ainv(r)
    assert np.allclose(got.ravel(), want, rtol=1e-9, atol=1e-11 * np.abs(want).max())
