"""Pins for Theorem 3.1 and its proof (Section 3): the iteration matrix of the
inexact Uzawa method, its factorisation, and the convergence factor rho_U of
eq. (3.5) (``spectral.rho_uzawa``).

The iteration matrix on the error e = [p* - p; u* - u] is, with Q = H~/omega
and S~ = K^T A~^{-1} K + K + K^T + A,

    Mit = [[I - A~^{-1} A,               A~^{-1} K    ],
           [-Q^{-1} K^T (I - A~^{-1} A), I - Q^{-1} S~]],

and the proof shows ||Mit||_D <= max|mu| over the generalized eigenproblem
Nmat v = mu Emat v <= rho_U, with Nmat = [[A~, -K], [-K^T, S~ - Q]],
Emat = diag(A~/rho_A, Q) and D = diag(omega rho_A A~, H~).  The bound is
attained by scalar instances in which every inequality of the proof is an
equality, which pins rho_U itself (an over- or under-estimate fails)."""
import numpy as np
import pytest
import scipy.linalg as sla

import synth
from oracle import euler, spacetime as st, spectral, uzawa
from oracle.precond import Preconditioners

from _dense import dense_vcycle


def _sqrtm_spd(D):
    w, V = np.linalg.eigh(D)
    return (V * np.sqrt(w)) @ V.T, (V / np.sqrt(w)) @ V.T


def _dnorm(Mit, D):
    Dh, Dmh = _sqrtm_spd(D)
    return np.linalg.norm(Dh @ Mit @ Dmh, 2)


def _pieces(At, A, K, Ht, omega):
    n = A.shape[0]
    I = np.eye(n)
    Ai = np.linalg.inv(At)
    Q = Ht / omega
    Qi = np.linalg.inv(Q)
    St = K.T @ Ai @ K + K + K.T + A
    Mit = np.block([[I - Ai @ A, Ai @ K], [-Qi @ K.T @ (I - Ai @ A), I - Qi @ St]])
    Nm = np.block([[At, -K], [-K.T, St - Q]])
    return Mit, Nm, St, Ai, Qi


@pytest.fixture(scope="module")
def tiny():
    """Dense pieces of a 2-D problem with time-varying kappa and one V-cycle
    in both preconditioners (the V-cycle matrices built independently)."""
    prob = synth.small_problem(2, 7, 4, seed=6)
    N = prob.N
    pc = Preconditioners(prob, spatial="mg")
    M, Al, taus, Aref = st.fd_dense_pieces(prob)
    sysd = st.dense_system(M, Al, taus)
    VA = [dense_vcycle(pc.hier, 0.0, taus[i] * prob.tcoef[:, i])[0] for i in range(N)]
    mu = 2.0 * np.sin((2 * np.arange(1, N + 1) - 1) * np.pi / (4 * N))
    VH = [dense_vcycle(pc.hier, mu[k], prob.tau * st.kref_coef(prob))[0] for k in range(N)]
    At = sla.block_diag(*[np.linalg.inv(v) for v in VA])
    Ht = st.dense_H(M, Aref, prob.tau, N, Hk_list=[np.linalg.inv(v) for v in VH])
    return dict(prob=prob, pc=pc, At=0.5 * (At + At.T), Ht=0.5 * (Ht + Ht.T), **sysd)


def test_iteration_matrix_is_one_uzawa_step(tiny):
    """One step of the oracle's iteration maps the error by Mit, and
    Mit = -Rm Nm Qm with Rm = diag(A~^{-1}, Q^{-1}), Qm = diag(A~^{-1}A - I, I)."""
    prob, omega = tiny["prob"], 0.6
    At, A, K, Ht = tiny["At"], tiny["A"], tiny["K"], tiny["Ht"]
    Mit, Nm, _, Ai, Qi = _pieces(At, A, K, Ht, omega)
    n = A.shape[0]
    Rm = sla.block_diag(Ai, Qi)
    Qm = sla.block_diag(Ai @ A - np.eye(n), np.eye(n))
    assert np.allclose(Mit, -Rm @ Nm @ Qm, atol=1e-12 * np.abs(Mit).max())
    ue = euler.seq_euler(prob).ravel()
    rng = np.random.default_rng(8)
    shape = (prob.N, prob.n, prob.n)
    p0, u0 = rng.standard_normal(shape), rng.standard_normal(shape)
    seen = []
    uzawa.uzawa(prob, omega=omega, tol=0.0, max_iter=1, pc=tiny["pc"], u_init=u0, p_init=p0,
                callback=lambda j, u, p, r: seen.append((u.copy(), p.copy())))
    # seen[0] = (u_0, p_1), seen[1] = (u_1, p_2): the step maps (p_0, u_0) to (p_1, u_1)
    e0 = np.concatenate([-ue - p0.ravel(), ue - u0.ravel()])
    e1 = np.concatenate([-ue - seen[0][1].ravel(), ue - seen[1][0].ravel()])
    assert np.allclose(e1, Mit @ e0, rtol=1e-9, atol=1e-10 * np.abs(e1).max())


@pytest.mark.parametrize("omega", [0.3, 0.6, 0.9])
def test_dnorm_bounded_by_rho_uzawa(tiny, omega):
    """||Mit||_D <= max |Sigma| <= rho_U (Lemmas of Section 3) with the
    measured rho_A and the exact extreme eigenvalues of H~^{-1} S."""
    At, A, K, Ht, S = tiny["At"], tiny["A"], tiny["K"], tiny["Ht"], tiny["S"]
    n = A.shape[0]
    # rho_A = ||I - A~^{-1} A||_{A~} = spectral radius (self-adjoint in the A~ inner product)
    rhoA = np.abs(np.linalg.eigvals(np.eye(n) - np.linalg.solve(At, A))).max()
    assert 0 < rhoA < 1
    lam = sla.eigh(S, Ht, eigvals_only=True)
    Mit, Nm, _, _, _ = _pieces(At, A, K, Ht, omega)
    Em = sla.block_diag(At / rhoA, Ht / omega)
    sig = sla.eigh(Nm, Em, eigvals_only=True)
    D = sla.block_diag(omega * rhoA * At, Ht)
    dn = _dnorm(Mit, D)
    rhoU = spectral.rho_uzawa(rhoA, omega, lam.min(), lam.max())
    assert dn <= np.abs(sig).max() * (1 + 1e-9)
    assert np.abs(sig).max() <= rhoU * (1 + 1e-9)


def _scalar_case(rhoA, omega, lam, sign):
    """1 x 1 blocks with K + K^T + A = 0 and A~ = A/(1 -+ rho_A): the proof's
    inequalities hold with equality (S~ = (1 -+ rho_A) S, Q^T E Q = D/omega)."""
    a = 1.0
    k = -a / 2
    at = a / (1 - rhoA) if sign < 0 else a / (1 + rhoA)
    S = k * k / a + 2 * k + a
    ht = S / lam                       # H~^{-1} S = lam
    M1 = lambda x: np.array([[x]])
    return M1(at), M1(a), M1(k), M1(ht)


@pytest.mark.parametrize("rhoA,omega,lam,sign", [
    (0.3, 0.5, 0.6, -1), (0.1, 0.9, 0.5, -1), (0.6, 0.2, 1.0, -1),   # sigma_- dominates
    (0.3, 0.6, 1.6, +1), (0.5, 0.4, 2.0, +1), (0.05, 1.1, 1.7, +1),  # sigma_+ dominates
])
def test_rho_uzawa_is_attained(rhoA, omega, lam, sign):
    At, A, K, Ht = _scalar_case(rhoA, omega, lam, sign)
    Mit, Nm, _, _, _ = _pieces(At, A, K, Ht, omega)
    D = sla.block_diag(omega * rhoA * At, Ht)
    Em = sla.block_diag(At / rhoA, Ht / omega)
    sig = sla.eigh(Nm, Em, eigvals_only=True)
    rhoU = spectral.rho_uzawa(rhoA, omega, lam, lam)
    assert _dnorm(Mit, D) == pytest.approx(rhoU, rel=1e-12)
    assert np.abs(sig).max() == pytest.approx(rhoU, rel=1e-12)
    # the attaining eigenvalue has the sign the proof assigns to sigma_- / sigma_+
    assert np.sign(sig[np.argmax(np.abs(sig))]) == sign


def test_rho_uzawa_exact_solves_is_richardson_rate():
    """rho_A = 0 (Remark 3.1): rho_U = max(1 - omega lam_min, omega lam_max - 1),
    the spectral radius of I - omega H^{-1} S computed densely."""
    prob = synth.small_problem(1, 7, 8, seed=5)
    M, Al, taus, Aref = st.fd_dense_pieces(prob)
    S = st.dense_system(M, Al, taus)["S"]
    H = st.dense_H(M, Aref, prob.tau, prob.N)
    lam = sla.eigh(S, H, eigvals_only=True)
    for omega in (0.5, 0.8, 1.0):
        rad = np.abs(np.linalg.eigvals(np.eye(S.shape[0]) - omega * np.linalg.solve(H, S))).max()
        assert spectral.rho_uzawa(0.0, omega, lam.min(), lam.max()) == pytest.approx(rad, rel=1e-10)
