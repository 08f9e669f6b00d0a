"""Pins for the oracle's inexact Uzawa iteration (Section 3, eq. (3.1); Theorem 3.1)."""
import numpy as np
import pytest
import scipy.linalg as sla

import synth
from oracle import dst, euler, mg, spacetime as st, spectral, uzawa
from oracle.precond import Preconditioners


@pytest.mark.parametrize("d,n,N,spatial", [(1, 63, 64, "exact"), (1, 31, 16, "mg"),
                                           (2, 15, 16, "mg"), (2, 7, 8, "exact"), (3, 7, 8, "mg")])
def test_converges_to_sequential_euler(d, n, N, spatial):
    prob = synth.heat1d_random(n=n, N=N) if d == 1 else synth.small_problem(d, n, N)
    res = uzawa.uzawa(prob, omega=0.7, tol=1e-10, spatial=spatial, max_iter=400)
    assert res["status"] == "converged"
    ue = euler.seq_euler(prob)
    err = np.linalg.norm(res["u"] - ue) / np.linalg.norm(ue)
    assert err < 1e-8
    # auxiliary variable tends to -u (Section 2.1)
    assert np.linalg.norm(res["p"] + res["u"]) / np.linalg.norm(ue) < 1e-7
    # residual history decreases overall
    h = res["history"]
    assert h[-1] <= 1e-10 and h[0] > h[-1]


def test_exact_solves_is_preconditioned_richardson():
    """Remark 3.1: with exact A-tilde the iteration is Richardson on S with H;
    the H-norm error contracts by at most max|1 - omega lambda| each step and
    asymptotically by that factor."""
    prob = synth.small_problem(1, 7, 8, seed=5)
    M, Al, taus, Aref = st.fd_dense_pieces(prob)
    S = st.dense_system(M, Al, taus)["S"]
    H = st.dense_H(M, Aref, prob.tau, prob.N)
    lam = sla.eigh(S, H, eigvals_only=True)
    omega = 0.8
    rho = max(abs(1 - omega * lam.min()), abs(1 - omega * lam.max()))
    ue = euler.seq_euler(prob).ravel()
    errs = []

    def cb(j, u, p, r):
        e = ue - u.ravel()
        errs.append(np.sqrt(e @ H @ e))
    uzawa.uzawa(prob, omega=omega, tol=0.0, max_iter=80, spatial="exact", callback=cb)
    ratios = np.array(errs[1:]) / np.array(errs[:-1])
    assert ratios.max() <= rho * (1 + 1e-8)
    tail = (errs[-1] / errs[-21]) ** (1 / 20)
    assert tail > 0.97 * rho


def test_theorem_3_1_contraction():
    """Theorem 3.1 with V-cycles: ||e_{j+1}||_D <= rho_U ||e_j||_D where
    ||(q, v)||_D^2 = omega rho_A ||q||_{A~}^2 + ||v||_{H~}^2."""
    prob = synth.small_problem(2, 7, 4, seed=6)
    N, m, tau = prob.N, prob.npts, prob.tau
    pc = Preconditioners(prob, spatial="mg")
    M, Al, taus, Aref = st.fd_dense_pieces(prob)
    D = st.dense_system(M, Al, taus)
    S = D["S"]
    # dense V-cycle matrices
    I = np.eye(m).reshape((m,) + (prob.n,) * 2)

    def vmat(sig, c):
        return pc.hier.vcycles(np.full(m, sig), np.tile(c, (m, 1)), I).reshape(m, m).T
    VA = [vmat(pc.sigA[i], pc.cA[i]) for i in range(N)]
    VH = [vmat(pc.sigH[k], pc.cH[k]) for k in range(N)]
    Atil = sla.block_diag(*[np.linalg.inv(v) for v in VA])        # diag(tau_n A~_n)
    Hk = [np.linalg.inv(v) for v in VH]
    Htil = st.dense_H(M, Aref, tau, N, Hk_list=Hk)
    rhoA = max(np.abs(np.linalg.eigvals(np.eye(m) - VA[i] @ (taus[i] * Al[i]))).max() for i in range(N))
    lam = sla.eigh(S, Htil, eigvals_only=True)
    # damping condition (3.7): omega lambda_max < 2 (1 - rho_A) / (1 + rho_A); take 80 % of the limit
    omega = 0.8 * 2 * (1 - rhoA) / ((1 + rhoA) * lam.max())
    rhoU = spectral.rho_uzawa(rhoA, omega, lam.min(), lam.max())
    assert rhoU < 1
    ue = euler.seq_euler(prob).ravel()
    Dm = sla.block_diag(omega * rhoA * Atil, Htil)
    states = []

    def cb(j, u, p, r):
        states.append((u.copy(), p.copy()))
    uzawa.uzawa(prob, omega=omega, tol=0.0, max_iter=25, pc=pc, callback=cb)
    norms = []
    # states[j] = (u_j, p_{j+1}); theorem iterate j+1 = (p_{j+1}, u_{j+1}) = (states[j][1], states[j+1][0])
    for j in range(len(states) - 1):
        p_, u_ = states[j][1], states[j + 1][0]
        e = np.concatenate([-ue - p_.ravel(), ue - u_.ravel()])
        norms.append(np.sqrt(e @ Dm @ e))
    ratios = np.array(norms[1:]) / np.array(norms[:-1])
    assert ratios.max() <= rhoU * (1 + 1e-9)


def test_iterations_flat_in_N():
    """Iteration counts stay bounded as N grows (Theorem 4.1 / Table 2 pattern)."""
    its = []
    for N in [16, 64, 256]:
        prob = synth.heat1d_random(n=31, N=N)
        its.append(uzawa.uzawa(prob, omega=0.7, tol=1e-8, spatial="exact")["iters"])
    assert max(its) - min(its) <= 6, its
    assert max(its) < 60


def test_zero_right_hand_side_stops_at_once():
    """f = 0 (F = 0, u0 = 0): the solution is zero and the absolute residual
    test stops at iteration 0; from a nonzero guess the iterates tend to 0."""
    prob = synth.small_problem(2, 7, 4, seed=9)
    prob.F = np.zeros_like(prob.F)
    prob.u0 = np.zeros_like(prob.u0)
    res = uzawa.uzawa(prob, omega=0.7, tol=1e-10)
    assert res["status"] == "converged" and res["iters"] == 0 and res["history"][0] == 0.0
    g = np.random.default_rng(1).standard_normal(res["u"].shape)
    res = uzawa.uzawa(prob, omega=0.7, tol=1e-10, u_init=g, max_iter=400)
    assert res["status"] == "converged" and np.abs(res["u"]).max() < 1e-8 * np.abs(g).max()
