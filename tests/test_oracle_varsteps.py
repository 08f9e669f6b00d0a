"""Pins of the oracle with non-uniform time steps tau_n (Section 2: the
partition 0 = t_0 < ... < t_N = T with tau_n = t_n - t_{n-1}; eqs. (2.1)-(2.3),
the reference pair (tau, A) of eq. (2.2), Theorem 4.1)."""
import numpy as np
import pytest

import synth
from oracle import euler, krylov, uzawa
from oracle import omega as om
from oracle import spacetime as st
from oracle.precond import Preconditioners


def graded(d, n, N, R=1, ratio=8.0, seed=3):
    steps = synth.graded_steps(N, 1.0, ratio=ratio, jitter=0.3, seed=seed)
    if d == 1:
        return synth.heat1d_random(n=n, N=N, seed=seed, steps=steps)
    return synth.small_problem(d, n, N, seed=seed, R=R, steps=steps)


def test_graded_steps_sum_and_ratio():
    s = synth.graded_steps(64, 2.0, ratio=8.0)
    assert abs(s.sum() - 2.0) < 1e-14 and abs(s[-1] / s[0] - 8.0) < 1e-12
    assert np.all(np.diff(s) > 0)
    p = graded(2, 3, 10)
    assert np.allclose(np.cumsum(p.taus)[-1], p.T) and p.tau == p.T / p.N


@pytest.mark.parametrize("d,n", [(1, 15), (2, 7)])
def test_euler_closed_form_variable_steps(d, n):
    """Spatially constant kappa(t), F = 0, u0 one sine mode: the discrete
    solution is u_n = prod_{m <= n} (1 + tau_m kappa(t_m) lambda_k)^{-1} u0."""
    prob = graded(d, n, 12)
    prob.F = np.zeros_like(prob.F)
    h = prob.h
    ks = (2, 3, 1)[:d]
    x = np.arange(1, n + 1) * h
    mode = np.ones(())
    for a in range(d):
        mode = np.multiply.outer(np.sin(ks[a] * np.pi * x), mode)
    prob.u0 = mode.reshape((n,) * d)
    lam = sum(4.0 / h ** 2 * np.sin(k * np.pi * h / 2) ** 2 for k in ks)
    kap_t = prob.tcoef[0] * prob.kfields[0].flat[0]
    fac = np.cumprod(1.0 / (1.0 + prob.taus * kap_t * lam))
    want = fac.reshape((-1,) + (1,) * d) * prob.u0[None]
    got = euler.seq_euler(prob)
    assert np.abs(got - want).max() < 1e-12 * np.abs(want).max()


@pytest.mark.parametrize("d,n,N,spatial", [(1, 15, 16, "exact"), (2, 7, 12, "mg")])
def test_uzawa_and_gmres_reach_sequential_euler(d, n, N, spatial):
    """B u = f with A = diag(tau_n A_n) and f_n = tau_n F_n (+ u0) has the
    sequential solution; both solvers reach it."""
    prob = graded(d, n, N, R=2 if d > 1 else 1)
    ref = euler.seq_euler(prob)
    pc = Preconditioners(prob, spatial=spatial)
    w = om.auto_omega(prob, spatial=spatial, pc=pc)["omega"]
    out = uzawa.uzawa(prob, omega=w, tol=1e-12, max_iter=2000, pc=pc)
    assert out["status"] == "converged"
    assert np.abs(out["u"] - ref).max() < 1e-9 * np.abs(ref).max()
    g = krylov.gmres(prob, omega=w, tol=1e-12, restart=20, max_iter=600, pc=pc)
    assert g["status"] == "converged"
    assert np.abs(g["u"] - ref).max() < 1e-9 * np.abs(ref).max()


def test_exact_spatial_solves_use_the_step_lengths():
    """With exact spatial solves A~ = A = diag(tau_n A_n), so I - A~^{-1} A = 0
    (a uniform tau in A~ would leave a contraction of the order of the step
    ratio)."""
    prob = graded(1, 15, 8, ratio=6.0)
    pc = Preconditioners(prob, spatial="exact")
    assert om.rho_A(prob, pc, m=4) < 1e-12


def alpha_of(prob):
    """Smallest alpha with (1/alpha) tau A <= tau_n A_n <= alpha tau A (eq. (2.2))."""
    import scipy.linalg as sla
    M, A_list, taus, Aref = st.fd_dense_pieces(prob)
    lo, hi = np.inf, 0.0
    for An, tn in zip(A_list, taus):
        ev = sla.eigh(tn * An, prob.tau * Aref, eigvals_only=True)
        lo, hi = min(lo, ev[0]), max(hi, ev[-1])
    return max(hi, 1.0 / lo)


@pytest.mark.parametrize("ratio", [1.0, 4.0, 16.0])
def test_theorem_4_1_bounds_with_graded_steps(ratio):
    """eig(H^{-1} S) lies in [1/(2 alpha), 3 alpha] for the reference pair
    tau = T/N, A = A(kappa_ref) (Theorem 4.1 holds for any tau_n)."""
    prob = graded(1, 7, 8, ratio=ratio, seed=5)
    M, A_list, taus, Aref = st.fd_dense_pieces(prob)
    sysm = st.dense_system(M, A_list, taus)
    H = st.dense_H(M, Aref, prob.tau, prob.N)
    ev = np.linalg.eigvals(np.linalg.solve(H, sysm["S"])).real
    a = alpha_of(prob)
    assert ev.min() >= 1.0 / (2 * a) * (1 - 1e-10) and ev.max() <= 3 * a * (1 + 1e-10), (ev.min(), ev.max(), a)
    if ratio > 1:
        assert a > 1.3          # the grading is visible in alpha


def test_reference_operator_is_step_average():
    """tau A(kappa_ref) = (1/N) sum_n tau_n A_n (reading of eq. (2.2) for
    non-uniform steps); uniform steps give the plain time mean."""
    prob = graded(2, 3, 6, R=2)
    M, A_list, taus, Aref = st.fd_dense_pieces(prob)
    avg = sum(t * A for t, A in zip(taus, A_list)) / prob.N
    assert np.allclose(prob.tau * Aref, avg, atol=1e-12 * np.abs(avg).max())
    uni = synth.small_problem(2, 3, 6, seed=3, R=2)
    assert np.array_equal(st.kref_coef(uni), uni.tcoef.mean(axis=1))
