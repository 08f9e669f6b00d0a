"""Pins for the time-global formulation (Sections 2, 4, 6, 7) on tiny dense systems."""
import numpy as np
import pytest
import scipy.linalg as sla

import synth
from oracle import dst, euler, fem1d, spacetime as st


def _fd(d, n, N, seed=3):
    prob = synth.small_problem(d, n, N, seed=seed)
    M, Al, taus, Aref = st.fd_dense_pieces(prob)
    return prob, M, Al, taus, Aref


@pytest.mark.parametrize("d,n,N", [(1, 5, 6), (2, 3, 5), (3, 3, 3)])
def test_saddle_structure(d, n, N):
    prob, M, Al, taus, Aref = _fd(d, n, N)
    D = st.dense_system(M, Al, taus)
    S, sad, B, K, A = D["S"], D["saddle"], D["B"], D["K"], D["A"]
    m = n ** d
    # symmetry of the saddle-point matrix and of S (eqs. (2.5), (2.7))
    assert np.array_equal(sad, sad.T)
    assert np.allclose(S, S.T, rtol=1e-12, atol=1e-9 * np.abs(S).max())
    # S = K^T A^{-1} K + K + K^T + A
    S2 = K.T @ np.linalg.solve(A, K) + K + K.T + A
    assert np.allclose(S, S2, rtol=1e-11, atol=1e-10 * np.abs(S).max())
    # the Schur complement of the saddle matrix is -S (the paper calls S "the" Schur complement)
    sch = sad[N * m:, N * m:] - sad[N * m:, :N * m] @ np.linalg.solve(sad[:N * m, :N * m], sad[:N * m, N * m:])
    assert np.allclose(sch, -S, rtol=1e-10, atol=1e-9 * np.abs(S).max())
    # inertia: N*m positive and N*m negative eigenvalues
    ev = np.linalg.eigvalsh(sad)
    assert (ev > 0).sum() == N * m and (ev < 0).sum() == N * m
    # solution: second block = B^{-1} f = sequential Euler, first block p = -u
    f = st.rhs(prob).ravel()
    sol = np.linalg.solve(sad, np.concatenate([-f, -f]))
    ue = euler.seq_euler(prob).ravel()
    assert np.allclose(sol[N * m:], ue, rtol=1e-9, atol=1e-11)
    assert np.allclose(sol[:N * m], -ue, rtol=1e-9, atol=1e-11)
    # matrix-free operators agree with the dense ones
    rng = np.random.default_rng(0)
    x = rng.standard_normal((N,) + (n,) * d)
    y = rng.standard_normal((N,) + (n,) * d)
    assert np.allclose(st.apply_B(prob, x).ravel(), B @ x.ravel(), rtol=1e-12, atol=1e-9)
    top, bot = st.apply_saddle(prob, x, y)
    ref = sad @ np.concatenate([x.ravel(), y.ravel()])
    assert np.allclose(np.concatenate([top.ravel(), bot.ravel()]), ref, rtol=1e-12, atol=1e-9)


@pytest.mark.parametrize("d,n,N", [(1, 5, 7), (2, 3, 4)])
def test_S_norm_identity_and_max_norm(d, n, N):
    """Theorem 6.2 (eq. (6.11)-(6.14)) in matrix form with M = I:
    v^T S v = sum_n [ (1/tau)|dv_n|^2_{A_n^{-1}} + tau |v_n|^2_{A_n} + |dv_n|^2 ] + |v_N|^2,
    dv_n = v_n - v_{n-1} (v_0 = 0); and Corollary 6.3: max_n |v_n| <= |v|_S."""
    prob, M, Al, taus, Aref = _fd(d, n, N)
    S = st.dense_system(M, Al, taus)["S"]
    rng = np.random.default_rng(1)
    for _ in range(5):
        v = rng.standard_normal((N, n ** d))
        dv = np.diff(np.vstack([np.zeros((1, n ** d)), v]), axis=0)
        s = sum(dv[i] @ np.linalg.solve(Al[i], dv[i]) / taus[i] + taus[i] * v[i] @ Al[i] @ v[i] + dv[i] @ dv[i]
                for i in range(N)) + v[-1] @ v[-1]
        vSv = v.ravel() @ S @ v.ravel()
        assert abs(s - vSv) <= 1e-11 * abs(vSv)
        assert np.max(np.linalg.norm(v, axis=1)) <= np.sqrt(vSv)


def test_inf_sup_identity():
    """eq. (2.6): sup_v v^T B u / |v|_A = |u|_S, attained at v = P u."""
    prob, M, Al, taus, Aref = _fd(2, 3, 4)
    D = st.dense_system(M, Al, taus)
    B, A, P, S = D["B"], D["A"], D["P"], D["S"]
    rng = np.random.default_rng(2)
    u = rng.standard_normal(B.shape[0])
    Lc = np.linalg.cholesky(A)
    # sup over v of v^T B u / |v|_A = |A^{-1/2} B u|  (= |Bu|_{A^{-1}})
    sup = np.sqrt((B @ u) @ np.linalg.solve(A, B @ u))
    assert abs(sup - np.sqrt(u @ S @ u)) <= 1e-11 * sup
    v = P @ u
    assert abs((v @ B @ u) / np.sqrt(v @ A @ v) - sup) <= 1e-11 * sup
    for _ in range(20):
        w = rng.standard_normal(B.shape[0])
        assert (w @ B @ u) / np.sqrt(w @ A @ w) <= sup * (1 + 1e-12)
    del Lc


def test_mixed_inf_sup_bounds():
    """eq. (2.8): singular values of the saddle matrix in the |.|_* norm
    (blocks A and S) lie in [(sqrt5-1)/2, (sqrt5+1)/2]."""
    prob, M, Al, taus, Aref = _fd(1, 5, 6)
    D = st.dense_system(M, Al, taus)
    Dn = sla.block_diag(D["A"], D["S"])
    L = np.linalg.cholesky(Dn)
    Li = np.linalg.inv(L)
    sv = np.linalg.svd(Li @ D["saddle"] @ Li.T, compute_uv=False)
    assert sv.min() >= (np.sqrt(5) - 1) / 2 - 1e-10
    assert sv.max() <= (np.sqrt(5) + 1) / 2 + 1e-10


def test_example_constant_coefficients():
    """Example 4.1: uniform steps, A_n = A: S = (1/tau) K^T K (x) M A^{-1} M
    + (K + K^T) (x) M + tau I (x) A, with the printed tridiagonal K^T K and K + K^T."""
    n, N, tau = 6, 5, 0.2
    M, A = fem1d.mass(n), fem1d.stiffness(n)
    S = st.dense_system(M, [A] * N, [tau] * N)["S"]
    K = st.Kmat(N)
    KtK = 2 * np.eye(N) - np.eye(N, k=1) - np.eye(N, k=-1)
    KtK[-1, -1] = 1
    KpKt = 2 * np.eye(N) - np.eye(N, k=1) - np.eye(N, k=-1)
    assert np.array_equal(K.T @ K, KtK) and np.array_equal(K + K.T, KpKt)
    S2 = np.kron(KtK, M @ np.linalg.solve(A, M)) / tau + np.kron(KpKt, M) + tau * np.kron(np.eye(N), A)
    assert np.allclose(S, S2, rtol=1e-12, atol=1e-12 * np.abs(S).max())


@pytest.mark.parametrize("d,n,N", [(1, 7, 8), (2, 3, 6)])
def test_spectral_equivalence_theorem(d, n, N):
    """Theorem 4.1: (1/2 alpha) H <= S <= 3 alpha H, with alpha from eq. (2.2),
    and the intermediate S_dagger = Phi^T Dhat Phi satisfies H/2 <= S_dagger <= H."""
    prob, M, Al, taus, Aref = _fd(d, n, N)
    tau = prob.tau
    S = st.dense_system(M, Al, taus)["S"]
    H = st.dense_H(M, Aref, tau, N)
    a = []
    for An in Al:
        e = sla.eigh(An, Aref, eigvals_only=True)
        a += [e.min(), e.max()]
    alpha = max(max(a), 1.0 / min(a))
    ev = sla.eigh(S, H, eigvals_only=True)
    assert ev.min() >= 1 / (2 * alpha) - 1e-10 and ev.max() <= 3 * alpha + 1e-10
    Ainv = np.linalg.inv(Aref)
    mu = dst.mu(N)
    Dhat = sla.block_diag(*[(N / 2) * (mu[k] ** 2 / tau * M @ Ainv @ M + tau * Aref) for k in range(N)])
    Phi = np.kron(dst.phi_matrix(N), np.eye(M.shape[0]))
    Sd = Phi.T @ Dhat @ Phi
    ev2 = sla.eigh(Sd, H, eigvals_only=True)
    assert ev2.min() >= 0.5 - 1e-10 and ev2.max() <= 1 + 1e-10


def test_pearson_wathen_lemma():
    """Lemma 7.4 for random SPD M, A and lambda >= 0."""
    rng = np.random.default_rng(4)
    for _ in range(5):
        X = rng.standard_normal((6, 6))
        Y = rng.standard_normal((6, 6))
        M = X @ X.T + 0.1 * np.eye(6)
        A = Y @ Y.T + 0.1 * np.eye(6)
        lam = rng.uniform(0, 10)
        Ai = np.linalg.inv(A)
        num = M @ Ai @ M + lam * A
        den = (M + np.sqrt(lam) * A) @ Ai @ (M + np.sqrt(lam) * A)
        ev = sla.eigh(num, den, eigvals_only=True)
        assert ev.min() >= 0.5 - 1e-10 and ev.max() <= 1 + 1e-10


def test_manufactured_source_has_closed_form_solution():
    """The manufactured source of the 3-D lognormal workloads,
    F_n = (u*_n - u*_{n-1})/tau + A_n u*_n with u*_n = exp(-3 pi^2 t_n) S(x),
    makes u* the exact solution of implicit Euler (eq. 2.1): checked against the
    oracle's sequential stepping, which shares no code with the construction
    beyond the spatial operator."""
    from oracle import euler, fd
    prob = synth.heat3d_lognormal(n=7, N=6, seed=3, contrast=1e2, source="none")
    S = prob.u0
    tau = prob.tau
    e = np.exp(-3 * np.pi ** 2 * tau * np.arange(prob.N + 1))
    AS = fd.apply(prob.kfields[0], S, prob.h, 3)
    prob.F = np.multiply.outer((e[1:] - e[:-1]) / tau, S) + np.multiply.outer(prob.tcoef[0] * e[1:], AS)
    ue = euler.seq_euler(prob)
    us = np.multiply.outer(e[1:], S)
    assert np.abs(ue - us).max() < 1e-13 * np.abs(us).max()


@pytest.mark.parametrize("d,n,N", [(1, 5, 7), (2, 3, 4)])
def test_s_norm_matches_dense_S(d, n, N):
    """The matrix-free ||v||_S equals sqrt(v^T S v) with S assembled densely
    (eq. (2.5)), also with non-uniform steps."""
    steps = synth.graded_steps(N, 1.0, ratio=5.0, jitter=0.2, seed=n)
    for st_ in (None, steps):
        prob = synth.heat1d_random(n=n, N=N, seed=4, steps=st_) if d == 1 else \
            synth.small_problem(d, n, N, seed=4, steps=st_)
        M, Al, taus, Aref = st.fd_dense_pieces(prob)
        S = st.dense_system(M, Al, taus)["S"]
        v = np.random.default_rng(2).standard_normal((N,) + (n,) * d)
        want = np.sqrt(v.ravel() @ S @ v.ravel())
        assert abs(st.s_norm(prob, v) - want) <= 1e-11 * want
