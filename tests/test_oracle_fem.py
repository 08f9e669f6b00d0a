"""Pins for the oracle's finite-element matrices, multigrid and space-time
method with a general mass matrix (Section 2; the elements of Section 8)."""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import dst, fem, fem1d
from oracle import spacetime as st


def test_p1_1d_equals_closed_forms():
    M, A = fem.matrices(1, 9)
    assert np.allclose(M.toarray(), fem1d.mass(9), atol=1e-15)
    assert np.allclose(A.toarray(), fem1d.stiffness(9), atol=1e-13)


def test_q1_3d_sine_modes_are_generalized_eigenvectors():
    """Q1 on a uniform mesh: M and A are tensor products of the 1-D P1
    matrices, so each sine mode is an eigenvector of both with eigenvalues
    prod_a m(k_a) and sum_a a(k_a) prod_{b != a} m(k_b),
    m(k) = (h/3)(2 + cos k pi h), a(k) = (2/h)(1 - cos k pi h)."""
    n = 7
    h = 1.0 / (n + 1)
    M, A = fem.matrices(3, n)
    for ks in [(1, 1, 1), (2, 5, 3), (7, 1, 4)]:
        v = np.einsum("i,j,k->ijk", *[np.sin(k * np.pi * np.arange(1, n + 1) * h) for k in reversed(ks)]).ravel()
        m = [(h / 3) * (2 + np.cos(k * np.pi * h)) for k in ks]
        a = [(2 / h) * (1 - np.cos(k * np.pi * h)) for k in ks]
        assert np.allclose(M @ v, np.prod(m) * v, atol=1e-14)
        lam_A = a[0] * m[1] * m[2] + m[0] * a[1] * m[2] + m[0] * m[1] * a[2]
        assert np.allclose(A @ v, lam_A * v, atol=1e-12)


def test_p1_2d_stencils():
    """P1 on the lower-left/upper-right triangulation: the stiffness is the
    5-point Laplacian (4, -1) and the mass stencil (h^2/12)(6; 1 on the E, W,
    N, S, NE and SW neighbours)."""
    n = 7
    h = 1.0 / (n + 1)
    M, A = fem.matrices(2, n)
    M, A = M.toarray(), A.toarray()
    idx = lambda x, y: (y - 1) * n + (x - 1)   # noqa: E731
    c = idx(4, 4)
    wantA = {idx(4, 4): 4.0, idx(3, 4): -1.0, idx(5, 4): -1.0, idx(4, 3): -1.0, idx(4, 5): -1.0}
    wantM = {idx(4, 4): 6.0, idx(3, 4): 1.0, idx(5, 4): 1.0, idx(4, 3): 1.0, idx(4, 5): 1.0,
             idx(5, 5): 1.0, idx(3, 3): 1.0}
    for j in range(n * n):
        assert A[c, j] == pytest.approx(wantA.get(j, 0.0), abs=1e-13)
        assert M[c, j] == pytest.approx(h * h / 12 * wantM.get(j, 0.0), abs=1e-16)
    assert np.allclose(M, M.T) and np.allclose(A, A.T)


@pytest.mark.parametrize("d,n", [(1, 15), (2, 15), (3, 7)])
def test_galerkin_coarse_operator_is_the_coarse_mesh_operator(d, n):
    """Nested meshes and interpolation prolongation: R L_h P = L_{2h} / 2^d
    with R = P^T / 2^d (so the coarse levels are the element operators of the
    coarse meshes, scaled)."""
    H = fem.Hierarchy(d, n)
    Mc, Ac = fem.matrices(d, (n - 1) // 2)
    assert abs(H.M[1] - Mc / 2 ** d).max() < 1e-15
    assert abs(H.A[1] - Ac / 2 ** d).max() < 1e-13
    # P reproduces linear functions on the coarse cells away from the boundary
    P = fem.prolongation(d, n)
    nc = (n - 1) // 2
    hc = 1.0 / (nc + 1)
    xc = np.arange(1, nc + 1) * hc
    xf = np.arange(1, n + 1) / (n + 1)
    gc = np.meshgrid(*([xc] * d), indexing="ij")
    gf = np.meshgrid(*([xf] * d), indexing="ij")
    lin_c = sum((a + 1) * g for a, g in enumerate(gc)).ravel()
    lin_f = sum((a + 1) * g for a, g in enumerate(gf)).ravel()
    inner = np.all([(g >= hc - 1e-12) & (g <= 1 - hc + 1e-12) for g in gf], axis=0).ravel()
    assert np.allclose((P @ lin_c)[inner], lin_f[inner])


@pytest.mark.parametrize("d,n", [(2, 31), (3, 15)])
def test_vcycle_symmetric_and_contracting(d, n):
    H = fem.Hierarchy(d, n)
    m = n ** d
    rng = np.random.default_rng(d)
    for sig, c, bound in [(0.0, 1.0, 0.5), (1.0, 1e-3, 0.5), (1.0, 1e3, 0.5), (1.0, 1e-5, 0.9)]:
        L = sig * H.M[0] + c * H.A[0]
        x, y = rng.standard_normal(m), rng.standard_normal(m)
        assert x @ H.vcycle(sig, c, y) == pytest.approx(y @ H.vcycle(sig, c, x), rel=1e-11)
        e = rng.standard_normal(m)
        for _ in range(25):
            en = e - H.vcycle(sig, c, L @ e)
            rate = np.sqrt(en @ (L @ en) / (e @ (L @ e)))
            e = en / np.linalg.norm(en)
        assert rate < bound, (sig, c, rate)   # mass-dominated operators: weaker, still contracting


def test_vcycle_matches_dense_construction():
    """One cycle equals the dense error-propagation matrix
    (I - W L)(I - P V_c R L)(I - W L) with the Galerkin coarse cycle."""
    d, n = 2, 7
    H = fem.Hierarchy(d, n)
    sig, c = 0.6, 0.02

    def dense(l):
        L = (sig * H.M[l] + c * H.A[l]).toarray()
        if l == len(H.ns) - 1:
            return np.linalg.inv(np.diag(np.diag(L))), L
        W = fem.L1_THETA / np.abs(L).sum(axis=1).max() * np.eye(L.shape[0])
        P = H.P[l].toarray()
        Vc, _ = dense(l + 1)
        I = np.eye(L.shape[0])
        E = (I - W @ L) @ (I - P @ Vc @ (P.T / 2 ** d) @ L) @ (I - W @ L)
        return (I - E) @ np.linalg.inv(L), L
    V, _ = dense(0)
    b = np.random.default_rng(3).standard_normal(n * n)
    assert np.allclose(H.vcycle(sig, c, b), V @ b, rtol=1e-11, atol=1e-13)


def _problem(d, n, N, seed=0, T=1.0):
    rng = np.random.default_rng(seed)
    t = T * np.arange(1, N + 1) / N
    return fem.FemProblem(d, n, N, T, 1.0 + 0.5 * np.sin(2 * np.pi * t + 0.3),
                          rng.standard_normal((N, n ** d)), rng.standard_normal(n ** d))


def test_sequential_euler_sine_mode_decay():
    """F = 0, u0 a sine mode (Q1, 3-D): u_n = prod_{m<=n} (1 + tau a_m lambda)^{-1} u0
    with lambda the generalized eigenvalue A v = lambda M v."""
    n, N = 7, 6
    h = 1.0 / (n + 1)
    prob = _problem(3, n, N)
    ks = (2, 1, 3)
    v = np.einsum("i,j,k->ijk", *[np.sin(k * np.pi * np.arange(1, n + 1) * h) for k in reversed(ks)]).ravel()
    prob.F[:] = 0.0
    prob.u0 = v
    m = [(h / 3) * (2 + np.cos(k * np.pi * h)) for k in ks]
    a = [(2 / h) * (1 - np.cos(k * np.pi * h)) for k in ks]
    lam = (a[0] * m[1] * m[2] + m[0] * a[1] * m[2] + m[0] * m[1] * a[2]) / np.prod(m)
    fac = np.cumprod(1.0 / (1.0 + prob.tau * prob.a * lam))
    assert np.allclose(fem.seq_euler(prob), fac[:, None] * v, rtol=1e-12, atol=1e-14)


def test_time_global_system_with_mass_matrix():
    """The sequential solution satisfies B u = f with K = bidiag (x) M (eq. (2.3)),
    and matches the dense assembly of the time-global system."""
    prob = _problem(2, 7, 5)
    M, A = fem.matrices(2, 7)
    u = fem.seq_euler(prob)
    f = fem.rhs(prob, M)
    assert np.linalg.norm(fem.apply_B(prob, M, A, u) - f) <= 1e-13 * np.linalg.norm(f)
    D = st.dense_system(M.toarray(), [prob.a[i] * A.toarray() for i in range(prob.N)], [prob.tau] * prob.N)
    assert np.allclose(D["B"] @ u.ravel(), f.ravel(), rtol=1e-12, atol=1e-13 * np.abs(f).max())


def test_Hinv_equals_dense_solve():
    """H-tilde^{-1} with exact spatial solves = dense solve with
    H = Phi^T (N/2tau) diag(H_k A^{-1} H_k) Phi, H_k = mu_k M + tau a_ref A."""
    prob = _problem(2, 7, 6)
    M, A = fem.matrices(2, 7)
    pc = fem.Preconditioners(prob, spatial="exact")
    H = st.dense_H(M.toarray(), np.mean(prob.a) * A.toarray(), prob.tau, prob.N)
    r = np.random.default_rng(2).standard_normal((prob.N, 49))
    assert np.allclose(pc.Hinv(r).ravel(), np.linalg.solve(H, r.ravel()), rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("d,n,N,spatial", [(1, 31, 16, "exact"), (2, 15, 12, "mg"), (3, 7, 8, "mg"),
                                           (2, 7, 8, "exact")])
def test_uzawa_converges_to_sequential_euler(d, n, N, spatial):
    prob = _problem(d, n, N, seed=d)
    res = fem.uzawa(prob, omega=0.7, tol=1e-11, max_iter=500, spatial=spatial)
    assert res["status"] == "converged"
    ue = fem.seq_euler(prob)
    assert np.linalg.norm(res["u"] - ue) / np.linalg.norm(ue) < 1e-9


@pytest.mark.parametrize("sweeps", [2, 3])
def test_vcycle_with_several_sweeps_matches_dense(sweeps):
    """s sweeps per side: E = (I - W L)^s (I - P V_c R L)(I - W L)^s."""
    d, n = 3, 7
    H = fem.Hierarchy(d, n)
    sig, c = 0.3, 0.05

    def dense(l):
        L = (sig * H.M[l] + c * H.A[l]).toarray()
        if l == len(H.ns) - 1:
            return np.linalg.inv(np.diag(np.diag(L))), L
        W = fem.L1_THETA / np.abs(L).sum(axis=1).max() * np.eye(L.shape[0])
        P = H.P[l].toarray()
        Vc, _ = dense(l + 1)
        I = np.eye(L.shape[0])
        S = np.linalg.matrix_power(I - W @ L, sweeps)
        E = S @ (I - P @ Vc @ (P.T / 2 ** d) @ L) @ S
        return (I - E) @ np.linalg.inv(L), L
    V, _ = dense(0)
    b = np.random.default_rng(4).standard_normal(n ** d)
    assert np.allclose(H.vcycle(sig, c, b, sweeps=sweeps), V @ b, rtol=1e-10, atol=1e-12)


def test_table2_with_p1_elements():
    """Section 8.2 with P1 elements (2-D, T = 1, u(0) = sin sin, F = 0,
    omega = 0.9): iterations to ||u - u_j||_S < 1e-6 ||u||_S.  Exact spatial
    solves need 19; one V-cycle with three Jacobi sweeps per side needs 20-21
    (the paper prints 20-22 for one V-cycle, smoothing unstated), equal for
    h = 1/8 and 1/16."""
    def count(n, N, spatial, sweeps=1):
        x = np.arange(1, n + 1) / (n + 1)
        prob = fem.FemProblem(2, n, N, 1.0, np.ones(N), np.zeros((N, n * n)),
                              np.outer(np.sin(np.pi * x), np.sin(np.pi * x)).ravel())
        ue = fem.seq_euler(prob)
        sc = fem.s_norm(prob, ue)
        us = fem.stationary(prob, fem.Preconditioners(prob, spatial, sweeps=sweeps), 0.9, 30)
        return next(k for k, u in enumerate(us) if fem.s_norm(prob, ue - u) / sc < 1e-6)
    assert count(7, 128, "exact") == 19
    c = [count(n, 128, "mg", 3) for n in (7, 15)]
    assert all(20 <= v <= 22 for v in c) and abs(c[0] - c[1]) <= 1, c


def test_s_norm_with_mass_matrix_equals_dense():
    prob = _problem(2, 7, 5)
    M, A = fem.matrices(2, 7)
    S = st.dense_system(M.toarray(), [prob.a[i] * A.toarray() for i in range(prob.N)], [prob.tau] * prob.N)["S"]
    v = np.random.default_rng(6).standard_normal((prob.N, 49))
    assert fem.s_norm(prob, v) == pytest.approx(np.sqrt(v.ravel() @ S @ v.ravel()), rel=1e-11)
