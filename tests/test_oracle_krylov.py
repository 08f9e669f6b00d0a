"""Pins of the oracle's GMRES acceleration of the inexact Uzawa method
(Section 8.3; the stationary form of eq. (3.1) on the system of eq. (2.7)):
the preconditioner is one Uzawa sweep, the iterates are the least-squares
minimisers over the preconditioned Krylov space, never worse than the Uzawa
iterates, and exact after as many steps as unknowns."""
import numpy as np
import pytest

import synth
from oracle import euler, krylov, uzawa
from oracle import spacetime as st
from oracle.precond import Preconditioners


def small(d, n, N, seed=5, R=2):
    return synth.heat1d_random(n=n, N=N, seed=seed) if d == 1 else synth.small_problem(d, n, N, seed=seed, R=R)


@pytest.mark.parametrize("d,n,N,spatial", [(2, 7, 6, "mg"), (1, 9, 5, "exact")])
def test_stationary_form_reproduces_uzawa(d, n, N, spatial):
    """x_{k+1} = x_k + P^{-1}(g - S x_k) from zero gives the (u_k, p_{k+1}) of
    the Uzawa solver: P^{-1} and g encode eq. (3.1) and eq. (2.7)."""
    prob = small(d, n, N)
    pc = Preconditioners(prob, spatial=spatial)
    xs = krylov.stationary(prob, pc, 0.7, 5)
    for k in (1, 2, 4):
        ref = uzawa.uzawa_fixed(prob, k, omega=0.7, pc=pc)
        scale = np.abs(ref["u"]).max()
        assert np.abs(xs[k][1] - ref["u"]).max() < 1e-12 * scale
        assert np.abs(xs[k + 1][0] - ref["p"]).max() < 1e-12 * np.abs(ref["p"]).max()


def flat(pu):
    return np.concatenate([pu[0].ravel(), pu[1].ravel()])


def test_gmres_iterate_is_least_squares_minimiser():
    """The k-th GMRES iterate minimises ||g - S x|| over the span of
    P^{-1} r_0, P^{-1} (S P^{-1}) r_0, ...: solved here as a dense least-squares
    problem on an orthonormalised basis of those directions."""
    prob = small(2, 3, 4, seed=11)
    pc = Preconditioners(prob, spatial="mg")
    w = 0.6
    g = flat(krylov.saddle_rhs(prob))
    n = g.size // 2
    shape = (prob.N,) + (prob.n,) * prob.dim

    def S(v):
        return flat(krylov.saddle_apply(prob, v[:n].reshape(shape), v[n:].reshape(shape)))

    def Pinv(v):
        return flat(krylov.uzawa_precond(prob, pc, w, v[:n].reshape(shape), v[n:].reshape(shape)))

    for k in (1, 3, 6):
        q = g.copy()
        dirs = []
        for _ in range(k):
            z = Pinv(q)
            dirs.append(z)
            q = S(z)
        Zb, _ = np.linalg.qr(np.array(dirs).T)
        c, *_ = np.linalg.lstsq(np.array([S(z) for z in Zb.T]).T, g, rcond=None)
        x_ls = Zb @ c
        out = krylov.gmres(prob, omega=w, tol=0.0, restart=50, max_iter=k, pc=pc)
        x_gm = np.concatenate([out["p"].ravel(), out["u"].ravel()])
        assert out["iters"] == k
        assert np.abs(x_gm - x_ls).max() < 1e-8 * np.abs(x_ls).max(), k
        assert abs(out["rel"] - np.linalg.norm(g - S(x_ls)) / np.linalg.norm(g)) < 1e-9


@pytest.mark.parametrize("omega", [0.5, 0.8, 1.2])
def test_gmres_never_worse_than_uzawa(omega):
    """Without restarts the k-th GMRES residual is at most the k-th stationary
    (Uzawa) residual, for any omega (also one where Uzawa diverges)."""
    prob = small(2, 7, 8, seed=3)
    pc = Preconditioners(prob, spatial="mg")
    g = flat(krylov.saddle_rhs(prob))
    xs = krylov.stationary(prob, pc, omega, 10)
    out = krylov.gmres(prob, omega=omega, tol=0.0, restart=50, max_iter=10, pc=pc)
    hist = out["history"] * np.linalg.norm(g)
    for k in range(1, 11):
        r_uz = np.linalg.norm(g - flat(krylov.saddle_apply(prob, *xs[k])))
        assert hist[k] <= r_uz * (1 + 1e-10), (k, hist[k], r_uz)
    assert np.all(np.diff(hist) <= 1e-12 * hist[0])      # monotone within a cycle


def test_gmres_estimate_is_true_residual():
    """The Givens estimate equals ||g - S x_k|| of the iterate formed from it."""
    prob = small(2, 7, 8, seed=4)
    pc = Preconditioners(prob, spatial="mg")
    for k in (2, 5, 9):
        out = krylov.gmres(prob, omega=0.8, tol=0.0, restart=50, max_iter=k, pc=pc)
        assert abs(out["history"][-1] - out["rel"]) < 1e-10 * max(out["rel"], 1e-3)


@pytest.mark.parametrize("d,n,N,spatial", [(1, 5, 3, "exact"), (2, 3, 2, "mg")])
def test_gmres_exact_after_dimension_steps(d, n, N, spatial):
    """With a restart length equal to the number of unknowns GMRES ends at the
    solution [-B^{-1} f; B^{-1} f] (the sequential implicit Euler solve)."""
    prob = small(d, n, N, seed=8)
    pc = Preconditioners(prob, spatial=spatial)
    dim = 2 * prob.N * prob.npts
    out = krylov.gmres(prob, omega=0.8, tol=1e-12, restart=dim, max_iter=dim, pc=pc)
    ref = euler.seq_euler(prob)
    assert out["status"] == "converged" and out["iters"] <= dim
    assert np.abs(out["u"] - ref).max() < 1e-9 * np.abs(ref).max()
    assert np.abs(out["p"] + ref).max() < 1e-9 * np.abs(ref).max()


def test_gmres_restarted_reaches_tolerance_with_paper_stop_test():
    """Restarted GMRES stops on ||f - B u|| <= tol ||f|| like the Uzawa solver,
    needs fewer steps than Uzawa iterations, and its residual estimates never
    rise within a cycle."""
    prob = small(2, 15, 16, seed=6)
    pc = Preconditioners(prob, spatial="mg")
    uz = uzawa.uzawa(prob, omega=0.75, tol=1e-8, max_iter=400, pc=pc)
    out = krylov.gmres(prob, omega=0.75, tol=1e-8, restart=5, max_iter=400, pc=pc)
    assert out["status"] == "converged" and out["rel_res"] <= 1e-8
    assert out["iters"] < uz["iters"]
    f = st.rhs(prob)
    assert np.linalg.norm(f - st.apply_B(prob, out["u"])) <= 1e-8 * np.linalg.norm(f)
    h = out["history"]
    for c in range(0, len(h) - 1, 5):                  # cycles of 5 steps
        seg = h[c + 1:c + 6]
        assert np.all(np.diff(seg) <= 1e-12 * h[0])


def test_minres_matches_library_minres():
    """The oracle's preconditioned MINRES (Remark 3.4, P = diag(A~, H~)) gives
    the iterates of scipy's MINRES with the same operator and preconditioner."""
    import scipy.sparse.linalg as spla
    prob = small(2, 3, 4, seed=21)
    pc = Preconditioners(prob, spatial="mg")
    g = flat(krylov.saddle_rhs(prob))
    n = g.size // 2
    shape = (prob.N,) + (prob.n,) * prob.dim
    S = spla.LinearOperator((2 * n, 2 * n), dtype=np.float64,
                            matvec=lambda v: flat(krylov.saddle_apply(prob, v[:n].reshape(shape), v[n:].reshape(shape))))
    M = spla.LinearOperator((2 * n, 2 * n), dtype=np.float64,
                            matvec=lambda v: flat(krylov.block_precond(prob, pc, v[:n].reshape(shape), v[n:].reshape(shape))))
    for k in (1, 4, 9):
        x_lib, _ = spla.minres(S, g, M=M, maxiter=k, rtol=0.0)
        out = krylov.minres(prob, tol=0.0, max_iter=k, pc=pc)
        x = np.concatenate([out["p"].ravel(), out["u"].ravel()])
        assert out["iters"] == k
        assert np.abs(x - x_lib).max() < 1e-10 * np.abs(x_lib).max(), k


def test_minres_needs_no_damping_and_reaches_euler():
    """MINRES has no omega; it reaches the sequential solution on a problem
    where Uzawa with omega = 1.2 diverges, and its residual estimate never
    rises."""
    prob = small(2, 7, 8, seed=3)
    pc = Preconditioners(prob, spatial="mg")
    assert uzawa.uzawa(prob, omega=1.2, tol=1e-10, max_iter=300, pc=pc)["status"] != "converged"
    out = krylov.minres(prob, tol=1e-12, max_iter=600, pc=pc)
    assert out["status"] == "converged"
    ref = euler.seq_euler(prob)
    assert np.abs(out["u"] - ref).max() < 1e-9 * np.abs(ref).max()
    assert np.all(np.diff(out["history"]) <= 1e-12)
