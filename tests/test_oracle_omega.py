"""Pins of the oracle's automatic damping parameter (Theorem 3.1, eq. (3.7);
Theorem 4.1): the counter-based start vectors, the Lanczos extreme
eigenvalues, the power estimate of rho_A, and the damping it picks."""
import numpy as np
import pytest

import synth
from oracle import omega as om
from oracle import spacetime as st
from oracle import uzawa
from oracle.precond import Preconditioners


def test_splitmix64_reference_outputs():
    # first five outputs of the SplitMix64 reference generator seeded with 1234567
    got = om.splitmix64(np.arange(5, dtype=np.uint64), 1234567)
    want = [6457827717110365317, 3203168211198807973, 9817491932198370423, 4593380528125082431,
            16408922859458223821]
    assert [int(v) for v in got] == want


def test_uniform_pm1_range_and_moments():
    v = om.uniform_pm1((4, 1000), 7)
    assert v.min() >= -1.0 and v.max() < 1.0
    assert abs(v.mean()) < 0.03 and abs(v.var() - 1.0 / 3.0) < 0.02


def dense_columns(fn, shape):
    n = int(np.prod(shape))
    cols = []
    for i in range(n):
        e = np.zeros(n)
        e[i] = 1.0
        cols.append(fn(e.reshape(shape)).ravel())
    return np.array(cols).T


@pytest.mark.parametrize("spatial,d,n,N", [("mg", 2, 3, 2), ("exact", 1, 5, 3)])
def test_lanczos_exact_with_full_krylov_space(spatial, d, n, N):
    """With as many CG steps as unknowns the Ritz values are the eigenvalues:
    the extremes equal those of the densely assembled H~^{-1} S~."""
    prob = synth.heat1d_random(n=n, N=N, seed=9) if d == 1 else synth.small_problem(d, n, N, seed=9, R=2)
    pc = Preconditioners(prob, spatial=spatial)
    shape = (N,) + (n,) * d
    M = dense_columns(lambda v: pc.Hinv(om.apply_S_tilde(prob, pc, v)), shape)
    ev = np.sort(np.linalg.eigvals(M).real)
    lmin, lmax = om.lanczos_extremes(prob, pc, m=int(np.prod(shape)))
    assert abs(lmin - ev[0]) < 1e-8 * ev[-1] and abs(lmax - ev[-1]) < 1e-8 * ev[-1]
    # S~ is symmetric positive definite (a pin of its assembly, eq. (2.7))
    S = dense_columns(lambda v: om.apply_S_tilde(prob, pc, v), shape)
    assert np.allclose(S, S.T, atol=1e-12 * np.abs(S).max())
    assert np.linalg.eigvalsh(0.5 * (S + S.T)).min() > 0


def test_S_tilde_is_schur_complement_with_exact_solves():
    """With exact spatial solves S~ equals S = K^T A^{-1} K + K + K^T + A, the
    (negated) Schur complement of the saddle matrix of eq. (2.7)."""
    prob = synth.heat1d_random(n=4, N=3, seed=2)
    pc = Preconditioners(prob, spatial="exact")
    shape = (3, 4)
    S = dense_columns(lambda v: om.apply_S_tilde(prob, pc, v), shape)
    Sad = dense_columns(lambda x: np.concatenate([t.ravel() for t in st.apply_saddle(prob, x[:3], x[3:])]),
                        (6, 4))
    n = 12
    A11, A12, A21, A22 = Sad[:n, :n], Sad[:n, n:], Sad[n:, :n], Sad[n:, n:]
    schur = A22 - A21 @ np.linalg.solve(A11, A12)
    assert np.allclose(-schur, S, atol=1e-10 * np.abs(S).max())


def test_rho_A_power_iteration():
    prob = synth.small_problem(2, 7, 3, seed=4, R=2)
    pc = Preconditioners(prob, spatial="mg")
    shape = (3, 7, 7)
    E = dense_columns(lambda v: v - pc.Ainv(st.apply_Ablk(prob, v)), shape)
    rho = max(abs(np.linalg.eigvals(E)))
    # the leading eigenvalues of E lie close together, so the estimate rises
    # slowly towards the spectral radius from below
    ests = [om.rho_A(prob, pc, m=m) for m in (8, 80, 400)]
    assert ests[0] < ests[1] < ests[2] <= rho * (1 + 1e-12)
    assert abs(ests[2] - rho) < 2e-3 * rho and abs(ests[0] - rho) < 0.1 * rho
    # exact spatial solves: A~ = A, so E = 0
    p1 = synth.heat1d_random(n=15, N=8, seed=3)
    assert om.rho_A(p1, Preconditioners(p1, spatial="exact"), m=3) < 1e-12


def test_auto_omega_near_optimal_damping():
    """The chosen damping is within 10% of the damping that minimises the
    spectral radius of the full iteration matrix (eq. (3.1), f = 0), and the
    iteration converges with it."""
    prob = synth.small_problem(2, 3, 4, seed=3, R=1)
    pc = Preconditioners(prob, spatial="mg")

    def step(p, u, w):
        p2 = p + pc.Ainv(st.apply_K(u) - st.apply_Ablk(prob, p))
        u2 = u + w * pc.Hinv(-st.apply_KT(p2) - (st.apply_K(u) + st.apply_KT(u) + st.apply_Ablk(prob, u)))
        return p2, u2

    def radius(w):
        G = dense_columns(lambda x: np.concatenate([t.ravel() for t in step(x[:4], x[4:], w)]), (8, 3, 3))
        return max(abs(np.linalg.eigvals(G)))

    ws = np.linspace(0.3, 1.2, 37)
    rad = np.array([radius(w) for w in ws])
    w_best = ws[rad.argmin()]
    r = om.auto_omega(prob, pc=pc)
    assert abs(r["omega"] - w_best) < 0.1 * w_best, (r, w_best)
    assert radius(r["omega"]) < 1.0
    assert r["omega"] < 2.0 / r["lmax"]
    out = uzawa.uzawa(prob, omega=r["omega"], tol=1e-10, max_iter=500, pc=pc)
    assert out["status"] == "converged"
