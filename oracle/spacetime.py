"""Time-global operators of Section 2 (eqs. (2.3)-(2.7)) and the ideal Schur
preconditioner H of eq. (4.4).

Matrix-free versions act on FD problems (M = I) with vectors shaped
(N,) + spatial; dense versions assemble the matrices for tiny sizes with a
general SPD mass matrix M.

    K = (lower bidiagonal: 1 on the diagonal, -1 below) (x) M          eq. (2.4)
    A = diag(tau_n A_n),  B = K + A                                     eq. (2.3)
    f = [tau_1 f_1 + M u_I, tau_2 f_2, ..., tau_N f_N]
    P = A^{-1} K + I,  S = P^T B = K^T A^{-1} K + K + K^T + A           eq. (2.5)
    saddle = [[A, -K], [-K^T, -(K + K^T + A)]],  rhs [-f; -f]           eq. (2.7)
    H = Phi^T Hhat Phi,  Hhat = (N / 2 tau) diag(H_k A^{-1} H_k),
    H_k = mu_k M + tau A                                                eq. (4.4)-(4.5)
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from . import dst, fd


# ---------------------------------------------------------------------------
# matrix-free, FD problems (M = I)
# ---------------------------------------------------------------------------

def _bcast(v, x):
    return v.reshape((-1,) + (1,) * (x.ndim - 1))


def apply_K(x: np.ndarray) -> np.ndarray:
    y = x.copy()
    y[1:] -= x[:-1]
    return y


def apply_KT(x: np.ndarray) -> np.ndarray:
    y = x.copy()
    y[:-1] -= x[1:]
    return y


def apply_Ablk(prob, x: np.ndarray) -> np.ndarray:
    """(A x)_n = tau_n A(kappa(t_n)) x_n, using linearity of A in kappa."""
    out = np.zeros_like(x)
    for r in range(prob.R):
        out += _bcast(prob.taus * prob.tcoef[r], x) * fd.apply(prob.kfields[r], x, prob.h, prob.dim)
    return out


def rhs(prob) -> np.ndarray:
    f = _bcast(prob.taus, prob.F) * prob.F.astype(np.float64)
    f[0] += prob.u0
    return f


def apply_B(prob, x):
    return apply_K(x) + apply_Ablk(prob, x)


def s_norm(prob, v: np.ndarray) -> float:
    """||v||_S by the identity of Theorem 6.2 (eqs. (6.11)-(6.14)) with M = I:
    v^T S v = sum_n [ (1/tau_n)|dv_n|^2_{A_n^{-1}} + tau_n |v_n|^2_{A_n} + |dv_n|^2 ] + |v_N|^2,
    dv_n = v_n - v_{n-1}, v_0 = 0; A_n^{-1} by a sparse LU per distinct step operator."""
    import scipy.sparse.linalg as spla
    Ar = [fd.assemble(prob.kfields[r], prob.n, prob.dim, prob.h) for r in range(prob.R)]
    lus = {}
    total = 0.0
    prev = np.zeros(prob.npts)
    for i in range(prob.N):
        key = tuple(prob.tcoef[:, i])
        An = sum(prob.tcoef[r, i] * Ar[r] for r in range(prob.R)).tocsc()
        if key not in lus:
            lus[key] = spla.splu(An)
        vi = v[i].ravel()
        dv = vi - prev
        t = prob.taus[i]
        total += dv @ lus[key].solve(dv) / t + t * (vi @ (An @ vi)) + dv @ dv
        prev = vi
    total += prev @ prev
    return float(np.sqrt(total))


def apply_saddle(prob, p, u):
    """saddle [p; u] = [A p - K u;  -K^T p - (K + K^T + A) u]."""
    Ap = apply_Ablk(prob, p)
    Au = apply_Ablk(prob, u)
    top = Ap - apply_K(u)
    bot = -apply_KT(p) - (apply_K(u) + apply_KT(u) + Au)
    return top, bot


def kref_coef(prob) -> np.ndarray:
    """Coefficients of the reference operator A = A(kappa_ref) used in H_k:
    kappa_ref = time mean of kappa(t_n, .), i.e. abar_r = mean_n tcoef[r, n];
    with non-uniform steps the step-weighted mean sum_n tau_n tcoef[r, n] / T
    (the reference tau is T/N, so tau A_ref = sum_n tau_n A_n / N)."""
    if prob.steps is None:
        return prob.tcoef.mean(axis=1)
    return (prob.tcoef * prob.taus[None, :]).sum(axis=1) / prob.taus.sum()


# ---------------------------------------------------------------------------
# dense assembly, general M (tiny sizes)
# ---------------------------------------------------------------------------

def Kmat(N: int) -> np.ndarray:
    return np.eye(N) - np.eye(N, k=-1)


def dense_system(M: np.ndarray, A_list, taus):
    """Assemble K, A, B, P, S and the saddle-point matrix from M, [A_n], [tau_n]."""
    N = len(A_list)
    m = M.shape[0]
    Kb = np.kron(Kmat(N), M)
    Ab = sla.block_diag(*[taus[i] * A_list[i] for i in range(N)])
    B = Kb + Ab
    P = np.linalg.solve(Ab, Kb) + np.eye(N * m)
    S = P.T @ B
    sad = np.block([[Ab, -Kb], [-Kb.T, -(Kb + Kb.T + Ab)]])
    return dict(K=Kb, A=Ab, B=B, P=P, S=S, saddle=sad)


def dense_rhs(M, taus, fs, uI):
    f = np.concatenate([taus[i] * np.asarray(fs[i]) for i in range(len(taus))])
    m = M.shape[0]
    f[:m] += M @ uI
    return f


def dense_H(M: np.ndarray, Aref: np.ndarray, tau: float, N: int, Hk_list=None):
    """H = Phi^T Hhat Phi with Hhat = (N/2tau) diag(Ht_k A^{-1} Ht_k).

    ``Hk_list`` replaces H_k = mu_k M + tau A by given SPD approximations
    (eq. (4.6)); default is the exact H_k."""
    m = M.shape[0]
    mu = dst.mu(N)
    Ainv = np.linalg.inv(Aref)
    blocks = []
    for k in range(N):
        Hk = mu[k] * M + tau * Aref if Hk_list is None else Hk_list[k]
        blocks.append((N / (2 * tau)) * Hk @ Ainv @ Hk)
    Hhat = sla.block_diag(*blocks)
    Phi = np.kron(dst.phi_matrix(N), np.eye(m))
    return Phi.T @ Hhat @ Phi


def fd_dense_pieces(prob):
    """M = I and the dense A_n of an FD problem (tiny sizes only)."""
    m = prob.npts
    A_list = []
    for i in range(prob.N):
        kap = fd.kappa_at(prob.kfields, prob.tcoef[:, i])
        A_list.append(fd.assemble(kap, prob.n, prob.dim, prob.h).toarray())
    Aref = fd.assemble(fd.kappa_at(prob.kfields, kref_coef(prob)), prob.n, prob.dim, prob.h).toarray()
    return np.eye(m), A_list, list(prob.taus), Aref
