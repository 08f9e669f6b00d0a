"""Sequential implicit Euler, eq. (2.1) of Section 2: for n = 1..N solve

    M (u_n - u_{n-1}) + tau_n A_n u_n = tau_n f_n,   u_0 = u_I,

with M = I (finite differences) and A_n = A(kappa(t_n, .)).  This is the
result the space-time method reaches exactly: the second block of the
saddle-point solution equals B^{-1} f (Section 2.1).

Spatial solves: sparse LU (scipy) by default; for large 3-D grids a CG
iteration preconditioned by the oracle's own V-cycle, run to a relative
residual of ``rtol``.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import fd


def step_matrices(prob):
    """Sparse A(kappa_r) for every separable coefficient term r."""
    return [fd.assemble(prob.kfields[r], prob.n, prob.dim, prob.h) for r in range(prob.R)]


def seq_euler(prob, nsteps: int | None = None, method: str = "lu", rtol: float = 1e-14,
              u_start=None, n_start: int = 1) -> np.ndarray:
    """Return u_1..u_nsteps (array (nsteps,) + spatial shape).

    ``u_start``/``n_start`` resume from a given u_{n_start-1} (default u_0 = u0).
    """
    N = prob.N if nsteps is None else nsteps
    shape = (prob.n,) * prob.dim
    Ar = step_matrices(prob)
    Id = sp.identity(prob.npts, format="csr")
    u = (prob.u0 if u_start is None else u_start).ravel().astype(np.float64)
    out = np.empty((N - n_start + 1,) + shape)
    for m in range(n_start, N + 1):
        tau = prob.taus[m - 1]
        An = sum(prob.tcoef[r, m - 1] * Ar[r] for r in range(prob.R))
        L = (Id + tau * An).tocsc()
        rhs = u + tau * prob.F[m - 1].ravel()
        if method == "lu":
            u = spla.spsolve(L, rhs)
        elif method == "cg":
            u = _pcg_mg(prob, m, L, rhs, u, rtol)
        else:
            raise ValueError(method)
        out[m - n_start] = u.reshape(shape)
    return out


def _pcg_mg(prob, m, L, rhs, x0, rtol):
    """CG on (I + tau A_m) x = rhs preconditioned by one V-cycle of the same operator."""
    from . import mg
    hier = mg.Hierarchy(prob.kfields, prob.n, prob.dim)
    c = (prob.taus[m - 1] * prob.tcoef[:, m - 1])[None, :]
    sigma = np.array([1.0])
    shape = (1,) + (prob.n,) * prob.dim

    def M(v):
        return hier.vcycle(sigma, c, v.reshape(shape)).ravel()

    x = x0.copy()
    r = rhs - L @ x
    z = M(r)
    pdir = z.copy()
    rz = r @ z
    nb = np.linalg.norm(rhs)
    for _ in range(1000):
        if np.linalg.norm(r) <= rtol * nb:
            break
        Ap = L @ pdir
        alpha = rz / (pdir @ Ap)
        x += alpha * pdir
        r -= alpha * Ap
        z = M(r)
        rz_new = r @ z
        pdir = z + (rz_new / rz) * pdir
        rz = rz_new
    return x
