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


def seq_euler_modal(prob, factors=None) -> np.ndarray:
    """Sequential implicit Euler, eq. (2.1), for coefficients that depend on
    time only (every field of ``prob.kfields`` constant in space), by the
    spatial sine transform that diagonalises all A_n at once.

    With kappa(t_n) = sum_r tcoef[r, n-1] kfields[r] and the constant-coefficient
    operator's sine eigenvalues lambda_k = sum_a (4/h^2) sin^2(k_a pi h / 2),
    each mode obeys the scalar recurrence
        uh_n = (uh_{n-1} + tau_n Fh_n) / (1 + tau_n kappa(t_n) lambda_k),
    where hats are DST-I coefficients (scipy.fft.dstn, type 1).  The source is
    ``prob.F`` or, when ``factors`` is given, the separable sum
    F_n = sum_i g_t,i[n-1] (prod_a g_a,i) of ``synth.gaussian_factors`` (whose
    sine transform is the tensor product of the 1-D transforms, so the full
    F is never formed).  Returns u_1..u_N, shape (N,) + (n,)*dim.
    """
    import scipy.fft as sfft

    d, n, N = prob.dim, prob.n, prob.N
    kf = np.asarray(prob.kfields, dtype=np.float64)
    kconst = np.array([kf[r].ravel()[0] for r in range(prob.R)])
    for r in range(prob.R):
        if not np.all(kf[r] == kconst[r]):
            raise ValueError("seq_euler_modal needs coefficient fields constant in space")
    kap = kconst @ prob.tcoef                                   # kappa(t_n), n = 1..N
    axes = tuple(range(-d, 0))
    ks = np.arange(1, n + 1)
    lam1 = 4.0 * (n + 1) ** 2 * np.sin(ks * np.pi / (2 * (n + 1))) ** 2
    lam = lam1
    for _ in range(d - 1):
        lam = np.add.outer(lam1, lam)                           # axes (z, y, x)
    if factors is not None:
        fh = [(gt, [sfft.dst(g, type=1) for g in gx]) for gt, gx in factors]

        def Fhat(m):
            out = np.zeros((n,) * d)
            for gt, gxh in fh:
                term = gxh[0]
                for g in gxh[1:]:
                    term = np.multiply.outer(g, term)           # (x, y, z) factors -> (z, y, x)
                out += gt[m] * term
            return out
    else:
        def Fhat(m):
            return sfft.dstn(prob.F[m], type=1, axes=axes)
    uh = sfft.dstn(np.asarray(prob.u0, dtype=np.float64), type=1, axes=axes)
    out = np.empty((N,) + (n,) * d)
    for m in range(N):
        t = prob.taus[m]
        uh = (uh + t * Fhat(m)) / (1.0 + t * kap[m] * lam)
        out[m] = sfft.idstn(uh, type=1, axes=axes)
    return out
