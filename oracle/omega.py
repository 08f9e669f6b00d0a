"""Automatic damping parameter omega of the inexact Uzawa iteration (oracle).

Test infrastructure: only tests, smoke checks and the CPU baseline use this
package.

Theorem 3.1 bounds the contraction of the iteration through rho_A (the
contraction of the approximate solves A~^{-1}, eq. (3.6)) and the extreme
eigenvalues lambda_min, lambda_max of H~^{-1} S; the iteration converges when
omega lambda_max < 2 (1 - rho_A) / (1 + rho_A) (eq. (3.7)).  Theorem 4.1
bounds the eigenvalues by the constant alpha of eq. (2.2), which is too loose
to pick omega from.  This module estimates the three numbers instead:

  * lambda_min, lambda_max of H~^{-1} S~ with
        S~ = K^T A~^{-1} K + K + K^T + A,
    the operator that one Uzawa sweep applies to u when p restarts from zero
    and f = 0 (eq. (3.1)); S~ = S when A~ = A.  Estimated as the extreme Ritz
    values of m steps of conjugate gradients on S~ preconditioned by H~^{-1}
    (the Lanczos tridiagonal matrix built from the CG coefficients).
  * rho_A by power iteration on E = I - A~^{-1} A (ratio of successive
    Euclidean norms).

omega = min( balance * 2 / (lambda_min + lambda_max),  safety * 2 / lambda_max ).
The first term is the damping that balances the two ends of the spectrum for
preconditioned Richardson, the limit of the method as rho_A -> 0 (Remark 3.2);
the second keeps clear of the limit omega < 2 / lambda_max that condition
(3.7) approaches in the same limit.  The sufficient condition (3.7) itself is
reported (omega_theorem) but not imposed: with the rho_A of one V-cycle it
is far tighter than what the iteration needs (on small problems it gives
about half the damping that minimises the spectral radius of the full
iteration matrix, which the balanced value matches within a few percent).

Start vectors come from SplitMix64 (Steele, Lea and Flood, 2014; the mixing
constants of Vigna's reference implementation) evaluated at the global index,
so the GPU library can reproduce them without sharing code.
"""
from __future__ import annotations

import numpy as np

from . import spacetime as st
from .precond import Preconditioners

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(index: np.ndarray, seed: int) -> np.ndarray:
    """SplitMix64 output for state = seed + (index + 1) * golden gamma (mod 2^64)."""
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + (index.astype(np.uint64) + np.uint64(1)) * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def uniform_pm1(shape, seed: int) -> np.ndarray:
    """Values in [-1, 1): 53 high bits of SplitMix64 at the row-major index."""
    n = int(np.prod(shape))
    z = splitmix64(np.arange(n, dtype=np.uint64), seed)
    return ((z >> np.uint64(11)).astype(np.float64) * (2.0 ** -52) - 1.0).reshape(shape)


def apply_S_tilde(prob, pc: Preconditioners, v: np.ndarray) -> np.ndarray:
    Kv = st.apply_K(v)
    return st.apply_KT(pc.Ainv(Kv)) + Kv + st.apply_KT(v) + st.apply_Ablk(prob, v)


def tridiag_from_cg(alphas, betas) -> np.ndarray:
    """Lanczos matrix of m CG steps: T_kk = 1/a_k + b_{k-1}/a_{k-1},
    T_k,k+1 = sqrt(b_k)/a_k."""
    m = len(alphas)
    T = np.zeros((m, m))
    for k in range(m):
        T[k, k] = 1.0 / alphas[k] + (betas[k - 1] / alphas[k - 1] if k > 0 else 0.0)
        if k + 1 < m:
            T[k, k + 1] = T[k + 1, k] = np.sqrt(betas[k]) / alphas[k]
    return T


def lanczos_extremes(prob, pc: Preconditioners, m: int = 12, seed: int = 0x5EED) -> tuple[float, float]:
    shape = (prob.N,) + (prob.n,) * prob.dim
    r = uniform_pm1(shape, seed)
    z = pc.Hinv(r)
    p = z.copy()
    rz = float(np.vdot(r, z))
    alphas, betas = [], []
    for _ in range(m):
        q = apply_S_tilde(prob, pc, p)
        a = rz / float(np.vdot(p, q))
        r = r - a * q
        z = pc.Hinv(r)
        rz_new = float(np.vdot(r, z))
        b = rz_new / rz
        alphas.append(a)
        betas.append(b)
        p = z + b * p
        rz = rz_new
    ev = np.linalg.eigvalsh(tridiag_from_cg(alphas, betas))
    return float(ev[0]), float(ev[-1])


def rho_A(prob, pc: Preconditioners, m: int = 8, seed: int = 0xA5EED) -> float:
    shape = (prob.N,) + (prob.n,) * prob.dim
    e = uniform_pm1(shape, seed)
    e /= np.linalg.norm(e)
    ratio = 0.0
    for _ in range(m):
        e2 = e - pc.Ainv(st.apply_Ablk(prob, e))
        ratio = float(np.linalg.norm(e2))
        if ratio == 0.0:
            return 0.0
        e = e2 / ratio
    return ratio


def auto_omega(prob, spatial: str = "mg", m_lanczos: int = 12, m_power: int = 8, balance: float = 0.95,
               safety: float = 0.9, pc: Preconditioners | None = None) -> dict:
    pc = pc or Preconditioners(prob, spatial=spatial)
    lmin, lmax = lanczos_extremes(prob, pc, m_lanczos)
    rho = rho_A(prob, pc, m_power)
    w = min(balance * 2.0 / (lmin + lmax), safety * 2.0 / lmax)
    w_thm = 2.0 * (1.0 - rho) / ((1.0 + rho) * lmax)
    return dict(omega=w, lmin=lmin, lmax=lmax, rho_A=rho, omega_theorem=w_thm)
