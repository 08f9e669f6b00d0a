"""Spectral quantities of the method.

* Eigenvalues of H^{-1} S (Theorem 4.1; Section 8.1, Table 1) for constant
  coefficients, uniform steps and alpha = 1.  When A_n = A for all n, M and A
  are diagonalised together by their generalized eigenvectors
  (A v_j = lambda_j M v_j, v_j^T M v_j = 1), and both S (eq. (2.5)) and
  H (eq. (4.4)) split into independent N x N blocks, one per spatial mode j,
  with z = tau lambda_j:

      S_j = K^T K / z + K + K^T + z I,
      H_j = Phi^T diag_k( (N/2) (mu_k + z)^2 / z ) Phi,

  (M -> 1, A -> lambda_j, M A^{-1} M -> 1/lambda_j).  eig(H^{-1}S) is the union
  of eig(H_j^{-1} S_j).
* The convergence factor rho_U of Theorem 3.1, eq. (3.5).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from . import dst
from .spacetime import Kmat


def mode_blocks(N: int, z: float):
    K = Kmat(N)
    S = K.T @ K / z + K + K.T + z * np.eye(N)
    Phi = dst.phi_matrix(N)
    mu = dst.mu(N)
    H = Phi.T @ np.diag((N / 2.0) * (mu + z) ** 2 / z) @ Phi
    return S, H


def extreme_eigs_per_mode(N: int, lambdas, tau: float):
    lo, hi = np.inf, -np.inf
    for lam in lambdas:
        S, H = mode_blocks(N, tau * lam)
        ev = sla.eigh(S, H, eigvals_only=True)
        lo = min(lo, ev[0])
        hi = max(hi, ev[-1])
    return lo, hi


def rho_uzawa(rho_A: float, omega: float, lmin: float, lmax: float) -> float:
    """rho_U = max(sigma_-, sigma_+) of eq. (3.5)."""
    a = (1 - rho_A) * (1 - omega * lmin)
    sm = 0.5 * (a + np.sqrt(4 * rho_A + a * a))
    b = (1 + rho_A) * (1 + omega * lmax) - 2
    sp_ = 0.5 * (b + np.sqrt(4 * rho_A + b * b))
    return max(sm, sp_)
