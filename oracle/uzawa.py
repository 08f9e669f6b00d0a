"""The inexact Uzawa iteration of Section 3, eq. (3.1):

    p_{j+1} = p_j + A~^{-1} (K u_j - A p_j - f)
    u_{j+1} = u_j + omega H~^{-1} (f - K^T p_{j+1} - (K + K^T + A) u_j)

Stopping rule (the paper states "residual tolerance" without a norm): stop at
the first j with ||f - B u_j||_2 <= tol ||f||_2 (for f = 0, whose solution is
zero, the absolute ||B u_j||_2 <= tol).  The test is evaluated in
iteration j after the p-update (the same place the GPU library evaluates it),
so on return u = u_j and p = p_{j+1}; ``iters`` = j.  Initial guess
u_0 = p_0 = 0 unless given.
"""
from __future__ import annotations

import numpy as np

from . import spacetime as st
from .precond import Preconditioners


def uzawa(prob, omega: float = 0.8, tol: float = 1e-8, max_iter: int = 200,
          spatial: str = "mg", nu_A: int = 1, nu_H: int = 1, u_init=None, p_init=None,
          pc: Preconditioners | None = None, callback=None):
    pc = pc or Preconditioners(prob, spatial=spatial, nu_A=nu_A, nu_H=nu_H)
    f = st.rhs(prob)
    shape = f.shape
    u = np.zeros(shape) if u_init is None else np.array(u_init, dtype=np.float64).reshape(shape)
    p = np.zeros(shape) if p_init is None else np.array(p_init, dtype=np.float64).reshape(shape)
    fnorm = np.linalg.norm(f)
    den = fnorm if fnorm > 0 else 1.0        # f = 0: absolute residual
    hist = []
    status = "maxiter"
    j = 0
    while True:
        Au = st.apply_Ablk(prob, u)
        Ku = st.apply_K(u)
        rp = Ku - st.apply_Ablk(prob, p) - f
        p = p + pc.Ainv(rp)
        e = f - Ku - Au                      # f - B u_j
        res = np.linalg.norm(e)
        hist.append(res / den)
        if callback is not None:
            callback(j, u, p, res / den)
        if not np.isfinite(res):
            status = "diverged"
            break
        if res <= tol * den:
            status = "converged"
            break
        if j >= max_iter:
            break
        ru = f - st.apply_KT(p) - (Ku + st.apply_KT(u) + Au)
        u = u + omega * pc.Hinv(ru)
        j += 1
    return dict(u=u, p=p, iters=j, history=np.array(hist), status=status, fnorm=fnorm)


def uzawa_fixed(prob, iters: int, omega: float = 0.8, **kw):
    """Exactly ``iters`` updates of u (no stopping test): returns (u_iters, p_{iters+1}).

    Used for iterate-by-iterate parity."""
    return uzawa(prob, omega=omega, tol=0.0, max_iter=iters, **kw)
