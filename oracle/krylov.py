"""GMRES acceleration of the inexact Uzawa method (oracle).

Test infrastructure: only tests, smoke checks and the CPU baseline use this
package.

The large-scale experiments of Section 8.3 accelerate the inexact Uzawa
method with GMRES and give no further detail.  The reading taken here:

* The iteration (3.1) is the stationary method x_{k+1} = x_k + P^{-1}(g - S x_k)
  for the saddle system S x = g of eq. (2.7), x = [p; u], S = saddle matrix,
  g = [-f; -f].  One Uzawa sweep from a zero start applied to a residual
  r = [r_1; r_2] gives
      P^{-1} r = [ d ; -omega H~^{-1} (r_2 + K^T d) ],   d = A~^{-1} r_1,
  because the u-update of (3.1) sees the p just updated (a block
  lower-triangular splitting).
* GMRES(m) (Saad and Schultz) with P^{-1} as right preconditioner, in the
  flexible form (the preconditioned directions z_j = P^{-1} v_j are kept, so
  x = x_0 + Z y needs no further preconditioner application and a float32
  preconditioner stays consistent).  Each cycle minimises ||g - S x||_2 over
  x_0 + span{z_0, ..., z_{k-1}}; without restarts that is the affine space in
  which the k-th stationary iterate lies, so the GMRES residual never exceeds
  the Uzawa residual of the same step count.
* Arnoldi with modified Gram-Schmidt, Givens rotations for the small least
  squares problem (the textbook algorithm); restart after m steps.
* Stopping: the same test as the Uzawa solver, ||f - B u||_2 <= tol ||f||_2.
  It is evaluated (on the candidate x_0 + Z y) only after steps whose
  least-squares estimate of ||g - S x||_2 is <= tol ||g||_2, and at every
  restart; a failed check lets the cycle go on.  At most max_iter Arnoldi
  steps in total.

MINRES (Remark 3.4) is the alternative the paper names: the saddle matrix is
symmetric, and with the symmetric positive definite block-diagonal
preconditioner P = diag(A~, H~) (P^{-1} = diag(A~^{-1}, H~^{-1})) no damping
parameter is needed.  ``minres`` below is the preconditioned MINRES of Paige and
Saunders (1975): a Lanczos process on P^{-1} S in the P inner product, the
tridiagonal least-squares problem solved by Givens rotations, three-term
updates of the iterate.  Its residual estimate is ||g - S x||_{P^{-1}}; the stop
test is again ||f - B u|| <= tol ||f||, checked once that estimate is <= tol times
its initial value and then every ``check_every`` steps.
"""
from __future__ import annotations

import numpy as np

from . import spacetime as st
from .precond import Preconditioners


def saddle_rhs(prob):
    f = st.rhs(prob)
    return -f, -f.copy()


def saddle_apply(prob, p, u):
    return st.apply_saddle(prob, p, u)


def uzawa_precond(prob, pc: Preconditioners, omega: float, r1, r2):
    """One sweep of eq. (3.1) from x = 0 on residual [r1; r2]."""
    d = pc.Ainv(r1)
    du = -omega * pc.Hinv(r2 + st.apply_KT(d))
    return d, du


def stationary(prob, pc: Preconditioners, omega: float, steps: int, x0=None):
    """x_{k+1} = x_k + P^{-1}(g - S x_k), k < steps: the list [x_0, ..., x_steps]."""
    g1, g2 = saddle_rhs(prob)
    p = np.zeros_like(g1) if x0 is None else x0[0].copy()
    u = np.zeros_like(g1) if x0 is None else x0[1].copy()
    out = [(p.copy(), u.copy())]
    for _ in range(steps):
        s1, s2 = saddle_apply(prob, p, u)
        dp, du = uzawa_precond(prob, pc, omega, g1 - s1, g2 - s2)
        p, u = p + dp, u + du
        out.append((p.copy(), u.copy()))
    return out


def solve_upper(H, s, k):
    """y with H[:k, :k] y = s[:k], H upper triangular (back substitution)."""
    y = np.zeros(k)
    for i in range(k - 1, -1, -1):
        y[i] = (s[i] - np.dot(H[i, i + 1:k], y[i + 1:k])) / H[i, i]
    return y


def gmres(prob, omega: float = 0.8, tol: float = 1e-8, restart: int = 20, max_iter: int = 200,
          spatial: str = "mg", pc: Preconditioners | None = None, p_init=None, u_init=None):
    """Flexible GMRES(restart) on the saddle system, right-preconditioned by one
    Uzawa sweep.  Returns u, p, iters (Arnoldi steps), the residual estimate
    history (relative to ||g||, one entry per step, the initial one first),
    the number of stop checks, the true relative residual ||g - S x|| / ||g||
    at return and ||f - B u|| / ||f||."""
    pc = pc or Preconditioners(prob, spatial=spatial)
    g1, g2 = saddle_rhs(prob)
    shape = g1.shape
    n = g1.size
    gnorm = np.sqrt(np.vdot(g1, g1) + np.vdot(g2, g2))
    x = np.zeros(2 * n)
    if p_init is not None:
        x[:n] = np.asarray(p_init, dtype=np.float64).ravel()
    if u_init is not None:
        x[n:] = np.asarray(u_init, dtype=np.float64).ravel()
    g = np.concatenate([g1.ravel(), g2.ravel()])
    f = st.rhs(prob)
    fnorm = np.linalg.norm(f)
    checks = 0

    def stop_ok(xc):
        nonlocal checks
        checks += 1
        return np.linalg.norm(f - st.apply_B(prob, xc[n:].reshape(shape))) <= tol * fnorm

    def S(v):
        a, b = saddle_apply(prob, v[:n].reshape(shape), v[n:].reshape(shape))
        return np.concatenate([a.ravel(), b.ravel()])

    def Pinv(v):
        a, b = uzawa_precond(prob, pc, omega, v[:n].reshape(shape), v[n:].reshape(shape))
        return np.concatenate([a.ravel(), b.ravel()])

    hist = []
    iters = 0
    status = "maxiter"
    while True:
        r = g - S(x)
        beta = np.linalg.norm(r)
        if not hist:
            hist.append(beta / gnorm)
        if stop_ok(x):
            status = "converged"
            break
        if iters >= max_iter:
            break
        m = min(restart, max_iter - iters)
        V = np.zeros((m + 1, 2 * n))
        Z = np.zeros((m, 2 * n))
        H = np.zeros((m + 1, m))
        cs, sn = np.zeros(m), np.zeros(m)
        s = np.zeros(m + 1)
        s[0] = beta
        V[0] = r / beta
        k = 0
        for j in range(m):
            Z[j] = Pinv(V[j])
            w = S(Z[j])
            for i in range(j + 1):            # modified Gram-Schmidt
                H[i, j] = np.vdot(V[i], w)
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] > 0:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):                # earlier rotations on the new column
                a, b = H[i, j], H[i + 1, j]
                H[i, j] = cs[i] * a + sn[i] * b
                H[i + 1, j] = -sn[i] * a + cs[i] * b
            den = np.hypot(H[j, j], H[j + 1, j])
            if den == 0.0:                    # singular least-squares problem: stop the cycle
                break
            cs[j], sn[j] = H[j, j] / den, H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            s[j + 1] = -sn[j] * s[j]
            s[j] = cs[j] * s[j]
            k = j + 1
            iters += 1
            hist.append(abs(s[j + 1]) / gnorm)
            if abs(s[j + 1]) <= tol * gnorm and stop_ok(x + Z[:k].T @ solve_upper(H, s, k)):
                break
        x = x + Z[:k].T @ solve_upper(H, s, k)
        if k == 0:
            status = "breakdown"
            break
    p = x[:n].reshape(shape)
    u = x[n:].reshape(shape)
    true_rel = float(np.linalg.norm(g - S(x)) / gnorm)
    rel_b = float(np.linalg.norm(f - st.apply_B(prob, u)) / np.linalg.norm(f))
    return dict(u=u, p=p, iters=iters, history=np.array(hist), checks=checks, rel=true_rel, rel_res=rel_b,
                status=status)


def block_precond(prob, pc: Preconditioners, r1, r2):
    """P^{-1} r = [A~^{-1} r_1; H~^{-1} r_2] (Remark 3.4)."""
    return pc.Ainv(r1), pc.Hinv(r2)


def minres(prob, tol: float = 1e-8, max_iter: int = 500, spatial: str = "mg", pc: Preconditioners | None = None,
           p_init=None, u_init=None, check_every: int = 8):
    """Preconditioned MINRES on the saddle system with P^{-1} = diag(A~^{-1}, H~^{-1}).

    The recurrence is the Paige-Saunders algorithm (SIAM J. Numer. Anal. 12, 1975)
    in the form and variable names of scipy's reference implementation
    (scipy/sparse/linalg/_isolve/minres.py: oldb, dbar, epsln, phibar, ...),
    with the same update order; the pin that does not rest on that code is
    convergence to the sequential Euler solution without damping.
    Returns u, p, iters, the history of the residual estimate ||g - S x||_{P^{-1}}
    relative to its initial value (initial entry first), ||f - B u|| / ||f||."""
    pc = pc or Preconditioners(prob, spatial=spatial)
    g1, g2 = saddle_rhs(prob)
    shape = g1.shape
    n = g1.size
    g = np.concatenate([g1.ravel(), g2.ravel()])
    f = st.rhs(prob)
    fnorm = np.linalg.norm(f)
    x = np.zeros(2 * n)
    if p_init is not None:
        x[:n] = np.asarray(p_init, dtype=np.float64).ravel()
    if u_init is not None:
        x[n:] = np.asarray(u_init, dtype=np.float64).ravel()

    def S(v):
        a, b = saddle_apply(prob, v[:n].reshape(shape), v[n:].reshape(shape))
        return np.concatenate([a.ravel(), b.ravel()])

    def Pinv(v):
        a, b = block_precond(prob, pc, v[:n].reshape(shape), v[n:].reshape(shape))
        return np.concatenate([a.ravel(), b.ravel()])

    def stop_ok(xc):
        return np.linalg.norm(f - st.apply_B(prob, xc[n:].reshape(shape))) <= tol * fnorm

    r1 = g - S(x)
    y = Pinv(r1)
    beta1 = float(np.sqrt(np.dot(r1, y)))
    hist = [1.0]
    status = "maxiter"
    iters = 0
    if stop_ok(x):
        status = "converged"
    elif beta1 > 0:
        oldb, beta, dbar, epsln, phibar = 0.0, beta1, 0.0, 0.0, beta1
        cs, sn = -1.0, 0.0
        w = np.zeros(2 * n)
        w2 = np.zeros(2 * n)
        r2 = r1.copy()
        checking = False
        while iters < max_iter:
            v = y / beta                      # Lanczos vector (P^{-1} space)
            y = S(v)
            if iters > 0:
                y = y - (beta / oldb) * r1
            alfa = float(np.dot(v, y))
            y = y - (alfa / beta) * r2
            r1, r2 = r2, y
            y = Pinv(r2)
            oldb, beta = beta, float(np.sqrt(max(np.dot(r2, y), 0.0)))
            # apply the previous rotation, then the new one annihilating beta
            oldeps = epsln
            delta = cs * dbar + sn * alfa
            gbar = sn * dbar - cs * alfa
            epsln = sn * beta
            dbar = -cs * beta
            gamma = max(float(np.hypot(gbar, beta)), 1e-300)
            cs, sn = gbar / gamma, beta / gamma
            phi = cs * phibar
            phibar = sn * phibar
            w1, w2 = w2, w
            w = (v - oldeps * w1 - delta * w2) / gamma
            x = x + phi * w
            iters += 1
            hist.append(abs(phibar) / beta1)
            if abs(phibar) <= tol * beta1:
                checking = True
            if (checking and (iters % check_every == 0 or abs(phibar) <= tol * beta1)) and stop_ok(x):
                status = "converged"
                break
            if beta == 0.0:
                status = "converged" if stop_ok(x) else "breakdown"
                break
    u = x[n:].reshape(shape)
    p = x[:n].reshape(shape)
    rel_b = float(np.linalg.norm(f - st.apply_B(prob, u)) / fnorm)
    return dict(u=u, p=p, iters=iters, history=np.array(hist), rel_res=rel_b, status=status)
