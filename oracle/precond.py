"""The two preconditioners of the inexact Uzawa iteration.

* A-tilde = diag(tau_n A-tilde_n), eq. (3.2): A-tilde^{-1} r acts slab by slab,
  (tau_n A-tilde_n)^{-1} r_n = nu_A V-cycles for the operator tau_n A_n (or an
  exact solve).
* H-tilde = Phi^T Hhat_approx Phi, eq. (4.6), with
  Hhat_approx = (N / 2 tau) diag(H-tilde_k A^{-1} H-tilde_k) and H_k = mu_k M + tau A:
      H-tilde^{-1} r = Phi^{-1} Hhat_approx^{-1} Phi^{-T} r,
      (Hhat_approx^{-1})_k = (2 tau / N) H-tilde_k^{-1} A H-tilde_k^{-1},
  where H-tilde_k^{-1} is nu_H V-cycles for H_k (or an exact solve) and the
  middle A is the exact reference operator A = A(kappa_ref).

Reference pair (tau, A) of eq. (2.2): tau = T/N and kappa_ref = the time mean
of kappa(t_n, .), weighted by the step lengths when they differ (the paper
allows "an average"); A-tilde uses each step's own tau_n.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import dst, fd, mg, spacetime


class Preconditioners:
    def __init__(self, prob, spatial: str = "mg", nu_A: int = 1, nu_H: int = 1, kref_coef=None):
        self.prob = prob
        N, tau = prob.N, prob.tau
        self.N = N
        self.nu_A, self.nu_H = nu_A, nu_H
        self.abar = spacetime.kref_coef(prob) if kref_coef is None else np.asarray(kref_coef, dtype=np.float64)
        self.sigA = np.zeros(N)
        self.cA = (prob.taus[None, :] * prob.tcoef).T.copy()      # (N, R): tau_n A_n
        self.sigH = dst.mu(N)
        self.cH = np.tile(tau * self.abar, (N, 1))               # (N, R)
        self.cmid = np.tile((2.0 / N) * tau * self.abar, (N, 1))  # (2/N) tau A
        self.spatial = spatial
        if spatial == "mg":
            self.hier = mg.Hierarchy(prob.kfields, prob.n, prob.dim)
        elif spatial == "exact":
            Ar = [fd.assemble(prob.kfields[r], prob.n, prob.dim, prob.h) for r in range(prob.R)]
            Id = sp.identity(prob.npts, format="csc")

            def mat(sig, c):
                return (sig * Id + sum(c[r] * Ar[r] for r in range(prob.R))).tocsc()
            self.luA = [spla.splu(mat(self.sigA[i], self.cA[i])) for i in range(N)]
            self.luH = [spla.splu(mat(self.sigH[k], self.cH[k])) for k in range(N)]
        else:
            raise ValueError(spatial)

    # -- spatial pieces -----------------------------------------------------
    def _solve(self, which, b, nu):
        if self.spatial == "mg":
            sig, c = (self.sigA, self.cA) if which == "A" else (self.sigH, self.cH)
            return self.hier.vcycles(sig, c, b, nu)
        lus = self.luA if which == "A" else self.luH
        shape = b.shape[1:]
        return np.stack([lus[i].solve(b[i].ravel()).reshape(shape) for i in range(b.shape[0])])

    def mid(self, x):
        """(2/N) tau A_ref x, slab by slab."""
        out = np.zeros_like(x)
        for r in range(self.prob.R):
            out += self.cmid[0, r] * fd.apply(self.prob.kfields[r], x, self.prob.h, self.prob.dim)
        return out

    # -- the two preconditioners ---------------------------------------------
    def Ainv(self, r):
        """A-tilde^{-1} r."""
        return self._solve("A", r, self.nu_A)

    def Hhat_inv(self, rhat):
        """Hhat_approx^{-1} in the transformed basis, block k = (2tau/N) H~_k^{-1} A H~_k^{-1}."""
        x = self._solve("H", rhat, self.nu_H)
        return self._solve("H", self.mid(x), self.nu_H)

    def Hinv(self, r):
        """H-tilde^{-1} r = Phi^{-1} Hhat_approx^{-1} Phi^{-T} r."""
        return dst.inverse(self.Hhat_inv(dst.inverse_transpose(r)))
