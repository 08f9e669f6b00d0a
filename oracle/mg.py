"""Geometric multigrid V-cycle used for the spatial preconditioners
A-tilde_n^{-1} (eq. (3.2)) and H-tilde_k^{-1} (eq. (4.6)).

The paper (Section 8.2) uses "one or two MG V-cycles with Jacobi smoothers"
without further detail; the cycle below is this project's reading, shared as a
specification by the oracle and the GPU library:

* vertex-centred grids with n = 2^L - 1 interior nodes per axis; level l+1 has
  (n_l - 1)/2 nodes per axis; the coarsest level has a single node and is
  solved exactly;
* rediscretised operators: on every level L_s = sigma_s I + sum_r c_{s,r} A(kappa_{r,l}),
  the nodal fields restricted per axis by (1/4, 1/2, 1/4) at interior coarse
  nodes and by injection at the two boundary nodes;
* damped Jacobi with weight 2/3, 4/5, 6/7 in 1, 2, 3 dimensions: one sweep
  before (from the zero guess) and one after the coarse correction;
* full-weighting restriction (tensor product of (1/4, 1/2, 1/4)) and
  multilinear prolongation (2^d times its transpose).

For a right-hand side b the cycle returns
    x1 = W b,  x2 = x1 + P V_{l+1}(R (b - L x1)),  x = x2 + W (b - L x2),
with W = omega_J D^{-1}.  Everything is vectorised over a leading slab axis
(one operator (sigma_s, c_s) per slab).
"""
from __future__ import annotations

import numpy as np

from . import fd

JACOBI_WEIGHT = {1: 2.0 / 3.0, 2: 4.0 / 5.0, 3: 6.0 / 7.0}


def kappa_restriction_1d(n: int) -> np.ndarray:
    """(n_c+2) x (n+2) nodal restriction of a coefficient field along one axis."""
    nc = (n - 1) // 2
    Rm = np.zeros((nc + 2, n + 2))
    Rm[0, 0] = 1.0
    Rm[nc + 1, n + 1] = 1.0
    for I in range(1, nc + 1):
        Rm[I, 2 * I - 1] = 0.25
        Rm[I, 2 * I] = 0.5
        Rm[I, 2 * I + 1] = 0.25
    return Rm


def restrict_kappa(kappa: np.ndarray, d: int) -> np.ndarray:
    n = kappa.shape[-1] - 2
    Rm = kappa_restriction_1d(n)
    out = kappa
    for a in range(d):
        ax = out.ndim - d + a
        out = np.moveaxis(np.tensordot(Rm, out, axes=(1, ax)), 0, ax)
    return out


def restrict(r: np.ndarray, d: int) -> np.ndarray:
    """Full weighting: coarse node I <- (1/4, 1/2, 1/4) at fine nodes 2I-1, 2I, 2I+1 per axis."""
    out = r
    for a in range(d):
        ax = out.ndim - d + a
        n = out.shape[ax]

        def s(sl):
            idx = [slice(None)] * out.ndim
            idx[ax] = sl
            return tuple(idx)
        out = 0.25 * out[s(slice(0, n - 1, 2))] + 0.5 * out[s(slice(1, n, 2))] + 0.25 * out[s(slice(2, n + 1, 2))]
    return out


def prolong(e: np.ndarray, d: int) -> np.ndarray:
    """Multilinear interpolation, zero on the boundary."""
    out = e
    for a in range(d):
        ax = out.ndim - d + a
        nc = out.shape[ax]
        n = 2 * nc + 1
        pad = [(0, 0)] * out.ndim
        pad[ax] = (1, 1)
        ep = np.pad(out, pad)
        shape = list(out.shape)
        shape[ax] = n
        fine = np.zeros(shape)

        def s(arr_len, sl):
            idx = [slice(None)] * out.ndim
            idx[ax] = sl
            return tuple(idx)
        fine[s(n, slice(1, n, 2))] = ep[s(nc + 2, slice(1, nc + 1))]
        fine[s(n, slice(0, n, 2))] = 0.5 * (ep[s(nc + 2, slice(0, nc + 1))] + ep[s(nc + 2, slice(1, nc + 2))])
        out = fine
    return out


class Level:
    def __init__(self, kfields: np.ndarray, n: int, d: int):
        self.n = n
        self.d = d
        self.h = 1.0 / (n + 1)
        self.kfields = kfields                      # (R,) + (n+2,)*d
        self.diag_r = fd.diagonal(kfields, self.h, d)  # (R,) + (n,)*d

    def _cb(self, c, x):
        return c.reshape(c.shape + (1,) * self.d)

    def op(self, sigma, c, x):
        """L_s x_s = sigma_s x_s + sum_r c_{s,r} A(kappa_r) x_s."""
        out = self._cb(sigma, x) * x
        for r in range(self.kfields.shape[0]):
            out = out + self._cb(c[:, r], x) * fd.apply(self.kfields[r], x, self.h, self.d)
        return out

    def diag(self, sigma, c):
        D = self._cb(sigma, self.diag_r[0]) * np.ones_like(self.diag_r[0])
        for r in range(self.kfields.shape[0]):
            D = D + self._cb(c[:, r], self.diag_r[0]) * self.diag_r[r]
        return D


class Hierarchy:
    def __init__(self, kfields: np.ndarray, n: int, d: int):
        self.d = d
        self.levels = [Level(np.asarray(kfields, dtype=np.float64), n, d)]
        while n > 1:
            if n % 2 == 0:
                raise ValueError("multigrid needs n = 2^L - 1 interior nodes per axis")
            kfields = np.stack([restrict_kappa(kfields[r], d) for r in range(kfields.shape[0])])
            n = (n - 1) // 2
            self.levels.append(Level(kfields, n, d))

    def vcycle(self, sigma, c, b, l: int = 0):
        """One V-cycle for the slab operators (sigma_s, c_s) on level l, zero initial guess."""
        lev = self.levels[l]
        D = lev.diag(sigma, c)
        if l == len(self.levels) - 1:
            return b / D
        W = JACOBI_WEIGHT[self.d] / D
        x1 = W * b
        r = b - lev.op(sigma, c, x1)
        e = self.vcycle(sigma, c, restrict(r, self.d), l + 1)
        x2 = x1 + prolong(e, self.d)
        return x2 + W * (b - lev.op(sigma, c, x2))

    def vcycles(self, sigma, c, b, nu: int = 1):
        """nu V-cycles (each subsequent one applied to the current residual)."""
        x = self.vcycle(sigma, c, b)
        for _ in range(nu - 1):
            x = x + self.vcycle(sigma, c, b - self.levels[0].op(sigma, c, x))
        return x

    def apply_op(self, sigma, c, x):
        return self.levels[0].op(sigma, c, x)
