"""Finite-difference spatial operator A(kappa) = -div(kappa grad .) on the unit
d-cube with homogeneous Dirichlet conditions (d = 1, 2, 3).

The paper leaves the spatial discretisation abstract (Section 2: M and A_n are
any SPD matrices).  For the finite-difference workloads we take the lumped
mass M = I and the standard conservative 3/5/7-point scheme

    (A u)_i = h^{-2} * sum over the 2d faces f of node i of kappa_f (u_i - u_nb(f)),

with face coefficient kappa_f = arithmetic mean of the two nodal values it
joins and u = 0 on boundary nodes.  kappa is given on all (n+2)^d nodes.

Arrays are laid out (z, y, x) with the last axis x; ``apply`` and
``diagonal`` accept leading batch axes.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def _sl(ndim, axis, s):
    idx = [slice(None)] * ndim
    idx[axis] = s
    return tuple(idx)


def _face_kappa(kappa: np.ndarray, d: int, a: int, n: int) -> np.ndarray:
    """Face coefficients along spatial axis a (0 = first of the d trailing axes):
    faces i+1/2, i = 0..n, restricted to interior nodes in the other axes."""
    kd = kappa.ndim
    other = [slice(None)] * kd
    for b in range(d):
        if b != a:
            other[kd - d + b] = slice(1, n + 1)
    ka = kappa[tuple(other)]
    ax = kd - d + a
    return 0.5 * (ka[_sl(kd, ax, slice(0, n + 1))] + ka[_sl(kd, ax, slice(1, n + 2))])


def apply(kappa: np.ndarray, u: np.ndarray, h: float, d: int) -> np.ndarray:
    """Matrix-free A(kappa) u.  kappa: (..., n+2 [x d]); u: (..., n [x d])."""
    n = u.shape[-1]
    nd = u.ndim
    lead = u.shape[: nd - d]
    up = np.zeros(lead + (n + 2,) * d)
    up[(Ellipsis,) + (slice(1, n + 1),) * d] = u
    out = np.zeros(u.shape)
    for a in range(d):
        ax = nd - d + a
        other = [slice(None)] * nd
        for b in range(d):
            if b != a:
                other[nd - d + b] = slice(1, n + 1)
        upa = up[tuple(other)]
        kf = _face_kappa(kappa, d, a, n)
        flux = kf * (upa[_sl(nd, ax, slice(1, n + 2))] - upa[_sl(nd, ax, slice(0, n + 1))])
        out -= flux[_sl(nd, ax, slice(1, n + 1))] - flux[_sl(nd, ax, slice(0, n))]
    return out / (h * h)


def diagonal(kappa: np.ndarray, h: float, d: int) -> np.ndarray:
    """diag(A(kappa)) on the interior nodes: h^{-2} * sum of the 2d face coefficients."""
    n = kappa.shape[-1] - 2
    kd = kappa.ndim
    out = np.zeros(kappa.shape[: kd - d] + (n,) * d)
    for a in range(d):
        ax = kd - d + a
        kf = _face_kappa(kappa, d, a, n)
        out += kf[_sl(kd, ax, slice(0, n))] + kf[_sl(kd, ax, slice(1, n + 1))]
    return out / (h * h)


def assemble_loops(kappa: np.ndarray, n: int, d: int, h: float) -> sp.csr_matrix:
    """Sparse A(kappa) built by an explicit loop over every face of the node
    grid (slow; an independent route to the operator for small n)."""
    idx = np.arange(n ** d).reshape((n,) * d)
    rows, cols, vals = [], [], []
    diag = np.zeros((n,) * d)
    for a in range(d):
        for node in np.ndindex(*((n + 2,) * d)):
            if node[a] == n + 1:
                continue
            if not all(1 <= node[b] <= n for b in range(d) if b != a):
                continue
            nb = list(node)
            nb[a] += 1
            nb = tuple(nb)
            w = 0.5 * (kappa[node] + kappa[nb]) / (h * h)
            i_in = 1 <= node[a] <= n
            j_in = 1 <= nb[a] <= n
            if i_in:
                diag[tuple(c - 1 for c in node)] += w
            if j_in:
                diag[tuple(c - 1 for c in nb)] += w
            if i_in and j_in:
                i = idx[tuple(c - 1 for c in node)]
                j = idx[tuple(c - 1 for c in nb)]
                rows += [i, j]
                cols += [j, i]
                vals += [-w, -w]
    rows += list(range(n ** d))
    cols += list(range(n ** d))
    vals += list(diag.ravel())
    return sp.csr_matrix((vals, (rows, cols)), shape=(n ** d, n ** d))


def assemble(kappa: np.ndarray, n: int, d: int, h: float) -> sp.csr_matrix:
    """Sparse A(kappa), vectorised assembly (same entries as ``assemble_loops``)."""
    Np = n ** d
    idx = np.arange(Np).reshape((n,) * d)
    rows, cols, vals = [], [], []
    for a in range(d):
        kf = _face_kappa(kappa, d, a, n) / (h * h)          # faces 0..n along a
        inner = kf[_sl(d, a, slice(1, n))]                   # faces between interior nodes
        i0 = idx[_sl(d, a, slice(0, n - 1))]
        i1 = idx[_sl(d, a, slice(1, n))]
        rows += [i0.ravel(), i1.ravel()]
        cols += [i1.ravel(), i0.ravel()]
        vals += [-inner.ravel(), -inner.ravel()]
    rows.append(np.arange(Np))
    cols.append(np.arange(Np))
    vals.append(diagonal(kappa, h, d).ravel())
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(Np, Np))


def laplace_eigenvalue(ks, h: float) -> float:
    """Eigenvalue of the constant-coefficient (kappa = 1) operator for the sine
    mode prod_a sin(k_a pi x_a): sum_a (4/h^2) sin^2(k_a pi h / 2)."""
    return float(sum(4.0 / h ** 2 * np.sin(k * np.pi * h / 2) ** 2 for k in ks))


def kappa_at(prob_kfields: np.ndarray, tcoef_col: np.ndarray) -> np.ndarray:
    """kappa(t_n, .) = sum_r tcoef[r, n-1] * kfields[r] (nodal)."""
    return np.tensordot(tcoef_col, prob_kfields, axes=(0, 0))
