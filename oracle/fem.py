"""Finite-element spatial matrices and the space-time method with a general
SPD mass matrix (Section 2: M and A_n are any SPD matrices; the experiments of
Section 8 use P1 elements in 1-D and 2-D and Q1 hexahedra in 3-D).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Meshes: the unit d-cube with n interior nodes per axis, h = 1/(n+1),
homogeneous Dirichlet conditions, constant coefficient 1 in space (the
paper's experiments); a time factor a(t_n) scales the stiffness,
A_n = a_n A.  Matrices are assembled element by element from the local
element matrices, dropping the boundary nodes:

* 1-D P1: element [x_i, x_{i+1}], mass (h/6)[[2,1],[1,2]], stiffness (1/h)[[1,-1],[-1,1]].
* 2-D P1: every mesh square split by its diagonal from the lower-left to the
  upper-right corner; triangle mass (area/12)[[2,1,1],[1,2,1],[1,1,2]],
  stiffness area * G G^T with G the gradients of the barycentric functions.
* 3-D Q1: trilinear hexahedra; element mass = tensor product of the 1-D
  element masses, stiffness = sum over axes of (1-D element stiffness along
  the axis) x (1-D element masses along the others).

The time-global operators follow Section 2 with a general M:
    K = (lower bidiagonal 1, -1) (x) M,  A = diag(tau_n A_n),  B = K + A,
    f = [tau_1 M F_1 + M u_I, tau_2 M F_2, ...]   (F_n: nodal source values),
and the preconditioners of eqs. (3.2), (4.4)-(4.6) with H_k = mu_k M + tau A.
Spatial solves: exact (sparse LU) or the multigrid V-cycle of ``vcycle`` on
Galerkin coarse operators L_{l+1} = R L_l P, where P is the finite-element
interpolation from the coarse mesh (every second node) and R = P^T / 2^d.
"""
from __future__ import annotations

import dataclasses
import itertools

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import dst

# Smoother: damped l1-Jacobi, x <- x + theta (b - L x) / l1 with l1 the largest
# absolute row sum of L = sigma M + c A (a Gershgorin bound of lambda_max(D^{-1} L)
# times the constant diagonal, so theta < 2 keeps every sweep contracting for
# every mix of mass and stiffness); theta chosen by the measured V-cycle
# contraction (tests/test_oracle_fem.py)
L1_THETA = 1.6


# ---------------------------------------------------------------------------
# assembly
# ---------------------------------------------------------------------------
def _assemble(n, d, elements):
    """elements: iterable of (node tuple list, Me, Ae) with nodes in (x, y, z)
    order 0..n+1.  Returns sparse (M, A) on the interior nodes, index
    ((z-1) n + (y-1)) n + (x-1)."""
    rows, cols, mv, av = [], [], [], []

    def gidx(node):
        if any(c < 1 or c > n for c in node):
            return -1
        i = 0
        for c in reversed(node):          # z slowest, x fastest
            i = i * n + (c - 1)
        return i
    for nodes, Me, Ae in elements:
        g = [gidx(nd) for nd in nodes]
        for a, ga in enumerate(g):
            if ga < 0:
                continue
            for b, gb in enumerate(g):
                if gb < 0:
                    continue
                rows.append(ga)
                cols.append(gb)
                mv.append(Me[a, b])
                av.append(Ae[a, b])
    m = n ** d
    M = sp.csr_matrix((mv, (rows, cols)), shape=(m, m))
    A = sp.csr_matrix((av, (rows, cols)), shape=(m, m))
    M.sum_duplicates()
    A.sum_duplicates()
    return M, A


def _p1_1d(n):
    h = 1.0 / (n + 1)
    Me = (h / 6.0) * np.array([[2.0, 1.0], [1.0, 2.0]])
    Ae = (1.0 / h) * np.array([[1.0, -1.0], [-1.0, 1.0]])
    return [([(i,), (i + 1,)], Me, Ae) for i in range(n + 1)]


def _triangle(pts):
    """Mass and stiffness of the P1 triangle with vertices pts (3 x 2)."""
    P = np.hstack([np.ones((3, 1)), np.asarray(pts, dtype=float)])
    area = 0.5 * abs(np.linalg.det(P))
    G = np.linalg.inv(P)[1:, :].T          # rows: gradients of the barycentric functions
    Me = (area / 12.0) * (np.ones((3, 3)) + np.eye(3))
    Ae = area * G @ G.T
    return Me, Ae


def _p1_2d(n):
    h = 1.0 / (n + 1)
    out = []
    for j in range(n + 1):
        for i in range(n + 1):
            sw, se, nw, ne = (i, j), (i + 1, j), (i, j + 1), (i + 1, j + 1)
            for tri in ((sw, se, ne), (sw, ne, nw)):
                Me, Ae = _triangle([(a * h, b * h) for a, b in tri])
                out.append((list(tri), Me, Ae))
    return out


def _q1(n, d):
    h = 1.0 / (n + 1)
    m1 = (h / 6.0) * np.array([[2.0, 1.0], [1.0, 2.0]])
    k1 = (1.0 / h) * np.array([[1.0, -1.0], [-1.0, 1.0]])

    def kron_axes(mats):        # mats[a]: 2x2 factor along axis a; local index bits (x, y, z)
        out = np.ones((2 ** d, 2 ** d))
        for p, bp in enumerate(itertools.product((0, 1), repeat=d)):
            for q, bq in enumerate(itertools.product((0, 1), repeat=d)):
                v = 1.0
                for a in range(d):
                    v *= mats[a][bp[d - 1 - a], bq[d - 1 - a]]
                out[p, q] = v
        return out
    Me = kron_axes([m1] * d)
    Ae = sum(kron_axes([k1 if b == a else m1 for b in range(d)]) for a in range(d))
    out = []
    for corner in itertools.product(range(n + 1), repeat=d):   # (z, y, x)
        nodes = []
        for bits in itertools.product((0, 1), repeat=d):       # (z, y, x) bits
            nodes.append(tuple(corner[d - 1 - a] + bits[d - 1 - a] for a in range(d)))   # (x, y, z)
        out.append((nodes, Me, Ae))
    return out


def matrices(dim: int, n: int):
    """(M, A) of the paper's element for this dimension: P1 (1-D, 2-D), Q1 (3-D)."""
    if dim == 1:
        return _assemble(n, 1, _p1_1d(n))
    if dim == 2:
        return _assemble(n, 2, _p1_2d(n))
    return _assemble(n, 3, _q1(n, 3))


# ---------------------------------------------------------------------------
# multigrid transfer and V-cycle (Galerkin coarse operators)
# ---------------------------------------------------------------------------
def prolongation(dim: int, n: int) -> sp.csr_matrix:
    """Finite-element interpolation from the mesh with (n-1)/2 interior nodes per
    axis (every second node) to the mesh with n: nodal values of the coarse
    function at the fine nodes.  P1 in 2-D interpolates linearly on the coarse
    triangles (a fine node at the centre of a coarse square takes the mean of
    the square's lower-left and upper-right corners)."""
    nc = (n - 1) // 2
    hc = 1.0 / (nc + 1)
    h = 1.0 / (n + 1)
    rows, cols, vals = [], [], []
    for fine in itertools.product(range(1, n + 1), repeat=dim):   # (z, y, x)
        xf = [fine[dim - 1 - a] * h for a in range(dim)]           # (x, y, z) coordinates
        fi = 0
        for c in fine:
            fi = fi * n + (c - 1)
        # value at the fine node of every coarse nodal basis function whose
        # support contains it (coarse index floor(f/2) or ceil(f/2) per axis)
        cand = [sorted({f // 2, (f + 1) // 2} & set(range(1, nc + 1))) for f in fine]
        for coarse in itertools.product(*cand):
            xc = [coarse[dim - 1 - a] * hc for a in range(dim)]
            t = [(xf[a] - xc[a]) / hc for a in range(dim)]
            if dim == 2:
                v = _p1_hat(t[0], t[1])
            else:
                v = float(np.prod([max(0.0, 1.0 - abs(ta)) for ta in t]))
            if v != 0.0:
                ci = 0
                for c in coarse:
                    ci = ci * nc + (c - 1)
                rows.append(fi)
                cols.append(ci)
                vals.append(v)
    return sp.csr_matrix((vals, (rows, cols)), shape=(n ** dim, nc ** dim))


def _p1_hat(tx, ty):
    """P1 nodal basis function of the node at the origin on the triangulation
    with lower-left/upper-right diagonals, at offset (tx, ty) in mesh units."""
    if tx >= 0 and ty >= 0:
        return max(0.0, 1.0 - max(tx, ty))
    if tx <= 0 and ty <= 0:
        return max(0.0, 1.0 - max(-tx, -ty))
    return max(0.0, 1.0 - abs(tx) - abs(ty))


class Hierarchy:
    """Operators sigma M + c A on nested meshes down to one interior node, with
    Galerkin coarse matrices R L P (R = P^T / 2^d)."""

    def __init__(self, dim: int, n: int):
        self.dim = dim
        self.ns = [n]
        self.P = []
        while n > 1:
            if n % 2 == 0:
                raise ValueError("multigrid needs n = 2^L - 1 interior nodes per axis")
            self.P.append(prolongation(dim, n))
            n = (n - 1) // 2
            self.ns.append(n)
        M, A = matrices(dim, self.ns[0])
        self.M = [M]
        self.A = [A]
        for P in self.P:
            R = P.T / 2 ** dim
            self.M.append((R @ self.M[-1] @ P).tocsr())
            self.A.append((R @ self.A[-1] @ P).tocsr())

    def vcycle(self, sigma: float, c: float, b: np.ndarray, l: int = 0, sweeps: int = 1) -> np.ndarray:
        """One V-cycle for sigma M + c A on level l from the zero guess with
        ``sweeps`` l1-Jacobi sweeps x <- x + W (b - L x), W = theta / l1, before
        and after the coarse correction x <- x + P V_{l+1}(R (b - L x)); the
        one-node level is solved exactly."""
        L = sigma * self.M[l] + c * self.A[l]
        if l == len(self.ns) - 1:
            return b / L.diagonal()
        W = L1_THETA / abs(L).sum(axis=1).max()
        P = self.P[l]
        x = W * b
        for _ in range(sweeps - 1):
            x = x + W * (b - L @ x)
        x = x + P @ self.vcycle(sigma, c, (P.T @ (b - L @ x)) / 2 ** self.dim, l + 1, sweeps)
        for _ in range(sweeps):
            x = x + W * (b - L @ x)
        return x


# ---------------------------------------------------------------------------
# the space-time method with a general mass matrix
# ---------------------------------------------------------------------------
@dataclasses.dataclass
class FemProblem:
    dim: int
    n: int
    N: int
    T: float
    a: np.ndarray          # (N,) time factor of the stiffness at t_n
    F: np.ndarray          # (N, n^d) nodal source values at t_n
    u0: np.ndarray         # (n^d,) nodal initial datum

    @property
    def tau(self):
        return self.T / self.N

    @property
    def npts(self):
        return self.n ** self.dim


def rhs(prob, M):
    f = prob.tau * (M @ prob.F.T).T
    f[0] += M @ prob.u0
    return f


def seq_euler(prob):
    """(M + tau a_n A) u_n = M u_{n-1} + tau M F_n, u_0 = u0 (eq. (2.1)), by sparse LU."""
    M, A = matrices(prob.dim, prob.n)
    u = prob.u0.astype(float).copy()
    out = np.empty((prob.N, prob.npts))
    for m in range(prob.N):
        u = spla.spsolve((M + prob.tau * prob.a[m] * A).tocsc(), M @ (u + prob.tau * prob.F[m]))
        out[m] = u
    return out


def apply_B(prob, M, A, x):
    """(K + A) x with K = bidiag (x) M, A = diag(tau a_n A)."""
    y = (M @ x.T).T
    y[1:] -= (M @ x[:-1].T).T
    return y + prob.tau * prob.a[:, None] * (A @ x.T).T


class Preconditioners:
    """A-tilde^{-1} (eq. (3.2)) and H-tilde^{-1} (eq. (4.6)) with M; spatial
    solves exact (``spatial="exact"``) or one V-cycle (``"mg"``) with
    ``sweeps`` Jacobi sweeps per side.  The reference operator of H is a_ref A
    with a_ref the time mean of a_n."""

    def __init__(self, prob, spatial="mg", sweeps=1):
        self.prob = prob
        self.spatial = spatial
        self.sweeps = sweeps
        N, tau = prob.N, prob.tau
        self.M, self.A = matrices(prob.dim, prob.n)
        self.aref = float(np.mean(prob.a))
        self.mu = dst.mu(N)
        if spatial == "mg":
            self.hier = Hierarchy(prob.dim, prob.n)
        else:
            self.luA = [spla.splu((tau * prob.a[i] * self.A).tocsc()) for i in range(N)]
            self.luH = [spla.splu((self.mu[k] * self.M + tau * self.aref * self.A).tocsc()) for k in range(N)]

    def _solve(self, which, b):
        tau = self.prob.tau
        out = np.empty_like(b)
        for i in range(b.shape[0]):
            if self.spatial == "mg":
                sig, c = (0.0, tau * self.prob.a[i]) if which == "A" else (self.mu[i], tau * self.aref)
                out[i] = self.hier.vcycle(sig, c, b[i], sweeps=self.sweeps)
            else:
                out[i] = (self.luA if which == "A" else self.luH)[i].solve(b[i])
        return out

    def Ainv(self, r):
        return self._solve("A", r)

    def Hinv(self, r):
        """Phi^{-1} diag_k((2 tau / N) H~_k^{-1} a_ref A H~_k^{-1}) Phi^{-T} r."""
        N, tau = self.prob.N, self.prob.tau
        x = self._solve("H", dst.inverse_transpose(r))
        y = (2.0 * tau / N) * self.aref * (self.A @ x.T).T
        return dst.inverse(self._solve("H", y))


def uzawa(prob, omega=0.8, tol=1e-8, max_iter=500, spatial="mg", pc=None, callback=None):
    """The inexact Uzawa iteration (3.1) with M, from zero; stop at the first j
    with ||f - B u_j|| <= tol ||f|| (tested after the p-update, as for the
    finite-difference problems)."""
    pc = pc or Preconditioners(prob, spatial)
    M, A = pc.M, pc.A
    f = rhs(prob, M)
    fn = np.linalg.norm(f)
    u = np.zeros_like(f)
    p = np.zeros_like(f)
    tauA = lambda x: prob.tau * prob.a[:, None] * (A @ x.T).T   # noqa: E731
    Kx = lambda x: apply_B(prob, M, A, x) - tauA(x)              # noqa: E731

    def KTx(x):
        y = (M @ x.T).T
        y[:-1] -= (M @ x[1:].T).T
        return y
    hist = []
    j = 0
    status = "maxiter"
    while True:
        Ku = Kx(u)
        p = p + pc.Ainv(Ku - tauA(p) - f)
        res = np.linalg.norm(f - Ku - tauA(u))
        hist.append(res / fn)
        if callback is not None:
            callback(j, u, p, res / fn)
        if not np.isfinite(res):
            status = "diverged"
            break
        if res <= tol * fn:
            status = "converged"
            break
        if j >= max_iter:
            break
        ru = f - KTx(p) - (Ku + KTx(u) + tauA(u))
        u = u + omega * pc.Hinv(ru)
        j += 1
    return dict(u=u, p=p, iters=j, history=np.array(hist), status=status)


def s_norm(prob, v) -> float:
    """||v||_S by the identity of Theorem 6.2 with a mass matrix:
    v^T S v = sum_n [ (1/tau_n) |dv_n|^2_{M A_n^{-1} M} + tau_n |v_n|^2_{A_n} + |dv_n|^2_M ] + |v_N|^2_M,
    dv_n = v_n - v_{n-1}, v_0 = 0, A_n = a_n A (sparse LU of A)."""
    M, A = matrices(prob.dim, prob.n)
    lu = spla.splu(A.tocsc())
    tau = prob.tau
    total = 0.0
    prev = np.zeros(prob.npts)
    for i in range(prob.N):
        vi = v[i]
        dv = vi - prev
        Mdv = M @ dv
        total += (Mdv @ lu.solve(Mdv)) / (tau * prob.a[i]) + tau * prob.a[i] * (vi @ (A @ vi)) + dv @ Mdv
        prev = vi
    total += prev @ (M @ prev)
    return float(np.sqrt(total))


def stationary(prob, pc, omega, iters):
    """The iterates u_0..u_iters of the Uzawa iteration (3.1) with M (no stop test)."""
    out = []
    uzawa(prob, omega=omega, tol=0.0, max_iter=iters, pc=pc, callback=lambda j, u, p, r: out.append(u.copy()))
    return out
