"""Dense-matrix constructions used by several oracle pin tests (tiny sizes).

These are written from the definitions, independently of the oracle's
matrix-free code, so that a test can compare the two."""
import numpy as np

from oracle import fd, mg


def R1(n):
    """Full-weighting restriction along one axis as an (n_c x n) matrix."""
    nc = (n - 1) // 2
    R = np.zeros((nc, n))
    for I in range(nc):
        R[I, 2 * I:2 * I + 3] = [0.25, 0.5, 0.25]
    return R


def kron_d(M1, d):
    out = M1
    for _ in range(d - 1):
        out = np.kron(out, M1)
    return out


def dense_vcycle(hier, sigma, c, l=0):
    """V-cycle as a matrix: V = (I - E) L^{-1}, E = (I - W L)(I - P V_c R L)(I - W L),
    with the level operators assembled by ``fd.assemble`` on each level's fields."""
    lev = hier.levels[l]
    d = hier.d
    n = lev.n
    m = n ** d
    Ar = [fd.assemble(lev.kfields[r], n, d, lev.h).toarray() for r in range(lev.kfields.shape[0])]
    L = sigma * np.eye(m) + sum(c[r] * Ar[r] for r in range(len(Ar)))
    D = np.diag(np.diag(L))
    if l == len(hier.levels) - 1:
        return np.linalg.inv(D), L
    W = mg.JACOBI_WEIGHT[d] * np.linalg.inv(D)
    Rd = kron_d(R1(n), d)
    Pd = (2 ** d) * Rd.T
    Vc, _ = dense_vcycle(hier, sigma, c, l + 1)
    I = np.eye(m)
    E = (I - W @ L) @ (I - Pd @ Vc @ Rd @ L) @ (I - W @ L)
    return (I - E) @ np.linalg.inv(L), L


def dense_vcycles(hier, sigma, c, nu):
    """nu cycles, each on the residual the earlier ones leave:
    (I - (I - V L)^nu) L^{-1}."""
    V, L = dense_vcycle(hier, sigma, c)
    E = np.eye(L.shape[0]) - V @ L
    return (np.eye(L.shape[0]) - np.linalg.matrix_power(E, nu)) @ np.linalg.inv(L)
