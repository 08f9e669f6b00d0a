"""1-D P1 finite elements on a uniform mesh of (0,1) with h = 1/(n+1) and
homogeneous Dirichlet conditions: the spatial matrices of the Section 8.1
experiment (Table 1).

    M = (h/6) tridiag(1, 4, 1),   A = (1/h) tridiag(-1, 2, -1).
"""
from __future__ import annotations

import numpy as np


def mass(n: int) -> np.ndarray:
    h = 1.0 / (n + 1)
    return (h / 6.0) * (4 * np.eye(n) + np.eye(n, k=1) + np.eye(n, k=-1))


def stiffness(n: int) -> np.ndarray:
    h = 1.0 / (n + 1)
    return (1.0 / h) * (2 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1))


def generalized_eigenvalues(n: int) -> np.ndarray:
    """Eigenvalues of A v = lambda M v (sine eigenvectors):
    lambda_j = (6/h^2) (1 - cos(j pi h)) / (2 + cos(j pi h)), j = 1..n."""
    h = 1.0 / (n + 1)
    c = np.cos(np.arange(1, n + 1) * np.pi * h)
    return (6.0 / h ** 2) * (1 - c) / (2 + c)
