"""Reproduce Section 8.1, Table 1 (extremal eigenvalues of H^{-1} S, 1-D P1 FEM)."""
import os

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import fem1d, spacetime as st, spectral

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table1.txt")


def _rows():
    rows = []
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        ih, N, lo, hi, kap = line.split()
        rows.append((int(ih), int(N), float(lo), float(hi), float(kap)))
    return rows


@pytest.mark.parametrize("n,N", [(5, 4), (7, 6)])
def test_mode_reduction_matches_full_matrices(n, N):
    """The per-mode reduction gives the same spectrum as the assembled S and H."""
    M, A = fem1d.mass(n), fem1d.stiffness(n)
    tau = 1.0 / N
    S = st.dense_system(M, [A] * N, [tau] * N)["S"]
    H = st.dense_H(M, A, tau, N)
    full = np.sort(sla.eigh(S, H, eigvals_only=True))
    parts = []
    for lam in fem1d.generalized_eigenvalues(n):
        Sj, Hj = spectral.mode_blocks(N, tau * lam)
        parts += list(sla.eigh(Sj, Hj, eigvals_only=True))
    assert np.allclose(full, np.sort(parts), rtol=1e-9)


def _check(ih, N, lo, hi, kap):
    lam = fem1d.generalized_eigenvalues(ih - 1)
    glo, ghi = spectral.extreme_eigs_per_mode(N, lam, 1.0 / N)
    # every printed digit must be reproduced
    assert round(glo, 4) == pytest.approx(lo, abs=1e-12)
    assert round(ghi, 4) == pytest.approx(hi, abs=1e-12)
    assert round(ghi / glo, 4) == pytest.approx(kap, abs=1e-12)


@pytest.mark.parametrize("row", [r for r in _rows() if r[1] <= 256], ids=lambda r: f"h1/{r[0]}-N{r[1]}")
def test_table1(row):
    _check(*row)


@pytest.mark.parametrize("row", [r for r in _rows() if r[1] > 256], ids=lambda r: f"h1/{r[0]}-N{r[1]}")
def test_table1_large_N(row):
    """N = 512, 1024: about 90 s of dense eigen-solves on 8 cores."""
    _check(*row)
