"""The change of temporal basis of Section 4.

* mu_k = 2 sin((2k-1) pi / (4N)), eq. (4.5).
* Phi (eq. (4.2), type-III DST with weight 1/2 on n = N):
      uhat_k = (2/N) sum_n w_n u_n sin((2k-1) n pi / (2N)),   w_n = 1/(1 + delta_{nN}).
* Phi^{-1} (eq. (4.3), type-II DST):  u_n = sum_k uhat_k sin((2k-1) n pi / (2N)).

All transforms act on the leading (time) axis of an array shaped (N, ...).
Written as dense sums (the plain definition) up to N = 4096; above that the
N x N sine matrix no longer fits comfortably in memory and the same maps are
evaluated through scipy's unnormalised DST-II/III (a library FFT used as a
step; the reduction is pinned against the dense sums in the tests).  The fast
algorithms of the GPU are its own business.
"""
from __future__ import annotations

import numpy as np
import scipy.fft as sfft

DENSE_MAX_N = 4096


def sine_matrix(N: int) -> np.ndarray:
    """S[n-1, k-1] = sin((2k-1) n pi / (2N)), n, k = 1..N  (the matrix of Phi^{-1})."""
    n = np.arange(1, N + 1)[:, None]
    k = np.arange(1, N + 1)[None, :]
    return np.sin((2 * k - 1) * n * np.pi / (2 * N))


def weights(N: int) -> np.ndarray:
    w = np.ones(N)
    w[-1] = 0.5
    return w


def mu(N: int) -> np.ndarray:
    k = np.arange(1, N + 1)
    return 2.0 * np.sin((2 * k - 1) * np.pi / (4 * N))


def phi_matrix(N: int) -> np.ndarray:
    """Matrix of Phi, eq. (4.2): (2/N) S^T diag(w)."""
    return (2.0 / N) * sine_matrix(N).T * weights(N)[None, :]


def _along_time(Mat: np.ndarray, x: np.ndarray) -> np.ndarray:
    return np.tensordot(Mat, x, axes=(1, 0))


def forward(u: np.ndarray) -> np.ndarray:
    """uhat = Phi u (= dst3(u) / N)."""
    N = u.shape[0]
    if N > DENSE_MAX_N:
        return sfft.dst(u, type=3, axis=0) / N
    return _along_time(phi_matrix(N), u)


def inverse(uhat: np.ndarray) -> np.ndarray:
    """u = Phi^{-1} uhat (= dst2(uhat) / 2)."""
    if uhat.shape[0] > DENSE_MAX_N:
        return 0.5 * sfft.dst(uhat, type=2, axis=0)
    return _along_time(sine_matrix(uhat.shape[0]), uhat)


def inverse_transpose(r: np.ndarray) -> np.ndarray:
    """Phi^{-T} r = S^T r: rhat_k = sum_n sin((2k-1) n pi/(2N)) r_n
    (= dst3(r with r_N doubled) / 2)."""
    if r.shape[0] > DENSE_MAX_N:
        r2 = np.array(r, dtype=np.float64, copy=True)
        r2[-1] *= 2
        return 0.5 * sfft.dst(r2, type=3, axis=0)
    return _along_time(sine_matrix(r.shape[0]).T, r)
