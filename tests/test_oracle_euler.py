"""Pins for the oracle's sequential implicit Euler (eq. (2.1))."""
import numpy as np
import pytest
import scipy.fft as sfft

import synth
from oracle import euler, fd, spacetime as st


def _sine(n, d, ks):
    x = np.arange(1, n + 1) / (n + 1)
    out = 1.0
    for a, k in enumerate(ks):
        shape = [1] * d
        shape[a] = n
        out = out * np.sin(k * np.pi * x).reshape(shape)
    return out


@pytest.mark.parametrize("d,n,N", [(1, 31, 20), (2, 15, 12), (3, 7, 6)])
def test_sine_mode_decay_closed_form(d, n, N):
    """kappa spatially constant, F = 0, u0 a sine mode:
    u_n = prod_{m<=n} (1 + tau kappa(t_m) lambda_k)^{-1} u0."""
    T = 1.0
    t = T * np.arange(1, N + 1) / N
    ks = [2, 1, 3][:d]
    prob = synth.Problem(d, n, N, T, np.ones((1,) + (n + 2,) * d),
                         (1 + 0.5 * np.sin(2 * np.pi * t))[None, :],
                         np.zeros((N,) + (n,) * d), _sine(n, d, ks))
    lam = fd.laplace_eigenvalue(ks, prob.h)
    u = euler.seq_euler(prob)
    fac = np.cumprod(1.0 / (1.0 + prob.tau * prob.tcoef[0] * lam))
    exact = fac.reshape((N,) + (1,) * d) * prob.u0
    assert np.allclose(u, exact, rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("d,n,N", [(1, 63, 64), (2, 31, 16)])
def test_modal_recurrence_with_source(d, n, N):
    """kappa = kappa(t) only: a spatial DST-I diagonalises every A_n, so each mode
    follows uh_n = (uh_{n-1} + tau Fh_n) / (1 + tau kappa(t_n) lambda_k)
    (an independent route through scipy's DST-I)."""
    prob = synth.heat1d_random(n=n, N=N) if d == 1 else synth.small_problem(d, n, N, R=1)
    axes = tuple(range(-d, 0))
    Fh = sfft.dstn(prob.F, type=1, axes=axes)
    uh = sfft.dstn(prob.u0, type=1, axes=axes)
    ks = np.arange(1, n + 1)
    lam1 = 4 * (n + 1) ** 2 * np.sin(ks * np.pi / (2 * (n + 1))) ** 2
    lam = sum(np.meshgrid(*([lam1] * d), indexing="ij"))
    out = []
    for m in range(N):
        uh = (uh + prob.tau * Fh[m]) / (1 + prob.tau * prob.tcoef[0, m] * lam)
        out.append(sfft.idstn(uh, type=1, axes=axes))
    u = euler.seq_euler(prob)
    assert np.allclose(u, np.array(out), rtol=1e-11, atol=1e-12)


@pytest.mark.parametrize("d,n,N", [(1, 15, 9), (2, 7, 5), (3, 3, 4)])
def test_time_global_system(d, n, N):
    """The sequential solution satisfies the time-global system B u = f, eq. (2.3)."""
    prob = synth.small_problem(d, n, N)
    u = euler.seq_euler(prob)
    f = st.rhs(prob)
    assert np.linalg.norm(st.apply_B(prob, u) - f) <= 1e-13 * np.linalg.norm(f)


def test_cg_route_matches_lu():
    prob = synth.small_problem(3, 15, 3)
    a = euler.seq_euler(prob, method="lu")
    b = euler.seq_euler(prob, method="cg", rtol=1e-14)
    assert np.allclose(a, b, rtol=1e-11, atol=1e-12)
