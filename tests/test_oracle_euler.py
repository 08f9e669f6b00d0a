"""Pins for the oracle's sequential implicit Euler (eq. (2.1))."""
import numpy as np
import pytest

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


@pytest.mark.parametrize("d,n,N,graded", [(1, 63, 64, False), (2, 31, 16, False), (2, 15, 12, True), (3, 7, 6, False)])
def test_modal_route_matches_lu(d, n, N, graded):
    """kappa = kappa(t) only: the sine-transform route (``seq_euler_modal``)
    equals the sparse-LU route step by step."""
    steps = synth.graded_steps(N, ratio=5.0, jitter=0.2, seed=3) if graded else None
    prob = (synth.heat1d_random(n=n, N=N, steps=steps) if d == 1
            else synth.small_problem(d, n, N, R=1, steps=steps))
    assert np.allclose(euler.seq_euler_modal(prob), euler.seq_euler(prob), rtol=1e-11, atol=1e-12)


def test_modal_route_closed_form_and_factors():
    """A single sine mode with F = 0 decays by prod (1 + tau kappa(t_m) lambda_k)^{-1};
    a separable Gaussian source given as factors equals the assembled one."""
    n, N = 31, 10
    prob = synth.heat2d_gaussians(n=n, N=N, seed=9, phase=0.4)
    kf, tc, factors, u0 = synth.heat2d_parts(n=n, N=N, seed=9, phase=0.4)
    assert np.allclose(euler.seq_euler_modal(prob, factors=factors), euler.seq_euler(prob),
                       rtol=1e-11, atol=1e-12)
    mode = _sine(n, 2, [3, 2])
    q = synth.Problem(2, n, N, 1.0, kf, tc, np.zeros((N, n, n)), mode)
    lam = fd.laplace_eigenvalue([3, 2], q.h)
    fac = np.cumprod(1.0 / (1.0 + q.tau * tc[0] * lam))
    assert np.allclose(euler.seq_euler_modal(q), fac[:, None, None] * mode, rtol=1e-12, atol=1e-14)
    with pytest.raises(ValueError):
        euler.seq_euler_modal(synth.small_problem(2, 7, 3, R=2))


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
