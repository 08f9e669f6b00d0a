"""The oracle on the robustness study of Section 8.2 (Table 2) in
finite-difference form: 2-D heat equation, T = 1, u(0) = sin(pi x) sin(pi y),
F = 0, omega = 0.9; the count is the first Uzawa iteration j with
||u - u_j||_S < 1e-6 ||u||_S (u: the sequential implicit Euler solution).
The paper prints 20-22 iterations for every h = 1/8 .. 1/64 and N = 128 .. 1024."""
import numpy as np
import pytest

import synth
from oracle import euler, krylov, spacetime as st
from oracle.precond import Preconditioners


def count(n, N, spatial, nu, kmax=45):
    prob = synth.heat2d_sine(n, N)
    ue = euler.seq_euler(prob)
    scale = st.s_norm(prob, ue)
    pc = Preconditioners(prob, spatial=spatial, nu_A=nu, nu_H=nu)
    xs = krylov.stationary(prob, pc, 0.9, kmax)
    errs = [st.s_norm(prob, ue - xs[k][1]) / scale for k in range(kmax + 1)]
    return next(k for k, e in enumerate(errs) if e < 1e-6)


@pytest.mark.parametrize("spatial,nu", [("exact", 1), ("mg", 2)])
def test_counts_in_the_printed_range_and_flat_in_N(spatial, nu):
    """Exact spatial solves, or two V-cycles of the multigrid cycle used here,
    need as many iterations as the paper prints, independent of N."""
    c = [count(7, N, spatial, nu) for N in (128, 256)]
    assert all(18 <= x <= 23 for x in c), c
    assert abs(c[0] - c[1]) <= 1, c


def test_one_vcycle_is_slower_but_flat_in_h():
    """One V(1,1) damped-Jacobi cycle (contraction about 0.31 on tau A) puts
    omega = 0.9 above the sufficient bound 2 (1 - rho_A) / ((1 + rho_A) lambda_max)
    of eq. (3.7) (about 0.53 with lambda_max near 2): the method still
    converges, more slowly, with the same count for h = 1/8 and 1/16."""
    c = [count(n, 128, "mg", 1) for n in (7, 15)]
    assert all(30 <= x <= 40 for x in c) and abs(c[0] - c[1]) <= 1, c
