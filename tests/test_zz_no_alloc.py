"""The allocation-free GMRES entry point (stp_gmres_solve_noalloc) against
stp_gmres_solve: two calls in a row on one GPU, the second with a smaller
problem, give the same iterates, step counts and residual histories; the
call allocates no device memory; a problem whose Krylov space exceeds the
fixed array is rejected."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU test collected without a GPU")
    import paper_1802_08126_amd as stp
    stp.load()
    yield


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def _compare(prob, restart):
    import paper_1802_08126_amd as stp
    from paper_1802_08126_amd import binding as b
    max_iter = 300
    s = stp.from_problem(prob, omega=0.7, tol=1e-9, max_iter=max_iter)
    shape = (prob.N,) + (prob.n,) * prob.dim
    u1 = torch.zeros(shape, dtype=torch.float64, device="cuda")
    p1 = torch.zeros_like(u1)
    nb = stp.stp_gmres_workspace_bytes(s.ctx, restart)
    ws = torch.empty((nb + 7) // 8, dtype=torch.float64, device="cuda")
    st1, i1, h1 = b.stp_gmres_solve(s.ctx, u1, p1, restart, ws, max_iter)
    u2 = torch.zeros_like(u1)
    p2 = torch.zeros_like(u1)
    torch.cuda.synchronize()
    before = stp.stp_device_bytes_allocated()
    st2, i2, h2 = b.stp_gmres_solve_noalloc(s.ctx, u2, p2, restart, max_iter)
    torch.cuda.synchronize()
    assert stp.stp_device_bytes_allocated() == before
    assert st1 == st2 == stp.STP_OK, (st1, st2)
    assert i1.iters == i2.iters and i1.rel_res == i2.rel_res
    assert h1 == h2
    assert np.array_equal(host(u1), host(u2)) and np.array_equal(host(p1), host(p2))
    s.close()
    return i2.iters


def test_noalloc_gmres_equals_gmres_on_two_calls():
    big = synth.small_problem(2, 31, 32, seed=71)       # 30,752 DoFs per variable
    small = synth.small_problem(2, 15, 16, seed=72)     # the second call is smaller
    assert _compare(big, 6) > 0
    assert _compare(small, 4) > 0


def test_noalloc_gmres_3d_and_float32():
    import paper_1802_08126_amd as stp
    from paper_1802_08126_amd import binding as b
    prob = synth.small_problem(3, 15, 8, seed=73)
    s = stp.from_problem(prob, precision="f32", omega=0.7, tol=1e-9, max_iter=200)
    shape = (prob.N,) + (prob.n,) * 3
    u1, p1 = torch.zeros(shape, dtype=torch.float64, device="cuda"), torch.zeros(shape, dtype=torch.float64,
                                                                                  device="cuda")
    ws = torch.empty((stp.stp_gmres_workspace_bytes(s.ctx, 5) + 7) // 8, dtype=torch.float64, device="cuda")
    st1, i1, _ = b.stp_gmres_solve(s.ctx, u1, p1, 5, ws)
    u2, p2 = torch.zeros_like(u1), torch.zeros_like(u1)
    st2, i2, _ = b.stp_gmres_solve_noalloc(s.ctx, u2, p2, 5)
    assert st1 == st2 == stp.STP_OK and i1.iters == i2.iters
    assert np.array_equal(host(u1), host(u2)) and np.array_equal(host(p1), host(p2))
    s.close()


def test_noalloc_rejects_a_krylov_space_beyond_the_fixed_array():
    import paper_1802_08126_amd as stp
    from paper_1802_08126_amd import binding as b
    prob = synth.small_problem(2, 127, 64, seed=74)     # 1.03e6 DoFs per variable: > 64 MiB for GMRES(5)
    s = stp.from_problem(prob, omega=0.7, tol=1e-9, max_iter=10)
    assert stp.stp_gmres_workspace_bytes(s.ctx, 5) > 64 << 20
    u = torch.zeros((prob.N, prob.n, prob.n), dtype=torch.float64, device="cuda")
    p = torch.zeros_like(u)
    st, _, _ = b.stp_gmres_solve_noalloc(s.ctx, u, p, 5)
    assert st == stp.STP_EINVAL
    assert b"fixed scratch" in stp.load().stp_last_error()
    assert not host(u).any()
    s.close()
