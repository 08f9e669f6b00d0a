"""GPU parity: the HIP library (through its C ABI) against the CPU oracle."""
import numpy as np
import pytest

import synth
from oracle import euler, spacetime as st, uzawa
from oracle.precond import Preconditioners

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU test collected without a GPU")
    import paper_1802_08126_amd as stp
    stp.load()
    yield


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def relmax(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def solver(prob, **kw):
    import paper_1802_08126_amd as stp
    return stp.from_problem(prob, **kw)


CASES = [(1, 63, 64), (1, 10, 7), (2, 15, 16), (2, 31, 9), (2, 10, 5), (3, 7, 8), (3, 15, 4), (2, 1, 3), (3, 1, 1), (1, 5, 1)]


@pytest.mark.parametrize("d,n,N", CASES)
def test_apply_operator(d, n, N):
    import paper_1802_08126_amd as stp
    prob = synth.small_problem(d, n, N, seed=d * 100 + n)
    s = solver(prob, spatial="none")
    rng = np.random.default_rng(1)
    x = rng.standard_normal((N,) + (n,) * d)
    y = rng.standard_normal((N,) + (n,) * d)
    got = host(s.apply_operator(stp.STP_OP_B, dev(x)))
    assert relmax(got, st.apply_B(prob, x)) < 1e-13
    xy = np.stack([x, y])
    got2 = host(s.apply_operator(stp.STP_OP_SADDLE, dev(xy)))
    top, bot = st.apply_saddle(prob, x, y)
    assert relmax(got2[0], top) < 1e-13
    assert relmax(got2[1], bot) < 1e-13
    s.close()


@pytest.mark.parametrize("d,n,N", [(1, 63, 64), (1, 31, 8), (2, 15, 16), (2, 63, 8), (3, 7, 8), (3, 15, 4), (2, 1, 3),
                                   (2, 7, 256), (1, 15, 128), (2, 3, 2), (1, 7, 32), (2, 7, 512), (1, 7, 100)])
@pytest.mark.parametrize("which", ["A", "H"])
def test_apply_precond_f64(d, n, N, which):
    import paper_1802_08126_amd as stp
    prob = synth.small_problem(d, n, N, seed=7 + d)
    spatial = "mg"
    s = solver(prob, spatial=spatial)
    pc = Preconditioners(prob, spatial=spatial)
    rng = np.random.default_rng(2)
    r = rng.standard_normal((N,) + (n,) * d)
    if which == "A":
        got = host(s.apply_precond(stp.STP_PC_A, dev(r)))
        ref = pc.Ainv(r)
    else:
        got = host(s.apply_precond(stp.STP_PC_H, dev(r)))
        ref = pc.Hinv(r)
    assert relmax(got, ref) < 1e-12
    s.close()


@pytest.mark.parametrize("which", ["A", "H"])
def test_apply_precond_exact_1d(which):
    import paper_1802_08126_amd as stp
    prob = synth.heat1d_random()
    s = solver(prob, spatial="exact")
    pc = Preconditioners(prob, spatial="exact")
    r = np.random.default_rng(3).standard_normal((prob.N, prob.n))
    if which == "A":
        got, ref = host(s.apply_precond(stp.STP_PC_A, dev(r))), pc.Ainv(r)
    else:
        got, ref = host(s.apply_precond(stp.STP_PC_H, dev(r))), pc.Hinv(r)
    assert relmax(got, ref) < 1e-12
    s.close()


@pytest.mark.parametrize("d,n,N,spatial,iters", [(1, 63, 64, "exact", 5), (2, 15, 16, "mg", 4), (3, 7, 8, "mg", 3),
                                                 (2, 31, 12, "mg", 6)])
def test_uzawa_trajectory(d, n, N, spatial, iters):
    """Fixed number of iterations (no stop test): u_j and p_{j+1} equal the oracle's."""
    prob = synth.heat1d_random(n=n, N=N) if d == 1 else synth.small_problem(d, n, N, seed=11)
    s = solver(prob, spatial=spatial, omega=0.7, tol=0.0, max_iter=iters, check_every=2)
    u, p, info = s.solve()
    ref = uzawa.uzawa_fixed(prob, iters, omega=0.7, spatial=spatial)
    assert info["iters"] == iters
    assert relmax(host(u), ref["u"]) < 1e-11
    assert relmax(host(p), ref["p"]) < 1e-11
    assert abs(info["rel_res"] - ref["history"][-1]) <= 1e-9 * ref["history"][-1]
    s.close()


@pytest.mark.parametrize("d,n,N,spatial", [(1, 63, 64, "exact"), (2, 31, 32, "mg"), (3, 15, 16, "mg"),
                                           (2, 63, 40, "mg")])
def test_solution_matches_sequential_euler(d, n, N, spatial):
    prob = synth.heat1d_random(n=n, N=N) if d == 1 else synth.small_problem(d, n, N, seed=13)
    s = solver(prob, spatial=spatial, omega=0.7, tol=1e-10, max_iter=400)
    u, p, info = s.solve()
    assert info["status"] == 0, info
    ue = euler.seq_euler(prob)
    uh = host(u)
    assert np.linalg.norm(uh - ue) / np.linalg.norm(ue) < 1e-8
    assert relmax(uh, ue) < 1e-8
    ref = uzawa.uzawa(prob, omega=0.7, tol=1e-10, spatial=spatial, max_iter=400)
    assert abs(info["iters"] - ref["iters"]) <= 1
    s.close()


@pytest.mark.parametrize("prec", ["f32", "bf16"])
@pytest.mark.parametrize("d,n,N", [(2, 31, 32), (3, 15, 16)])
def test_mixed_precision_accuracy(prec, d, n, N):
    """Preconditioner in float32 / bfloat16 storage, outer iteration in float64:
    the solution still matches the float64 oracle to 1e-8 relative."""
    prob = synth.small_problem(d, n, N, seed=17)
    s = solver(prob, precision=prec, omega=0.7, tol=1e-10, max_iter=600)
    u, p, info = s.solve()
    assert info["status"] == 0, info
    ue = euler.seq_euler(prob)
    uh = host(u)
    assert np.linalg.norm(uh - ue) / np.linalg.norm(ue) < 1e-8
    assert relmax(uh, ue) < 1e-8
    s.close()


def test_error_paths():
    import paper_1802_08126_amd as stp
    prob = synth.small_problem(2, 15, 4)
    kf, F, u0 = dev(prob.kfields), dev(prob.F), dev(prob.u0)
    with pytest.raises(stp.StpError) as e:
        stp.SpaceTimeSolver(2, 15, 4, -1.0, kf, prob.tcoef, F, u0)
    assert e.value.status == stp.STP_EINVAL
    bad = prob.kfields.copy()
    bad[1] = -5.0        # kappa = 1 + amp sin(.) * (-5) becomes negative
    with pytest.raises(stp.StpError) as e:
        stp.SpaceTimeSolver(2, 15, 4, prob.tau, dev(bad), prob.tcoef, F, u0)
    assert e.value.status == stp.STP_EINVAL
    p10 = synth.small_problem(2, 10, 4)
    with pytest.raises(stp.StpError) as e:
        stp.from_problem(p10, spatial="mg")
    assert e.value.status == stp.STP_EUNSUPPORTED
    s = stp.from_problem(prob, max_iter=1, tol=1e-12)
    _, _, info = s.solve()
    assert info["status"] == stp.STP_ENOTCONV and info["iters"] == 1
    s.close()
    s = stp.from_problem(prob, omega=3.0, tol=1e-12, max_iter=300)
    u, _, info = s.solve()
    assert info["status"] == stp.STP_EDIVERGED
    s.close()


def test_graph_replay_matches_eager():
    """An iteration captured as a HIP graph gives bitwise the same iterates as
    eager launches, over several replays, repeated solves with eager work in
    between, and a re-capture for new buffers."""
    prob = synth.small_problem(2, 31, 16, seed=23)
    eager = solver(prob, omega=0.7, tol=0.0, max_iter=5, use_graph=False, check_every=2)
    ue, pe, ie = eager.solve()
    ue, pe = host(ue), host(pe)
    g = solver(prob, omega=0.7, tol=0.0, max_iter=5, use_graph=True, check_every=2)
    u = torch.zeros((16, 31, 31), dtype=torch.float64, device="cuda")
    p = torch.zeros_like(u)
    for rep in range(3):
        u.zero_()
        p.zero_()
        _, _, ig = g.solve(u, p)
        torch.cuda.synchronize()
        _ = (u * 2.0).sum().item()          # unrelated eager work between replays
        assert ig["iters"] == ie["iters"] == 5
        assert np.array_equal(host(u), ue) and np.array_equal(host(p), pe), rep
    u2, p2, _ = g.solve()                   # new buffers: the iteration is captured again
    assert np.array_equal(host(u2), ue) and np.array_equal(host(p2), pe)
    eager.close()
    g.close()


@pytest.mark.parametrize("N", [3, 7, 17, 33, 63, 100, 127, 255, 500, 1000, 1019, 2047])
@pytest.mark.parametrize("d,n", [(1, 7), (2, 3)])
def test_apply_precond_H_any_N(d, n, N):
    """H~^{-1} at step counts that are not powers of two: the time transforms
    run as Bluestein convolutions (N > 16) or dense sums (N <= 16)."""
    import paper_1802_08126_amd as stp
    prob = synth.small_problem(d, n, N, seed=N)
    s = solver(prob, spatial="mg")
    pc = Preconditioners(prob, spatial="mg")
    r = np.random.default_rng(N).standard_normal((N,) + (n,) * d)
    got = host(s.apply_precond(stp.STP_PC_H, dev(r)))
    assert relmax(got, pc.Hinv(r)) < 1e-11
    s.close()
    s = solver(prob, spatial="mg", precision="f32")
    got = host(s.apply_precond(stp.STP_PC_H, dev(r)))
    assert relmax(got, pc.Hinv(r)) < 2e-5
    s.close()


@pytest.mark.parametrize("N", [4096, 8192, 16384, 65536, 131072])
@pytest.mark.parametrize("d,n", [(1, 7), (2, 3)])
def test_apply_precond_H_large_N(d, n, N):
    """H~^{-1} at large power-of-two step counts: the time transforms run as
    four-step FFTs (N = N1 N2 with a complex scratch pass; N = 2^17 has
    N1 = 2 N2; in float64 also N = 4096, whose single-pass LDS FFT does not fit)."""
    import paper_1802_08126_amd as stp
    prob = synth.small_problem(d, n, N, seed=N % 1000)
    print(f"case d={d} n={n} N={N}", flush=True)
    s = solver(prob, spatial="mg")
    assert "fourstep" in s.schedule()
    pc = Preconditioners(prob, spatial="mg")
    r = np.random.default_rng(N).standard_normal((N,) + (n,) * d)
    want = pc.Hinv(r)
    got = host(s.apply_precond(stp.STP_PC_H, dev(r)))
    assert relmax(got, want) < 1e-11
    s.close()
    s = solver(prob, spatial="mg", precision="f32")
    got = host(s.apply_precond(stp.STP_PC_H, dev(r)))
    assert relmax(got, want) < 5e-5
    s.close()


def test_uzawa_iterations_large_N():
    """Three Uzawa iterations at N = 16384 (four-step transforms inside the
    captured iteration) against the oracle."""
    prob = synth.small_problem(2, 3, 16384, seed=5)
    s = solver(prob, omega=0.7, tol=0.0, max_iter=3)
    u, p, info = s.solve()
    ref = uzawa.uzawa_fixed(prob, 3, omega=0.7, spatial="mg")
    assert relmax(host(u), ref["u"]) < 1e-11 and relmax(host(p), ref["p"]) < 1e-11
    s.close()
