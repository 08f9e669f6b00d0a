"""GPU parity with non-uniform time steps tau_n (Section 2; the tau_steps
option): Uzawa and GMRES iterates against the oracle, convergence to the
sequential implicit Euler solution, batches of problems with their own
steps, and argument checks."""
import numpy as np
import pytest

import synth
from oracle import euler, krylov, uzawa
from oracle import omega as om

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


def relmax(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def graded(d, n, N, R=2, ratio=8.0, seed=81):
    steps = synth.graded_steps(N, 1.0, ratio=ratio, jitter=0.3, seed=seed)
    if d == 1:
        return synth.heat1d_random(n=n, N=N, seed=seed, steps=steps)
    return synth.small_problem(d, n, N, seed=seed, R=R, steps=steps)


CASES = [(2, 15, 16, 2, "mg", "f64"), (2, 31, 12, 1, "mg", "f64"), (3, 7, 8, 2, "mg", "f64"),
         (1, 63, 32, 1, "exact", "f64"), (2, 15, 40, 3, "mg", "f64"), (2, 15, 16, 2, "mg", "f32")]


@pytest.mark.parametrize("d,n,N,R,spatial,prec", CASES)
def test_uzawa_graded_steps_match_oracle(d, n, N, R, spatial, prec):
    import paper_1802_08126_amd as stp
    prob = graded(d, n, N, R)
    print(f"case d={d} n={n} N={N} R={R} {prec}", flush=True)
    s = stp.from_problem(prob, spatial=spatial, precision=prec, omega=0.6, tol=0.0, max_iter=4)
    u, p, info = s.solve()
    ref = uzawa.uzawa_fixed(prob, 4, omega=0.6, spatial=spatial)
    tol = 1e-11 if prec == "f64" else 2e-5
    assert info["iters"] == 4
    assert relmax(host(u), ref["u"]) < tol and relmax(host(p), ref["p"]) < tol
    s.close()


@pytest.mark.parametrize("d,n,N,R,spatial", [(2, 15, 16, 2, "mg"), (1, 63, 32, 1, "exact")])
def test_gmres_graded_steps_match_oracle(d, n, N, R, spatial):
    import paper_1802_08126_amd as stp
    prob = graded(d, n, N, R, seed=82)
    s = stp.from_problem(prob, spatial=spatial, omega=0.7, tol=0.0, max_iter=6)
    u, p, info = s.gmres(restart=4)
    ref = krylov.gmres(prob, omega=0.7, tol=0.0, restart=4, max_iter=6, spatial=spatial)
    assert relmax(host(u), ref["u"]) < 1e-10 and relmax(host(p), ref["p"]) < 1e-10
    assert np.abs(np.array(info["history"]) - ref["history"]).max() < 1e-10 * ref["history"][0]
    s.close()


def test_graded_steps_converge_to_sequential_euler():
    """Both solvers with the estimated omega reach the implicit Euler solution
    of the graded steps (relative error 1e-8 at residual 1e-10)."""
    import paper_1802_08126_amd as stp
    prob = graded(2, 31, 32, 2, ratio=4.0, seed=83)
    ref = euler.seq_euler(prob)
    s = stp.from_problem(prob, omega=0.0, tol=1e-10, max_iter=1000)
    g = s.omega_info()
    o = om.auto_omega(prob)
    assert abs(g["omega"] - o["omega"]) < 1e-9 * o["omega"]
    u, p, info = s.solve()
    assert info["status"] == stp.STP_OK
    assert relmax(host(u), ref) < 1e-8
    u2, p2, gi = s.gmres(restart=10)
    assert gi["status"] == stp.STP_OK and gi["iters"] < info["iters"]
    assert relmax(host(u2), ref) < 1e-8
    s.close()


def test_reference_step_defaults_to_mean_and_checks():
    import paper_1802_08126_amd as stp
    prob = graded(2, 15, 8, 2, seed=84)
    a = stp.from_problem(prob, omega=0.6, tol=0.0, max_iter=3)
    ua, pa, _ = a.solve()
    kf = torch.as_tensor(prob.kfields, dtype=torch.float64, device="cuda")
    F = torch.as_tensor(prob.F, dtype=torch.float64, device="cuda")
    u0 = torch.as_tensor(prob.u0, dtype=torch.float64, device="cuda")
    b = stp.SpaceTimeSolver(2, 15, 8, 0.0, kf, prob.tcoef, F, u0, omega=0.6, tol=0.0, max_iter=3,
                            tau_steps=list(prob.steps))
    ub, pb, _ = b.solve()
    # the mean of the steps equals T/N up to the rounding of their sum
    assert relmax(host(ub), host(ua)) < 1e-13 and relmax(host(pb), host(pa)) < 1e-13
    a.close()
    b.close()
    bad = list(prob.steps)
    bad[3] = 0.0
    with pytest.raises(stp.StpError):
        stp.SpaceTimeSolver(2, 15, 8, 0.0, kf, prob.tcoef, F, u0, tau_steps=bad)
    with pytest.raises(ValueError):      # a batch takes the steps of every problem
        stp.BatchSolver([stp.problem_dict(prob), stp.problem_dict(prob)], tau_steps=list(prob.steps))


def test_batch_with_per_problem_steps():
    """A batch whose problems have their own step lengths (one of them
    uniform): each problem's iterates equal its single-problem context's
    bitwise and the oracle's; a bad step of a later problem is rejected."""
    import paper_1802_08126_amd as stp
    probs = [graded(2, 15, 16, 2, seed=85), synth.small_problem(2, 31, 8, seed=86, R=1),
             graded(2, 31, 12, 3, ratio=4.0, seed=87)]
    b = stp.BatchSolver([stp.problem_dict(q) for q in probs], omega=0.6, tol=0.0, max_iter=4)
    us, ps, infos, _ = b.solve()
    for k, (q, u, p) in enumerate(zip(probs, us, ps)):
        print(f"case batch problem {k}", flush=True)
        s = stp.from_problem(q, omega=0.6, tol=0.0, max_iter=4)
        u1, p1, _ = s.solve()
        assert np.array_equal(host(u), host(u1)) and np.array_equal(host(p), host(p1))
        s.close()
        ref = uzawa.uzawa_fixed(q, 4, omega=0.6, spatial="mg")
        assert relmax(host(u), ref["u"]) < 1e-11 and relmax(host(p), ref["p"]) < 1e-11
    b.close()
    bad = [stp.problem_dict(q) for q in probs]
    bad[2]["steps"][5] = -1.0
    with pytest.raises(stp.StpError) as e:
        stp.BatchSolver(bad)
    assert e.value.status == stp.STP_EINVAL
