"""GPU parity with several V-cycles per spatial preconditioner application
(nu_A, nu_H > 1; Section 8.2 uses one or two): A~^{-1} and H~^{-1}, Uzawa and
GMRES iterates, the damping estimate and a batch against the oracle, whose
cycles each act on the residual the earlier ones leave."""
import numpy as np
import pytest

import synth
from oracle import krylov, uzawa
from oracle import omega as om
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


def make(d, n, N, R, seed=31):
    return synth.heat1d_random(n=n, N=N, seed=seed) if d == 1 else synth.small_problem(d, n, N, seed=seed, R=R)


# (d, n, N, R): tiled levels with per-slab and rank-1 coefficients, 3-D, a
# hierarchy solved entirely by the fused coarse kernel, a 1-D hierarchy
PC_CASES = [(2, 31, 12, 2), (2, 63, 8, 1), (3, 15, 6, 2), (2, 7, 40, 3), (1, 127, 16, 1)]


@pytest.mark.parametrize("nu", [2, 3])
@pytest.mark.parametrize("d,n,N,R", PC_CASES)
def test_apply_precond_nu(d, n, N, R, nu):
    import paper_1802_08126_amd as stp
    prob = make(d, n, N, R)
    print(f"case d={d} n={n} N={N} R={R} nu={nu}", flush=True)
    pc = Preconditioners(prob, spatial="mg", nu_A=nu, nu_H=nu)
    r = np.random.default_rng(nu).standard_normal((N,) + (n,) * d)
    wantA, wantH = pc.Ainv(r), pc.Hinv(r)
    # float32 storage: the residual b - L x between cycles cancels and keeps
    # about eps32 * cond(L) relative accuracy (1-D, n = 127: cond near 6.6e3)
    for prec, tol in (("f64", 1e-12), ("f32", 1e-4)):
        s = stp.from_problem(prob, spatial="mg", precision=prec, nu_A=nu, nu_H=nu)
        assert relmax(host(s.apply_precond(stp.STP_PC_A, dev(r))), wantA) < tol, prec
        assert relmax(host(s.apply_precond(stp.STP_PC_H, dev(r))), wantH) < tol, prec
        s.close()


@pytest.mark.parametrize("nu_A,nu_H", [(2, 2), (1, 3), (3, 1)])
@pytest.mark.parametrize("d,n,N,R", [(2, 31, 16, 2), (3, 15, 8, 1)])
def test_uzawa_trajectory_nu(d, n, N, R, nu_A, nu_H):
    import paper_1802_08126_amd as stp
    prob = make(d, n, N, R, seed=32)
    print(f"case d={d} n={n} N={N} R={R} nu=({nu_A},{nu_H})", flush=True)
    s = stp.from_problem(prob, spatial="mg", omega=0.8, tol=0.0, max_iter=5, nu_A=nu_A, nu_H=nu_H)
    u, p, info = s.solve()
    ref = uzawa.uzawa_fixed(prob, 5, omega=0.8, spatial="mg", nu_A=nu_A, nu_H=nu_H)
    assert info["iters"] == 5
    assert relmax(host(u), ref["u"]) < 1e-11 and relmax(host(p), ref["p"]) < 1e-11
    s.close()


def test_gmres_and_omega_estimate_nu2():
    import paper_1802_08126_amd as stp
    prob = make(2, 31, 16, 2, seed=33)
    pc = Preconditioners(prob, spatial="mg", nu_A=2, nu_H=2)
    s = stp.from_problem(prob, spatial="mg", omega=0.0, tol=0.0, max_iter=6, nu_A=2, nu_H=2)
    g = s.omega_info()
    ref = om.auto_omega(prob, spatial="mg", pc=pc)
    for k in ("lmin", "lmax", "omega"):
        assert abs(g[k] - ref[k]) < 1e-9 * abs(ref[k]), k
    assert abs(g["rho_A"] - ref["rho_A"]) < 1e-9 * ref["rho_A"]
    u, p, info = s.gmres(restart=4)
    want = krylov.gmres(prob, omega=g["omega"], tol=0.0, restart=4, max_iter=6, pc=pc)
    assert relmax(host(u), want["u"]) < 1e-10 and relmax(host(p), want["p"]) < 1e-10
    s.close()


def test_batch_nu2_and_graph_replay():
    """A batch with two cycles per application gives each problem's oracle
    iterates; a captured iteration replays bitwise like eager launches."""
    import paper_1802_08126_amd as stp
    probs = [make(2, 31, 12, 2, seed=34), make(2, 15, 20, 1, seed=35), make(2, 63, 6, 3, seed=36)]
    b = stp.BatchSolver([stp.problem_dict(q) for q in probs], omega=0.7, tol=0.0, max_iter=4, nu_A=2, nu_H=2)
    us, ps, infos, _ = b.solve()
    for q, u, p in zip(probs, us, ps):
        ref = uzawa.uzawa_fixed(q, 4, omega=0.7, spatial="mg", nu_A=2, nu_H=2)
        assert relmax(host(u), ref["u"]) < 1e-11 and relmax(host(p), ref["p"]) < 1e-11
    b.close()
    q = probs[0]
    e = stp.from_problem(q, omega=0.7, tol=0.0, max_iter=4, nu_A=2, nu_H=2, use_graph=False)
    g = stp.from_problem(q, omega=0.7, tol=0.0, max_iter=4, nu_A=2, nu_H=2, use_graph=True)
    ue, pe, _ = e.solve()
    for _ in range(2):
        ug, pg, _ = g.solve()
        assert np.array_equal(host(ug), host(ue)) and np.array_equal(host(pg), host(pe))
    e.close()
    g.close()


def test_nu_out_of_range():
    import paper_1802_08126_amd as stp
    prob = make(2, 15, 4, 1)
    for bad in ((0, 1), (1, 9)):
        with pytest.raises(stp.StpError) as ex:
            stp.from_problem(prob, nu_A=bad[0], nu_H=bad[1])
        assert ex.value.status == stp.STP_EINVAL


@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_mixed_precision_nu2_reaches_euler(prec):
    """Two cycles per application with float32 / bfloat16 storage: the
    float64 outer iteration still reaches the sequential implicit Euler
    solution to 1e-8 relative."""
    import paper_1802_08126_amd as stp
    from oracle import euler
    prob = make(3, 15, 16, 2, seed=37)
    s = stp.from_problem(prob, precision=prec, omega=0.0, tol=1e-10, max_iter=600, nu_A=2, nu_H=2)
    u, _, info = s.solve()
    assert info["status"] == stp.STP_OK, info
    ue = euler.seq_euler(prob)
    assert relmax(host(u), ue) < 1e-8
    s.close()


def test_nu2_with_graded_steps():
    """Non-uniform steps (per-slab tau_n in the A~ cycles and in the steps
    between them): Uzawa iterates against the oracle."""
    import paper_1802_08126_amd as stp
    steps = synth.graded_steps(12, 1.0, ratio=4.0, jitter=0.3, seed=38)
    prob = synth.small_problem(2, 31, 12, seed=38, R=2, steps=steps)
    s = stp.from_problem(prob, omega=0.6, tol=0.0, max_iter=4, nu_A=2, nu_H=3)
    u, p, _ = s.solve()
    ref = uzawa.uzawa_fixed(prob, 4, omega=0.6, spatial="mg", nu_A=2, nu_H=3)
    assert relmax(host(u), ref["u"]) < 1e-11 and relmax(host(p), ref["p"]) < 1e-11
    s.close()


def test_autotuned_schedule_with_nu2():
    """The autotuner rebuilds every launch table, the steps between cycles
    included: the tuned context still gives the oracle's iterates."""
    import paper_1802_08126_amd as stp
    prob = make(2, 63, 16, 2, seed=39)
    s = stp.from_problem(prob, omega=0.7, tol=0.0, max_iter=4, nu_A=2, nu_H=2)
    s.autotune(reps=1, use_cache=False)
    u, p, _ = s.solve()
    ref = uzawa.uzawa_fixed(prob, 4, omega=0.7, spatial="mg", nu_A=2, nu_H=2)
    assert relmax(host(u), ref["u"]) < 1e-11 and relmax(host(p), ref["p"]) < 1e-11
    s.close()


def test_exact_solves_ignore_nu():
    """Exact 1-D spatial solves need one application: nu > 1 gives bitwise the
    iterates of nu = 1 (no extra buffer, no extra launches)."""
    import paper_1802_08126_amd as stp
    prob = synth.heat1d_random(n=63, N=32, seed=40)
    a = stp.from_problem(prob, spatial="exact", omega=0.7, tol=0.0, max_iter=3)
    b = stp.from_problem(prob, spatial="exact", omega=0.7, tol=0.0, max_iter=3, nu_A=3, nu_H=2)
    ua, pa, _ = a.solve()
    ub, pb, _ = b.solve()
    assert np.array_equal(host(ua), host(ub)) and np.array_equal(host(pa), host(pb))
    a.close()
    b.close()
