"""GPU parity of the register-pencil multigrid sweeps: 3-D multigrid levels
whose coarse side is at least 24 run their restriction (down) and
prolongation-and-smoothing (up) sweeps as register pencils (rank-1
coefficients for both operator families, the H-blocks for any rank); the
up-sweep's three epilogues (store, add into the output of a later nu > 1
cycle, add into the float64 iterate) all occur.

The cases are ragged in every direction the kernel tiles: 63^3 has 31 coarse
nodes per axis (two x-pencils of 16 and 15, a last y-pencil of 3 rows and a
last z-pencil of 15 planes) and 127^3 has 63 (three x-pencils of 21); step
counts of 3 and 5 leave idle waves in the last four-slab block.  Rank-2
coefficients put the A family on the LDS tiles and the H family on pencils in
the same V-cycle schedule.  References are the oracle's preconditioners and
Uzawa iterates; a batch must reproduce its problems' standalone results bit for
bit, so the per-problem launch split keeps a problem's arithmetic independent
of the batch it is in."""
import numpy as np
import pytest

import synth
from oracle import uzawa
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


# float32 preconditioner against the float64 oracle: a V-cycle is a few tens of
# roundings per node and level at 6e-8 each, so 2e-5 of the largest entry;
# bfloat16 storage rounds every stored vector to 2^-9 relative, so a few of
# those per level: 3e-2 (an indexing mistake gives errors of order one)
TOL = {"f64": 1e-12, "f32": 2e-5, "bf16": 3e-2}


@pytest.mark.parametrize("n,N,R", [(63, 4, 1), (63, 5, 2), (63, 3, 1), (127, 2, 1)])
@pytest.mark.parametrize("which", ["A", "H"])
@pytest.mark.parametrize("prec", ["f64", "f32", "bf16"])
def test_pencil_precond_matches_oracle(n, N, R, which, prec):
    import paper_1802_08126_amd as stp
    print(f"pencil precond n={n} N={N} R={R} {which} {prec}", flush=True)
    prob = synth.small_problem(3, n, N, seed=40 + n + N + R, R=R)
    s = stp.from_problem(prob, spatial="mg", precision=prec)
    pc = Preconditioners(prob, spatial="mg")
    r = np.random.default_rng(3).standard_normal((N,) + (n,) * 3)
    if which == "A":
        got, ref = host(s.apply_precond(stp.STP_PC_A, dev(r))), pc.Ainv(r)
    else:
        got, ref = host(s.apply_precond(stp.STP_PC_H, dev(r))), pc.Hinv(r)
    assert np.isfinite(got).all()
    assert relmax(got, ref) < TOL[prec], relmax(got, ref)
    s.close()


@pytest.mark.parametrize("n,N", [(63, 5), (31, 3), (127, 2)])
def test_pencil_uzawa_iterates_match_oracle(n, N):
    """Rank 1: both operator families on pencils (63^3: level 0; 127^3: levels
    0 and 1; 31^3 stays on the LDS tiles); the iterates and the stop test's
    residual match the oracle's."""
    import paper_1802_08126_amd as stp
    prob = synth.small_problem(3, n, N, seed=91 + n, R=1)
    iters = 3
    s = stp.from_problem(prob, omega=0.7, tol=0.0, max_iter=iters)
    u, p, info = s.solve()
    assert info["iters"] == iters
    ref = uzawa.uzawa_fixed(prob, iters, omega=0.7, spatial="mg")
    assert relmax(host(u), ref["u"]) < 1e-11
    assert relmax(host(p), ref["p"]) < 1e-11
    # the residual of the last evaluated iterate: ||f - B u_3|| / ||f||
    assert abs(info["rel_res"] - ref["history"][iters]) <= 1e-10 * ref["history"][iters]
    s.close()


def test_pencil_batch_equals_standalone():
    """A batch mixing pencil levels (63^3) with tiled ones (15^3, and the A
    family of a rank-2 coefficient) gives each problem its standalone iterate."""
    import paper_1802_08126_amd as stp
    probs = [synth.small_problem(3, 63, 4, seed=92, R=1), synth.small_problem(3, 15, 8, seed=93, R=1),
             synth.small_problem(3, 63, 6, seed=94, R=2)]
    kw = dict(omega=0.7, tol=0.0, max_iter=2, check_every=2)
    b = stp.BatchSolver([stp.problem_dict(q) for q in probs], **kw)
    us, ps, infos, _ = b.solve()
    for i, q in enumerate(probs):
        s = stp.from_problem(q, **kw)
        u1, p1, _ = s.solve()
        assert np.array_equal(host(us[i]), host(u1)), i
        assert np.array_equal(host(ps[i]), host(p1)), i
        s.close()
    b.close()


@pytest.mark.parametrize("nu_A,nu_H", [(2, 2), (1, 3)])
def test_pencil_nu_cycles_match_oracle(nu_A, nu_H):
    """nu > 1 cycles: stores into the cycle buffer, the tiled operator in
    between, and the last H cycle adding into its output."""
    import paper_1802_08126_amd as stp
    prob = synth.small_problem(3, 63, 4, seed=95, R=1)
    s = stp.from_problem(prob, spatial="mg", nu_A=nu_A, nu_H=nu_H)
    pc = Preconditioners(prob, spatial="mg", nu_A=nu_A, nu_H=nu_H)
    r = np.random.default_rng(5).standard_normal((prob.N,) + (63,) * 3)
    assert relmax(host(s.apply_precond(stp.STP_PC_A, dev(r))), pc.Ainv(r)) < 1e-12
    assert relmax(host(s.apply_precond(stp.STP_PC_H, dev(r))), pc.Hinv(r)) < 1e-12
    s.close()
