"""GPU parity of batched contexts: many independent problems served by merged
launches.  Each problem of a batch must give exactly what its own
single-problem context gives (same kernels, same per-problem arithmetic and
reduction order), and that must match the oracle."""
import numpy as np
import pytest

import synth
from oracle import euler, uzawa

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


def make(specs, dim):
    out = []
    for k, (n, N) in enumerate(specs):
        if dim == 1:
            out.append(synth.heat1d_random(n=n, N=N, seed=500 + k))
        else:
            out.append(synth.small_problem(dim, n, N, seed=600 + 7 * k, R=1 + k % 4))
    return out


def standalone(prob, **kw):
    import paper_1802_08126_amd as stp
    s = stp.from_problem(prob, **kw)
    u, p, info = s.solve()
    res = host(u), host(p), info
    s.close()
    return res


# sides with 1..5 multigrid levels, step counts on every time-transform path:
# register FFT (8, 16, 64), Stockham (512) and dense (12, 40, 100)
MIXED_2D = [(31, 16), (7, 12), (15, 8), (1, 3), (31, 40), (3, 64), (15, 100), (7, 512)]


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_batch_fixed_iterations_equal_standalone(prec):
    import paper_1802_08126_amd as stp
    probs = make(MIXED_2D, 2)
    iters = 4
    kw = dict(precision=prec, omega=0.7, tol=0.0, max_iter=iters, check_every=3)
    b = stp.BatchSolver([stp.problem_dict(q) for q in probs], **kw)
    assert len(b) == len(probs) and stp.stp_batch_size(b.ctx) == len(probs)
    us, ps, infos, status = b.solve()
    assert status == stp.STP_ENOTCONV
    for i, q in enumerate(probs):
        u1, p1, i1 = standalone(q, **kw)
        assert infos[i]["iters"] == i1["iters"] == iters, (i, infos[i], i1)
        assert np.array_equal(host(us[i]), u1), (i, q.n, q.N)
        assert np.array_equal(host(ps[i]), p1), (i, q.n, q.N)
        assert infos[i]["rel_res"] == i1["rel_res"]
        if prec == "f64":
            ref = uzawa.uzawa_fixed(q, iters, omega=0.7, spatial="mg")
            assert relmax(u1, ref["u"]) < 1e-11, (i, q.n, q.N)
            assert relmax(p1, ref["p"]) < 1e-11, (i, q.n, q.N)
    b.close()


def test_batch_stops_each_problem_on_its_own():
    """With a tolerance, problems stop at different iterations; later launches
    skip a stopped problem, so its iterate is exactly the standalone one."""
    import paper_1802_08126_amd as stp
    probs = make([(31, 32), (15, 8), (7, 100), (31, 12), (3, 4)], 2)
    kw = dict(omega=0.5, tol=1e-10, max_iter=400, check_every=4)   # inside every problem's range (3.7)
    b = stp.BatchSolver([stp.problem_dict(q) for q in probs], **kw)
    us, ps, infos, status = b.solve()
    assert status == stp.STP_OK, infos
    its = set()
    for i, q in enumerate(probs):
        u1, p1, i1 = standalone(q, **kw)
        assert infos[i]["status"] == stp.STP_OK
        assert infos[i]["iters"] == i1["iters"]
        its.add(i1["iters"])
        assert np.array_equal(host(us[i]), u1), i
        assert np.array_equal(host(ps[i]), p1), i
        ue = euler.seq_euler(q)
        assert np.linalg.norm(u1 - ue) / np.linalg.norm(ue) < 1e-8
    assert len(its) > 1      # the batch really mixes stopping times
    b.close()


def test_batch_1d_exact_and_3d():
    import paper_1802_08126_amd as stp
    p1 = make([(63, 64), (31, 7), (15, 16), (10, 33)], 1)
    kw = dict(omega=0.7, tol=0.0, max_iter=3, check_every=2)
    b = stp.BatchSolver([stp.problem_dict(q) for q in p1], spatial="exact", **kw)
    us, ps, infos, _ = b.solve()
    for i, q in enumerate(p1):
        u1, pp1, _ = standalone(q, spatial="exact", **kw)
        assert np.array_equal(host(us[i]), u1) and np.array_equal(host(ps[i]), pp1), i
        ref = uzawa.uzawa_fixed(q, 3, omega=0.7, spatial="exact")
        assert relmax(u1, ref["u"]) < 1e-11
    b.close()
    p3 = make([(15, 8), (7, 4), (3, 16)], 3)
    b = stp.BatchSolver([stp.problem_dict(q) for q in p3], **kw)
    us, ps, infos, _ = b.solve()
    for i, q in enumerate(p3):
        u1, pp1, _ = standalone(q, **kw)
        assert np.array_equal(host(us[i]), u1) and np.array_equal(host(ps[i]), pp1), i
    b.close()


def test_batch_graph_replay_and_rebinding():
    """Graph replay over a batch equals eager launches; a second solve with new
    buffers reuses the captured graph through the rebound job tables."""
    import paper_1802_08126_amd as stp
    probs = make([(15, 16), (31, 8), (7, 40)], 2)
    kw = dict(omega=0.7, tol=0.0, max_iter=5, check_every=2)
    e = stp.BatchSolver([stp.problem_dict(q) for q in probs], use_graph=False, **kw)
    ue, pe, _, _ = e.solve()
    g = stp.BatchSolver([stp.problem_dict(q) for q in probs], use_graph=True, **kw)
    for rep in range(3):
        ug, pg, _, _ = g.solve()            # fresh buffers every time
        _ = sum(float(x.sum()) for x in ug)  # eager work between replays
        for i in range(len(probs)):
            assert np.array_equal(host(ug[i]), host(ue[i])) and np.array_equal(host(pg[i]), host(pe[i])), (rep, i)
    e.close()
    g.close()


def test_batch_of_64_workload_sample():
    """The 64-problem mixed-size batch workload (sides capped to keep the test
    short): every problem matches its standalone solve after 3 iterations."""
    import paper_1802_08126_amd as stp
    specs = synth.batch2d(count=64, side_cap=31, nt_cap=64)
    probs = [synth.batch2d_problem(sp) for sp in specs]
    kw = dict(omega=0.7, tol=0.0, max_iter=3, check_every=4)
    b = stp.BatchSolver([stp.problem_dict(q) for q in probs], **kw)
    us, ps, infos, _ = b.solve()
    for i in range(0, 64, 9):
        u1, p1, _ = standalone(probs[i], **kw)
        assert np.array_equal(host(us[i]), u1) and np.array_equal(host(ps[i]), p1), i
    b.close()


def test_batch_errors():
    import paper_1802_08126_amd as stp
    a = synth.small_problem(2, 7, 4, seed=1)
    c = synth.small_problem(3, 7, 4, seed=2)
    with pytest.raises(stp.StpError) as e:
        stp.BatchSolver([stp.problem_dict(a), stp.problem_dict(c)])
    assert e.value.status == stp.STP_EUNSUPPORTED
    with pytest.raises(stp.StpError) as e:
        stp.BatchSolver([stp.problem_dict(a), stp.problem_dict(a)], kref_coef=[1.0, 0.0])
    assert e.value.status == stp.STP_EINVAL
    b = stp.BatchSolver([stp.problem_dict(a), stp.problem_dict(a)])
    x = torch.zeros((4, 7, 7), dtype=torch.float64, device="cuda")
    with pytest.raises(stp.StpError) as e:
        b_op = stp.stp_apply_operator(b.ctx, stp.STP_OP_B, x, x.clone())  # noqa: F841
    assert e.value.status == stp.STP_EUNSUPPORTED
    b.close()
