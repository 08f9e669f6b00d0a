"""The benchmark's exact solutions (plain torch, used to report the error of
every GPU result) against the oracle, on the CPU."""
import numpy as np
import pytest
import torch

import bench
import synth
from oracle import euler, fd


@pytest.mark.parametrize("d,n", [(1, 9), (2, 7), (3, 5)])
def test_fd_apply_torch_equals_oracle_operator(d, n):
    rng = np.random.default_rng(d)
    kap = rng.uniform(0.2, 3.0, size=(n + 2,) * d)
    v = rng.standard_normal((n,) * d)
    got = bench.fd_apply_torch(torch.as_tensor(kap), torch.as_tensor(v), 1.0 / (n + 1)).numpy()
    assert np.allclose(got, fd.apply(kap, v, 1.0 / (n + 1), d), rtol=1e-13, atol=1e-12)


def test_manufactured_source_has_the_closed_form_solution():
    """The oracle's sequential implicit Euler on the manufactured 3-D problem
    returns exp(-3 pi^2 t_n) sin sin sin."""
    inp = bench.manufactured_3d(7, 5, 1003, 1e2, "cpu")
    prob = inp["prob"]
    prob.F = inp["F"].numpy()
    ue = euler.seq_euler(prob)
    exact = np.multiply.outer(inp["e"][1:], inp["S"].numpy())
    assert np.allclose(ue, exact, rtol=1e-11, atol=1e-13)
    err = bench.manufactured_error(torch.as_tensor(ue), inp["S"], inp["e"])
    assert err["rel_l2"] < 1e-11 and err["rel_max"] < 1e-11


def test_modal_error_against_oracle_modal_route():
    spec = dict(side=15, N=23, phase=1.1, seed=4003)
    q = synth.batch2d_problem(spec)
    kf, tc, factors, u0 = synth.batch2d_parts(spec)
    ue = euler.seq_euler(q)
    e0 = bench.modal_error(q.n, q.N, q.tau, tc[0] * kf[0, 0, 0], u0, factors, torch.as_tensor(ue))
    assert e0["rel_l2"] < 1e-12 and e0["rel_max"] < 1e-12
    bad = ue.copy()
    bad[7] *= 1 + 1e-6
    e1 = bench.modal_error(q.n, q.N, q.tau, tc[0] * kf[0, 0, 0], u0, factors, torch.as_tensor(bad))
    assert 1e-8 < e1["rel_l2"] < 1e-6 and e1["rel_max"] == pytest.approx(1e-6 * np.abs(ue[7]).max()
                                                                         / np.abs(ue).max(), rel=1e-3)


def test_algorithmic_bytes_of_the_headline_down_sweep():
    """Level-0 down-sweep of 255^3 x 64 in float32: fine b read, coarse b
    written, the field read once."""
    dims = bench.level_dims(3, 255, 64, 1)
    assert dims["npts"][:3] == [255 ** 3, 127 ** 3, 63 ** 3]
    b = bench.algorithmic_bytes("k_mg_down", 0, dims, 4)
    assert b == 64 * (255 ** 3 + 127 ** 3) * 4 + 257 ** 3 * 4
