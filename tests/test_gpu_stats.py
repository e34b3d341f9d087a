"""The FP64 statistics of Algorithm 3 on the GPU against the oracle's
per-iteration records: the relative change ||x_t - x_{t-1}|| / ||x_t|| and
the data-fidelity residuals r_j = ||Phi_j x~ - y_j|| that make up the
stopping test ("until convergence", Algorithm 3) and the constraint of the
constrained problem (Sec. 3), ||x_t||, max_j r_j / eps_j, and the SNR of
Sec. 5.  Both sides define r_j at the x~ an iteration starts from.

Tolerances follow from the parity bar of the iterates and operator outputs
(1e-5 relative, float32 against float64):
* ||x_t||: 1e-5 relative;
* rel_change: |d| <= 3e-5 + 1e-5 rel (each of x_t, x_{t-1} within 1e-5 of
  ||x_t||, so their difference within 2e-5 ||x_t||);
* r_j: |d| <= 1e-5 (||y_j|| + r_j) (Phi_j x~ within 1e-5 of its own norm,
  which is at most ||y_j|| + r_j);
* SNR: 0.05 dB.
"""
import numpy as np
import pytest

import synth
from oracle import ppd as O
from oracle import problem as oprob

from gpu_util import announce, check_stats, dev, host, require_gpu

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("graph", [False, True])
@pytest.mark.parametrize("case", ["ppd64", "tracks256"])
def test_statistics_match_oracle_records(case, graph):
    """30 iterations with the statistics of every iteration reduced on the
    device into a history, each row against the oracle's record."""
    P = require_gpu()
    import torch
    inp = synth.make_inputs(synth.WORKLOADS[case])
    n_itr = synth.WORKLOADS[case].n_itr
    announce(f"statistics vs oracle records {case} n_itr={n_itr} graph={graph}")
    w = inp.workload
    pb = oprob.problem_from_inputs(inp, with_eta=False)
    # any step size serves, as long as both sides use the same one
    eta = 1.0 / oprob.power_norm(pb.op, pb.U, inp.power_start, tol=1e-4, max_iter=30)
    T = 30
    ost = O.init_state(w.n, w.n, pb.y)
    recs = O.iterate(pb.op, pb.y, pb.U, pb.eps, pb.block_off, O.Params(eta=eta, mu=1.0, n_itr=n_itr), ost, T,
                     x_true=pb.x_true)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        plan = P.Plan(w.n, w.n, inp.wu[0], inp.wv[0], inp.block_off, stream=stream)
        perm = plan.permutation()
        y = dev(pb.y[perm].astype(np.complex64), torch.complex64)
        U = dev(pb.U[perm], torch.float64)
        xt = dev(pb.x_true.astype(np.float32), torch.float32)
        st = P.PPDState(plan, y)
        hist = torch.zeros(T * (8 + plan.d), dtype=torch.float64, device="cuda")
        s = P.ppd_iterate(plan, st, y, U, pb.eps, T, eta=eta, mu=1.0, n_itr=n_itr, x_true=xt, use_graph=graph,
                          stats_every=1, stats_history=hist)
        stream.synchronize()
    rows = host(hist).reshape(T, 8 + plan.d)
    check_stats(rows, recs, pb.y, pb.block_off, pb.eps, f"{case} graph={graph}")
    # the call's own statistics are the last row's
    assert s["rel_change"] == rows[-1, 0] and s["x_norm"] == rows[-1, 1]
    assert np.array_equal(s["residual"], rows[-1, 8:])


def test_relative_change_of_an_all_zero_iterate_is_zero():
    """With y = 0 every iterate stays 0 (the prox of a ball that holds its
    argument is the argument, so v stays 0 and P_C returns 0): the relative
    change of 0 over ||x|| = 0 is 0, the oracle's convention, not NaN."""
    P = require_gpu()
    import torch
    announce("rel_change of an all-zero iterate")
    x, wu, wv, off = synth.small_case(32, 2000, seed=21)
    eps = np.array([1.0])
    ost = O.init_state(32, 32, np.zeros(2000, np.complex128))
    op = oprob.Nufft(wu, wv, 32, 32)
    recs = O.iterate(op, np.zeros(2000, np.complex128), np.ones(2000), eps, off, O.Params(eta=1e-3), ost, 2)
    assert recs[-1]["rel_change"] == 0.0 and recs[-1]["x_norm"] == 0.0
    plan = P.Plan(32, 32, wu, wv, off)
    y = torch.zeros(2000, dtype=torch.complex64, device="cuda")
    U = dev(np.ones(2000), torch.float64)
    st = P.PPDState(plan, y)
    s = P.ppd_iterate(plan, st, y, U, eps, 2, eta=1e-3)
    assert float(host(st.x).max()) == 0.0
    assert s["rel_change"] == 0.0 and s["x_norm"] == 0.0 and s["residual_max"] == 0.0
