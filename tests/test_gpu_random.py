"""GPU parity of randomised Algorithm 3 (active sets of blocks and SARA
bases drawn per iteration) against the FP64
oracle fed the same draws."""
import numpy as np
import pytest

import synth
from oracle import ppd as O
from oracle import problem as oprob
from oracle import sara as osara

from gpu_util import announce, assert_op_close, dev, host, rel_err, require_gpu

pytestmark = pytest.mark.gpu


def _problem(seed=51, n=64, M=8000, d=4):
    x, wu, wv, off = synth.small_case(n, M, seed=seed, d=d)
    pb = oprob.make_problem(x, wu, wv, off, synth.noise_unit(M, 200 + seed), 30.0, np.ones((n, n)),
                            power_tol=1e-8)
    return pb, wu, wv


@pytest.mark.parametrize("graph,prox,tile,n_itr", [(False, "fb", 0, 2), (True, "fb", 0, 2), (False, "exact", 0, 2),
                                                   (True, "fb", 8, 2), (False, "exact", 8, 2),
                                                   (False, "fb", 8, 4), (True, "fb", 8, 4)])
def test_randomised_iterations_match_oracle(graph, prox, tile, n_itr):
    """With n_itr = 4 the middle Algorithm 2 steps run in the persistent
    launch, whose inactive blocks keep their z through every step."""
    P = require_gpu()
    import torch
    announce(f"randomised iterations graph={graph} prox={prox} tile={tile} n_itr={n_itr}")
    pb, wu, wv = _problem()
    n, d = pb.x_true.shape[0], len(pb.eps)
    T = 8
    bm, pm = synth.active_sets(T, d, 0.5, 0.6, seed=61)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        plan = P.Plan(n, n, wu, wv, pb.block_off, stream=stream, tile=tile)
        perm = plan.permutation()
        y = dev(pb.y[perm].astype(np.complex64), torch.complex64)
        U = dev(pb.U[perm], torch.float64)
        st = P.PPDState(plan, y)
        if n_itr > 2:
            assert plan.info.persistent == 1
        kw = dict(eta=pb.eta, mu=1.0, n_itr=n_itr, use_graph=graph)
        if prox == "exact":
            kw.update(prox=P.PROX_EXACT, n_newton=16)
        P.randomised_ppd(plan, st, y, U, pb.eps, bm, pm, **kw)
        stream.synchronize()
    ost = O.init_state(n, n, pb.y)
    O.iterate(pb.op, pb.y, pb.U, pb.eps, pb.block_off, O.Params(eta=pb.eta, mu=1.0, n_itr=n_itr, prox=prox), ost, T,
              active=list(zip(bm, pm)))
    assert_op_close(host(st.x), ost.x, what="x")
    assert_op_close(host(st.v), ost.v[perm], what="v")
    assert_op_close(host(st.z), ost.z[perm], what="z")
    u_scale = np.abs(osara.analysis(ost.xt)).max()
    assert np.abs(host(st.u) - ost.u).max() <= 1e-5 * u_scale
    # blocks / bases never drawn keep their initial values exactly
    for j in np.flatnonzero(bm.sum(0) == 0):
        s = slice(pb.block_off[j], pb.block_off[j + 1])
        assert np.abs(host(st.v)[np.isin(perm, np.arange(s.start, s.stop))]).max() == 0.0
    for i in np.flatnonzero(pm.sum(0) == 0):
        assert np.abs(host(st.u)[i]).max() == 0.0


def test_block_masks_need_fused_form():
    P = require_gpu()
    import torch
    announce("randomised plain form rejected")
    pb, wu, wv = _problem(seed=52)
    n, d = pb.x_true.shape[0], len(pb.eps)
    plan = P.Plan(n, n, wu, wv, pb.block_off)
    perm = plan.permutation()
    y = dev(pb.y[perm].astype(np.complex64), torch.complex64)
    U = dev(pb.U[perm], torch.float64)
    st = P.PPDState(plan, y)
    with pytest.raises(P.PPDError):
        P.ppd_iterate(plan, st, y, U, pb.eps, 1, eta=pb.eta, form=P.FORM_PLAIN,
                      block_active=dev(np.ones(d, np.uint8), torch.uint8))
