"""The persistent form of Algorithm 2's middle steps (n_itr > 1, fused
form): one launch runs the n_itr - 1 middle forward-backward steps of every
block with the per-point state in registers; each step waits (bounded) for
the partial norms of its own blocks only.

* At the benchmark's size (512^2, 1.3M points, 16 blocks, n_itr = 5) its
  iterations match the FP64 oracle element by element, eagerly and replayed
  from a graph.
* It agrees with the launch-pair form (PPD_PERSIST_OFF) on tracks256: the
  same arithmetic with the block norms summed in another order.
* A wait that runs out (forced from the host with a spin limit of one poll)
  releases every workgroup, the kernel ends normally, the call reports
  PPD_EDEVICE, and the next call runs normally.
* Small uneven blocks: workgroups spanning 4 blocks (the most one may
  span) match the oracle; a plan with 3072 consecutive points over 5
  blocks reports no persistent launch and runs launch pairs, which match
  the oracle too.
"""
import math

import numpy as np
import pytest

import synth
from oracle import ppd as O
from oracle import problem as oprob
from oracle import sara as osara

from gpu_util import announce, assert_op_close, dev, host, rel_err, require_gpu

pytestmark = pytest.mark.gpu


def test_persistent_nitr5_matches_oracle_at_ppd512():
    P = require_gpu()
    import torch
    announce("persistent Algorithm 2, ppd512, n_itr=5, eager then graph")
    inp = synth.make_inputs(synth.WORKLOADS["ppd512"])
    n = inp.workload.n
    pb = oprob.problem_from_inputs(inp, with_eta=False)
    eta = 1.0 / oprob.power_norm(pb.op, pb.U, inp.power_start, tol=1e-3, max_iter=10)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        plan = P.Plan(n, n, inp.wu[0], inp.wv[0], inp.block_off, stream=stream)
        assert plan.info.persistent == 1
        perm = plan.permutation()
        y = dev(pb.y[perm].astype(np.complex64), torch.complex64)
        U = dev(pb.U[perm], torch.float64)
        st = P.PPDState(plan, y)
        ost = O.init_state(n, n, pb.y)
        prm = O.Params(eta=eta, mu=1.0, n_itr=5)
        for graph in (False, True):
            O.iterate(pb.op, pb.y, pb.U, pb.eps, pb.block_off, prm, ost, 2)
            s = P.ppd_iterate(plan, st, y, U, pb.eps, 2, eta=eta, mu=1.0, n_itr=5, use_graph=graph)
            stream.synchronize()
            assert s["iter"] == ost.it
            mode = "graph" if graph else "eager"
            assert_op_close(host(st.x), ost.x, what=f"x after {ost.it} ({mode})")
            assert_op_close(host(st.xt), ost.xt, what=f"x tilde after {ost.it} ({mode})")
            assert_op_close(host(st.v), ost.v[perm], what=f"v after {ost.it} ({mode})")
            assert_op_close(host(st.z), ost.z[perm], what=f"z after {ost.it} ({mode})")
            u_scale = np.abs(osara.analysis(ost.xt)).max()
            assert np.abs(host(st.u) - ost.u).max() <= 1e-5 * u_scale


def test_persistent_agrees_with_launch_pairs():
    P = require_gpu()
    import torch
    announce("persistent vs launch pairs, tracks256, n_itr=5")
    inp = synth.make_inputs(synth.WORKLOADS["tracks256"])
    w = inp.workload
    pb = oprob.problem_from_inputs(inp, with_eta=False)
    eta = 1.0 / oprob.power_norm(pb.op, pb.U, inp.power_start, tol=1e-3, max_iter=20)
    plan = P.Plan(w.n, w.n, inp.wu[0], inp.wv[0], inp.block_off)
    assert plan.info.persistent == 1
    perm = plan.permutation()
    y = dev(pb.y[perm].astype(np.complex64), torch.complex64)
    U = dev(pb.U[perm], torch.float64)
    states = {}
    for mode in (P.PERSIST_AUTO, P.PERSIST_OFF):
        st = P.PPDState(plan, y)
        P.ppd_iterate(plan, st, y, U, pb.eps, 20, eta=eta, n_itr=5, persistent=mode)
        states[mode] = st
    a, b = states[P.PERSIST_AUTO], states[P.PERSIST_OFF]
    for k in ("x", "xt", "v", "u"):
        e = rel_err(host(getattr(a, k)), host(getattr(b, k)))
        assert e < 1e-6, (k, e)
    assert rel_err(host(a.z), host(b.z)) < 1e-10


def test_wait_give_up_is_reported_and_recovers():
    P = require_gpu()
    import torch
    announce("persistent wait give-up (spin limit 1) and recovery")
    inp = synth.make_inputs(synth.WORKLOADS["ppd512"])
    w = inp.workload
    n = w.n
    plan = P.Plan(n, n, inp.wu[0], inp.wv[0], inp.block_off)
    assert plan.info.persistent == 1
    perm = plan.permutation()
    U = P.ppd_uniform_weights(plan)
    xt = dev(inp.x_true.astype(np.float32), torch.float32)
    y0 = P.ppd_phi(plan, xt)
    sigma = math.sqrt(float((y0.abs().double() ** 2).sum()) / w.M * 10.0 ** (-w.isnr_db / 10.0))
    y = (y0 + sigma * dev(inp.noise[0][perm].astype(np.complex64), torch.complex64)).contiguous()
    Mj = np.diff(inp.block_off).astype(np.float64)
    eps = sigma * np.sqrt(Mj + 2.0 * np.sqrt(Mj))
    norm2, _ = P.ppd_op_norm(plan, U, dev(inp.power_start.astype(np.float32), torch.float32), 50, 1e-3)
    eta = 1.0 / norm2
    st = P.PPDState(plan, y)
    with pytest.raises(P.PPDError) as err:
        P.ppd_iterate(plan, st, y, U, eps, 1, eta=eta, n_itr=3, spin_limit=1)
    assert err.value.status == P.PPD_EDEVICE and "gave up" in str(err.value)
    # the flag is cleared and the slots were emptied by the last workgroup out
    a, b = P.PPDState(plan, y), P.PPDState(plan, y)
    P.ppd_iterate(plan, a, y, U, eps, 3, eta=eta, n_itr=3)
    P.ppd_iterate(plan, b, y, U, eps, 3, eta=eta, n_itr=3, persistent=P.PERSIST_OFF)
    assert rel_err(host(a.x), host(b.x)) < 1e-6


@pytest.mark.parametrize("M,d,seed,persistent", [(10000, 8, 73, 1), (16000, 12, 74, 0)])
def test_blocks_per_workgroup_edges(M, d, seed, persistent):
    P = require_gpu()
    import torch
    announce(f"persistent edges M={M} d={d} seed={seed}")
    n = 64
    x, wu, wv, off = synth.small_case(n, M, seed=seed, d=d)
    # blocks spanned by each run of 3072 consecutive points (blocks are contiguous in plan order)
    spans = [int(np.sum((off[:-1] < min((g + 1) * 3072, M)) & (off[1:] > g * 3072)))
             for g in range((M + 3071) // 3072)]
    assert max(spans) == (4 if persistent else 5)
    pb = oprob.make_problem(x, wu, wv, off, synth.noise_unit(M, 400 + seed), 30.0, np.ones((n, n)),
                            power_tol=1e-8)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        plan = P.Plan(n, n, wu, wv, off, stream=stream)
        assert plan.info.persistent == persistent
        perm = plan.permutation()
        y = dev(pb.y[perm].astype(np.complex64), torch.complex64)
        U = dev(pb.U[perm], torch.float64)
        st = P.PPDState(plan, y)
        ost = O.init_state(n, n, pb.y)
        prm = O.Params(eta=pb.eta, mu=1.0, n_itr=5)
        for graph in (False, True):
            O.iterate(pb.op, pb.y, pb.U, pb.eps, pb.block_off, prm, ost, 3)
            P.ppd_iterate(plan, st, y, U, pb.eps, 3, eta=pb.eta, mu=1.0, n_itr=5, use_graph=graph)
            stream.synchronize()
            mode = "graph" if graph else "eager"
            assert_op_close(host(st.x), ost.x, what=f"x ({mode})")
            assert_op_close(host(st.v), ost.v[perm], what=f"v ({mode})")
            assert_op_close(host(st.z), ost.z[perm], what=f"z ({mode})")
