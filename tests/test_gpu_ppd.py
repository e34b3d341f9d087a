"""GPU parity of Algorithm 3 (ppd_iterate) against the FP64 oracle."""
import numpy as np
import pytest

import synth
from oracle import ppd as O
from oracle import problem as oprob
from oracle import prox as oprox
from oracle import sara as osara

from gpu_util import announce, assert_op_close, dev, host, rel_err, require_gpu

pytestmark = pytest.mark.gpu


def _small_problem(seed=11, n=64, M=6000, d=3):
    x, wu, wv, off = synth.small_case(n, M, seed=seed, d=d)
    noise = synth.noise_unit(M, 200 + seed)
    pb = oprob.make_problem(x, wu, wv, off, noise, 30.0, np.ones((n, n)), power_tol=1e-8)
    return pb, wu, wv


def _gpu_inputs(P, plan, pb):
    import torch
    perm = plan.permutation()
    y = dev(pb.y[perm].astype(np.complex64), torch.complex64)
    U = dev(pb.U[perm], torch.float64)
    return perm, y, U


@pytest.mark.parametrize("tile", [0, 8])
@pytest.mark.parametrize("form", ["fused", "plain"])
@pytest.mark.parametrize("n_itr", [1, 3])
def test_iterations_match_oracle(form, n_itr, tile):
    P = require_gpu()
    import torch
    announce(f"ppd iterate small form={form} n_itr={n_itr} tile={tile}")
    pb, wu, wv = _small_problem()
    n = pb.x_true.shape[0]
    plan = P.Plan(n, n, wu, wv, pb.block_off, chunk=300, tile=tile)
    perm, y, U = _gpu_inputs(P, plan, pb)
    st = P.PPDState(plan, y)
    prm = O.Params(eta=pb.eta, mu=1.0, n_itr=n_itr)
    ost = O.init_state(n, n, pb.y)
    f = P.FORM_FUSED if form == "fused" else P.FORM_PLAIN
    for T in (1, 4):
        O.iterate(pb.op, pb.y, pb.U, pb.eps, pb.block_off, prm, ost, T)
        s = P.ppd_iterate(plan, st, y, U, pb.eps, T, eta=pb.eta, mu=1.0, n_itr=n_itr, form=f)
        assert s["iter"] == ost.it
        assert_op_close(host(st.x), ost.x, what=f"x after {ost.it}")
        assert_op_close(host(st.xt), ost.xt, what=f"x tilde after {ost.it}")
        assert_op_close(host(st.v), ost.v[perm], what=f"v after {ost.it}")
        assert_op_close(host(st.z), ost.z[perm], what=f"z after {ost.it}")
        # u is clipped to [-alpha, alpha]; its error is that of the clip
        # argument u + Psi^H x~, whose scale is the coefficient magnitude
        u_scale = np.abs(osara.analysis(ost.xt)).max()
        du = np.abs(host(st.u) - ost.u).max()
        assert du <= 1e-5 * u_scale, f"u after {ost.it}: {du:.3e} vs scale {u_scale:.3e}"


def test_first_iteration_closed_form_gpu():
    P = require_gpu()
    announce("first iteration closed form")
    pb, wu, wv = _small_problem(seed=12)
    n = pb.x_true.shape[0]
    plan = P.Plan(n, n, wu, wv, pb.block_off)
    perm, y, U = _gpu_inputs(P, plan, pb)
    st = P.PPDState(plan, y)
    P.ppd_iterate(plan, st, y, U, pb.eps, 1, eta=pb.eta, mu=1.0)
    z = np.empty_like(pb.y)
    for j in range(len(pb.eps)):
        s = slice(pb.block_off[j], pb.block_off[j + 1])
        z[s] = oprox.proj_B((1 - pb.U[s]) * pb.y[s], pb.y[s], pb.eps[j])
    x1 = np.maximum(0.49 * pb.eta * pb.op.phit(pb.U * z), 0.0)
    assert_op_close(host(st.x), x1, what="x1")
    assert_op_close(host(st.xt), 2 * x1, what="x tilde 1")
    assert np.abs(host(st.u)).max() == 0.0


def test_graph_replay_matches_eager():
    """A replayed graph runs the same kernels with the same fixed summation
    orders as eager launches (only the stream each branch runs on differs):
    the iterates agree bit for bit, replay after replay, with eager work in
    between."""
    P = require_gpu()
    import torch
    announce("graph replay vs eager")
    pb, wu, wv = _small_problem(seed=13)
    n = pb.x_true.shape[0]
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        plan = P.Plan(n, n, wu, wv, pb.block_off, stream=stream)
        perm, y, U = _gpu_inputs(P, plan, pb)
        a = P.PPDState(plan, y)
        b = P.PPDState(plan, y)
        for rep in range(3):   # replays with eager work in between
            P.ppd_iterate(plan, a, y, U, pb.eps, 5, eta=pb.eta, use_graph=False)
            P.ppd_iterate(plan, b, y, U, pb.eps, 5, eta=pb.eta, use_graph=True)
            stream.synchronize()
            for k in ("x", "xt", "v", "u", "z"):
                assert np.array_equal(host(getattr(b, k)), host(getattr(a, k))), (rep, k)


def test_workload64_snr_parity():
    """200 PPD and PD iterations on the 64x64 workload: SNR within 0.05 dB."""
    P = require_gpu()
    import torch
    w = synth.WORKLOADS["ppd64"]
    inp = synth.make_inputs(w)
    pb = oprob.problem_from_inputs(inp, power_tol=1e-9)
    plan = P.Plan(64, 64, inp.wu[0], inp.wv[0], inp.block_off)
    perm, y, U = _gpu_inputs(P, plan, pb)
    xt = dev(pb.x_true.astype(np.float32), torch.float32)
    for name, Uo, eta in [("ppd", pb.U, pb.eta), ("pd", np.ones_like(pb.U), pb.eta_pd)]:
        announce(f"workload64 {name} 200 iterations")
        ost = O.init_state(64, 64, pb.y)
        h = O.iterate(pb.op, pb.y, Uo, pb.eps, pb.block_off, O.Params(eta=eta, mu=1.0 / Uo.max()), ost, 200,
                      x_true=pb.x_true)
        st = P.PPDState(plan, y)
        Ud = U if name == "ppd" else dev(np.ones(pb.U.size), torch.float64)
        snr = []
        for k in range(20):
            s = P.ppd_iterate(plan, st, y, Ud, pb.eps, 10, eta=eta, mu=1.0, x_true=xt)
            snr.append(s["snr_db"])
            assert abs(s["snr_db"] - h[10 * k + 9]["snr"]) < 0.05, (name, k, s["snr_db"], h[10 * k + 9]["snr"])
        assert rel_err(host(st.x), ost.x) < 1e-3


@pytest.mark.parametrize("tile", [0, 8])
def test_many_blocks_per_tile(tile):
    """100 blocks spread over the whole u-v plane (each tile holds points of
    every block): work items are cut at 64 segments, and both the operators
    and the iteration still match the oracle."""
    P = require_gpu()
    import torch
    from oracle import nufft as onf
    announce(f"100 interleaved blocks tile={tile}")
    n, M, d = 32, 20000, 100
    x, wu, wv, _ = synth.small_case(n, M, seed=14, coverage="uniform")
    off = np.linspace(0, M, d + 1).astype(np.int64)
    pb = oprob.make_problem(x, wu, wv, off, synth.noise_unit(M, 214), 30.0, np.ones((n, n)), power_tol=1e-8)
    plan = P.Plan(n, n, wu, wv, off, tile=tile)
    info = plan.info
    assert info.n_chunks > (2 * n // info.tile) ** 2          # tiles split by the segment cap
    perm, y, U = _gpu_inputs(P, plan, pb)
    yg = P.ppd_phi(plan, dev(x.astype(np.float32), torch.float32))
    assert_op_close(host(yg), pb.op.phi(x.astype(np.float32).astype(np.float64))[perm], what="phi")
    st = P.PPDState(plan, y)
    ost = O.init_state(n, n, pb.y)
    prm = O.Params(eta=pb.eta, mu=1.0, n_itr=2)
    O.iterate(pb.op, pb.y, pb.U, pb.eps, pb.block_off, prm, ost, 3)
    P.ppd_iterate(plan, st, y, U, pb.eps, 3, eta=pb.eta, mu=1.0, n_itr=2)
    assert_op_close(host(st.x), ost.x, what="x")
    assert_op_close(host(st.z), ost.z[perm], what="z")


def test_per_kernel_timing_counts():
    """The per-launch event timer sees every launch of eager iterations (both
    streams) with the expected counts per kind, and none inside a captured
    graph (only the call's first row pass runs outside it)."""
    P = require_gpu()
    import torch
    announce("per-kernel timing")
    pb, wu, wv = _small_problem()
    n = pb.x_true.shape[0]
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        plan = P.Plan(n, n, wu, wv, pb.block_off, stream=stream)
        perm, y, U = _gpu_inputs(P, plan, pb)
        st = P.PPDState(plan, y)
        plan.timing(True)
        plan.timing_reset()
        P.ppd_iterate(plan, st, y, U, pb.eps, 3, eta=pb.eta, mu=1.0, stats=False)
        t = plan.timing_read()
        per_iter = {"fft_cols_fwd": 1, "degrid": 1, "grid": 1, "fold": 1, "fft_cols_inv": 1, "fft_rows_inv": 1,
                    "dwt": 3, "idwt": 2}   # levels 3: two coarsest synthesis levels in one launch + last
        for k, c in per_iter.items():
            assert t[k][0] == 3 * c, (k, t[k])
            assert t[k][1] > 0.0, (k, t[k])
        assert t["fft_rows_fwd"][0] == 1   # the first iteration's row pass; later ones are fused
        plan.timing_reset()
        P.ppd_iterate(plan, st, y, U, pb.eps, 3, eta=pb.eta, mu=1.0, stats=False, use_graph=True)
        t = plan.timing_read()
        plan.timing(False)
        stream.synchronize()
    assert t.get("fft_rows_fwd", (0, 0.0))[0] == 1
    assert all(t.get(k, (0, 0.0))[0] == 0 for k in per_iter), t


@pytest.mark.parametrize("graph", [False, True])
def test_periodic_statistics_history(graph):
    """stats_every = 2 over 6 iterations leaves on the device, row by row,
    the statistics that separate calls of 2 iterations report (same
    reductions, bit for bit), eagerly and replayed from a graph."""
    P = require_gpu()
    import torch
    announce(f"periodic statistics graph={graph}")
    pb, wu, wv = _small_problem()
    n = pb.x_true.shape[0]
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        plan = P.Plan(n, n, wu, wv, pb.block_off, stream=stream)
        perm, y, U = _gpu_inputs(P, plan, pb)
        xt = dev(pb.x_true.astype(np.float32), torch.float32)
        ref = []
        st = P.PPDState(plan, y)
        for _ in range(3):
            s = P.ppd_iterate(plan, st, y, U, pb.eps, 2, eta=pb.eta, x_true=xt, use_graph=graph)
            ref.append([s["rel_change"], s["x_norm"], s["snr_db"], s["residual_max"]] + list(s["residual"]))
        hist = torch.zeros(3 * (8 + plan.d), dtype=torch.float64, device="cuda")
        st2 = P.PPDState(plan, y)
        s2 = P.ppd_iterate(plan, st2, y, U, pb.eps, 6, eta=pb.eta, x_true=xt, use_graph=graph,
                           stats_every=2, stats_history=hist)
        stream.synchronize()
    h = host(hist).reshape(3, 8 + plan.d)
    got = np.concatenate([h[:, :4], h[:, 8:]], axis=1)
    assert np.array_equal(got, np.array(ref)), (got, np.array(ref))
    assert s2["iter"] == 6 and s2["rel_change"] == ref[-1][0]
    assert np.array_equal(host(st2.x), host(st.x))


@pytest.mark.parametrize("n_iter,every,n_itr", [(37, 10, 1), (21, 0, 1), (30, 25, 1), (25, 10, 4)])
def test_replayed_schedules_match_eager(n_iter, every, n_itr):
    """Calls whose replay mixes captured statistics periods, runs of 8
    iterations without statistics and single iterations (37 iterations with
    statistics every 10, 21 without periodic statistics, 30 with statistics
    every 25, and 25 with the persistent Algorithm 2 launch of n_itr = 4):
    the iterates and the statistics history agree bit for bit with eager
    launches."""
    P = require_gpu()
    import torch
    announce(f"replayed schedule n_iter={n_iter} every={every} n_itr={n_itr}")
    pb, wu, wv = _small_problem(seed=17)
    n = pb.x_true.shape[0]
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        plan = P.Plan(n, n, wu, wv, pb.block_off, stream=stream)
        assert n_itr == 1 or plan.info.persistent == 1
        perm, y, U = _gpu_inputs(P, plan, pb)
        xt = dev(pb.x_true.astype(np.float32), torch.float32)
        rows = max(1, n_iter // every) if every else 1
        out = {}
        for graph in (False, True):
            st = P.PPDState(plan, y)
            hist = torch.zeros(rows * (8 + plan.d), dtype=torch.float64, device="cuda")
            kw = dict(stats_every=every, stats_history=hist) if every else {}
            s = P.ppd_iterate(plan, st, y, U, pb.eps, n_iter, eta=pb.eta, x_true=xt, use_graph=graph,
                              n_itr=n_itr, **kw)
            stream.synchronize()
            out[graph] = (s, {k: host(getattr(st, k)) for k in ("x", "xt", "v", "u", "z")}, host(hist))
    (se, ae, he), (sg, ag, hg) = out[False], out[True]
    for k in ae:
        assert np.array_equal(ag[k], ae[k]), k
    assert np.array_equal(hg, he)
    assert sg["iter"] == se["iter"] == n_iter and sg["rel_change"] == se["rel_change"]
