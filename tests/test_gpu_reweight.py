"""GPU parity of the Algorithm 1 re-weighting (Sec. 3.2): weighted SARA
dual / synthesis, ppd_reweight, Algorithm 3 with weights and the outer
re-weighting loop, against the FP64 oracle."""
import numpy as np
import pytest

import synth
from oracle import ppd as O
from oracle import problem as oprob
from oracle import prox as oprox
from oracle import sara as osara

from gpu_util import announce, assert_op_close, dev, host, require_gpu

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n", [64, 256])
def test_weighted_sara_dual_and_synthesis(n):
    P = require_gpu()
    import torch
    announce(f"weighted sara n={n}")
    rng = np.random.default_rng(81 + n)
    x, wu, wv, off = synth.small_case(n, 64, seed=3, nx=n)
    plan = P.Plan(n, n, wu, wv, off)
    xt = rng.standard_normal((n, n)).astype(np.float32)
    W = rng.uniform(0.01, 1.0, (9, n, n)).astype(np.float32)
    u0 = (0.3 * rng.standard_normal((9, n, n))).astype(np.float32)
    alpha, lam = 0.25, 0.8
    coef = W.astype(np.float64) * osara.analysis(xt.astype(np.float64))
    ubar = oprox.clip_dual(u0 + coef, alpha)
    u1 = u0 + lam * (ubar - u0)
    Wd = dev(W, torch.float32)
    ud = dev(u0, torch.float32)
    rec = P.ppd_sara(plan, P.SARA_DUAL, dev(xt, torch.float32), u=ud, alpha=alpha, lam=lam, W=Wd)
    scale = np.abs(u0 + coef).max()
    assert np.abs(host(ud) - u1).max() <= 1e-5 * scale
    assert_op_close(host(rec), osara.synthesis(W * u1), what="weighted dual synthesis")
    out = P.ppd_sara(plan, P.SARA_SYNTHESIS, ud, W=Wd)
    assert_op_close(host(out), osara.synthesis(W * u1), what="weighted synthesis")


@pytest.mark.parametrize("omega", [1e-3, 0.1, 10.0])
def test_reweight_matches_oracle(omega):
    P = require_gpu()
    import torch
    announce(f"reweight omega={omega}")
    n = 128
    x, wu, wv, off = synth.small_case(n, 64, seed=4, nx=n)
    plan = P.Plan(n, n, wu, wv, off)
    x32 = x.astype(np.float32)
    Wg = host(P.ppd_reweight(plan, dev(x32, torch.float32), omega))
    Wo = O.reweights(x32.astype(np.float64), omega)
    # W = omega/(omega+|c|): dW = -W (1-W) dc/|c|, so an analysis error of
    # 1e-5 relative to max|c| moves W by at most 1e-5 max|c| / omega * W^2.
    cmax = np.abs(osara.analysis(x32.astype(np.float64))).max()
    bound = 1e-5 * cmax / omega * Wo ** 2 + 1e-7
    assert np.all(np.abs(Wg - Wo) <= bound), float(np.max(np.abs(Wg - Wo) - bound))
    assert Wg.max() <= 1.0 and Wg.min() > 0.0


def test_weighted_iterations_match_oracle():
    P = require_gpu()
    import torch
    announce("weighted ppd iterate")
    n, M = 64, 6000
    x, wu, wv, off = synth.small_case(n, M, seed=17, d=3)
    pb = oprob.make_problem(x, wu, wv, off, synth.noise_unit(M, 217), 30.0, np.ones((n, n)), power_tol=1e-8)
    W = O.reweights(x, 0.05).astype(np.float32)
    plan = P.Plan(n, n, wu, wv, pb.block_off)
    perm = plan.permutation()
    y = dev(pb.y[perm].astype(np.complex64), torch.complex64)
    U = dev(pb.U[perm], torch.float64)
    Wd = dev(W, torch.float32)
    for form in (P.FORM_FUSED, P.FORM_PLAIN):
        st = P.PPDState(plan, y)
        ost = O.init_state(n, n, pb.y)
        prm = O.Params(eta=pb.eta, mu=1.0, n_itr=2)
        for T in (1, 5):
            O.iterate(pb.op, pb.y, pb.U, pb.eps, pb.block_off, prm, ost, T, W=W.astype(np.float64))
            P.ppd_iterate(plan, st, y, U, pb.eps, T, eta=pb.eta, mu=1.0, n_itr=2, form=form, W=Wd)
            assert_op_close(host(st.x), ost.x, what=f"x after {ost.it} form {form}")
            assert_op_close(host(st.v), ost.v[perm], what=f"v after {ost.it} form {form}")
            u_scale = np.abs(W * osara.analysis(ost.xt)).max()
            du = np.abs(host(st.u) - ost.u).max()
            assert du <= 1e-5 * u_scale, f"u after {ost.it}: {du:.3e} vs scale {u_scale:.3e}"


def test_reweighted_loop_snr_parity():
    """Algorithm 1 on the 64x64 workload (2 re-weights, 150 iterations per
    solve): the GPU SNR at the end of every solve within 0.05 dB of the
    oracle's, and the re-weighted result above the unweighted one."""
    P = require_gpu()
    import torch
    announce("reweighted loop ppd64")
    w = synth.WORKLOADS["ppd64"]
    inp = synth.make_inputs(w)
    pb = oprob.problem_from_inputs(inp, power_tol=1e-9)
    ost = O.init_state(64, 64, pb.y)
    hists, _ = O.reweighted(pb.op, pb.y, pb.U, pb.eps, pb.block_off, O.Params(eta=pb.eta), ost, 2, 150,
                            x_true=pb.x_true)
    plan = P.Plan(64, 64, inp.wu[0], inp.wv[0], inp.block_off)
    perm = plan.permutation()
    y = dev(pb.y[perm].astype(np.complex64), torch.complex64)
    U = dev(pb.U[perm], torch.float64)
    xt = dev(pb.x_true.astype(np.float32), torch.float32)
    st = P.PPDState(plan, y)
    stats, W = P.reweighted_ppd(plan, st, y, U, pb.eps, 2, 150, x_true=xt, eta=pb.eta, mu=1.0)
    for k, (s, h) in enumerate(zip(stats, hists)):
        print(f"[reweight] solve {k}: GPU {s['snr_db']:.3f} dB oracle {h[-1]['snr']:.3f} dB", flush=True)
        assert abs(s["snr_db"] - h[-1]["snr"]) < 0.05, (k, s["snr_db"], h[-1]["snr"])
    assert stats[-1]["snr_db"] > stats[0]["snr_db"]


def test_native_outer_loop_matches_the_call_sequence():
    """ppd_reweighted (Algorithm 1's loop in the library) gives bitwise the
    iterate of the same calls made one by one: ppd_iterate, then
    ppd_reweight at omega0 decay^(k+1), then the next solve with W."""
    P = require_gpu()
    import torch
    announce("reweighted loop: native against the call sequence, ppd64")
    w = synth.WORKLOADS["ppd64"]
    inp = synth.make_inputs(w)
    pb = oprob.problem_from_inputs(inp, power_tol=1e-9)
    plan = P.Plan(64, 64, inp.wu[0], inp.wv[0], inp.block_off)
    perm = plan.permutation()
    y = dev(pb.y[perm].astype(np.complex64), torch.complex64)
    U = dev(pb.U[perm], torch.float64)
    a, b = P.PPDState(plan, y), P.PPDState(plan, y)
    stats, Wa = P.reweighted_ppd(plan, a, y, U, pb.eps, 2, 20, omega0=1e-2, decay=0.25, eta=pb.eta, mu=1.0)
    Wb, omega = None, 1e-2
    for k in range(3):
        P.ppd_iterate(plan, b, y, U, pb.eps, 20, W=Wb, eta=pb.eta, mu=1.0)
        if k < 2:
            omega *= 0.25
            Wb = P.ppd_reweight(plan, b.x, omega, Wb)
    torch.cuda.synchronize()
    assert a.iter == b.iter == 60 and len(stats) == 3
    for k in ("x", "xt", "v", "u", "z"):
        assert torch.equal(getattr(a, k), getattr(b, k)), k
    assert torch.equal(Wa, Wb)
