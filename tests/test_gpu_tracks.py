"""PD vs PPD on the tracks256 workload (256x256, 65536 points on 36
elliptical tracks, 4 uneven blocks, 30 dB): GPU SNR trajectories against the
FP64 oracle's (stored by tests/golden/make_tracks256.py), and the number of
iterations each method needs to reach the oracle's final PPD SNR."""
import json
import os

import numpy as np
import pytest

import synth
from oracle import problem as oprob

from gpu_util import announce, dev, require_gpu

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "tracks256_snr.json")


def test_pd_vs_ppd_tracks256():
    P = require_gpu()
    import torch
    if not os.path.exists(GOLDEN):
        pytest.fail("missing golden file: run tests/golden/make_tracks256.py")
    with open(GOLDEN) as f:
        ref = json.load(f)
    w = synth.WORKLOADS["tracks256"]
    inp = synth.make_inputs(w)
    pb = oprob.problem_from_inputs(inp, with_eta=False)
    assert np.allclose(pb.eps, ref["eps"], rtol=1e-12)
    plan = P.Plan(w.n, w.n, inp.wu[0], inp.wv[0], inp.block_off)
    perm = plan.permutation()
    y = dev(pb.y[perm].astype(np.complex64), torch.complex64)
    xt = dev(pb.x_true.astype(np.float32), torch.float32)
    T = ref["iterations"]
    target = ref["ppd"]["snr_db"][-1]
    reached = {}
    for name, U, eta in [("ppd", pb.U, ref["eta_ppd"]), ("pd", np.ones_like(pb.U), ref["eta_pd"])]:
        n_itr = ref[name]["n_itr"]
        announce(f"tracks256 {name} n_itr={n_itr} {T} iterations")
        Ud = dev(U[perm], torch.float64)
        st = P.PPDState(plan, y)
        step = 25
        gsnr = []
        for k in range(T // step):
            s = P.ppd_iterate(plan, st, y, Ud, pb.eps, step, eta=eta, mu=1.0 / U.max(), n_itr=n_itr, x_true=xt)
            o = ref[name]["snr_db"][(k + 1) * step - 1]
            assert abs(s["snr_db"] - o) < 0.05, (name, (k + 1) * step, s["snr_db"], o)
            gsnr.append(s["snr_db"])
        hit = [i for i, v in enumerate(ref[name]["snr_db"]) if v >= target - 1e-9]
        reached[name] = (hit[0] + 1) if hit else None
        print(f"[tracks256] {name}: final GPU SNR {gsnr[-1]:.3f} dB, oracle {ref[name]['snr_db'][-1]:.3f} dB, "
              f"iterations to reach {target:.3f} dB: {reached[name]}", flush=True)
    assert reached["ppd"] is not None


def test_ppd_nitr50_tracks256_vs_oracle_trajectory():
    """PPD with 50 Algorithm 2 iterations per outer iteration (the largest
    n_itr of Sec. 5.1) over 500 iterations: SNR within 0.05 dB of the
    oracle's every 25 iterations."""
    P = require_gpu()
    import torch
    with open(GOLDEN) as f:
        ref = json.load(f)
    if "ppd_nitr50" not in ref:
        pytest.fail("golden file lacks the n_itr = 50 run: run tests/golden/make_tracks256.py")
    w = synth.WORKLOADS["tracks256"]
    inp = synth.make_inputs(w)
    pb = oprob.problem_from_inputs(inp, with_eta=False)
    plan = P.Plan(w.n, w.n, inp.wu[0], inp.wv[0], inp.block_off)
    perm = plan.permutation()
    y = dev(pb.y[perm].astype(np.complex64), torch.complex64)
    xt = dev(pb.x_true.astype(np.float32), torch.float32)
    U = dev(pb.U[perm], torch.float64)
    announce("tracks256 ppd n_itr=50, 500 iterations")
    st = P.PPDState(plan, y)
    T, step = ref["iterations"], 25
    for k in range(T // step):
        s = P.ppd_iterate(plan, st, y, U, pb.eps, step, eta=ref["eta_ppd"], mu=1.0 / pb.U.max(), n_itr=50,
                          x_true=xt)
        o = ref["ppd_nitr50"]["snr_db"][(k + 1) * step - 1]
        assert abs(s["snr_db"] - o) < 0.05, ((k + 1) * step, s["snr_db"], o)
    print(f"[tracks256] ppd n_itr=50: final GPU SNR {s['snr_db']:.3f} dB, oracle {o:.3f} dB", flush=True)
