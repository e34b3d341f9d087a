"""PD vs PPD on the generalised-Gaussian coverage workloads (Sec. 5.2:
shape beta = 2, 0.5, 0.25 at 30 dB, and 0.25 at 50 dB input SNR), GPU SNR
trajectories against the FP64 oracle's (tests/golden/make_ggd256.py)."""
import json
import os
import time

import numpy as np
import pytest

import synth
from oracle import problem as oprob

from gpu_util import announce, dev, require_gpu

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "ggd256_snr.json")
NAMES = ("ggd256_b2", "ggd256_b05", "ggd256_b025", "ggd256_b025_50db")


@pytest.mark.parametrize("name", NAMES)
def test_ggd_pd_vs_ppd(name):
    P = require_gpu()
    import torch
    with open(GOLDEN) as f:
        ref = json.load(f)[name]
    w = synth.WORKLOADS[name]
    inp = synth.make_inputs(w)
    pb = oprob.problem_from_inputs(inp, with_eta=False)
    assert np.allclose(pb.eps, ref["eps"], rtol=1e-12)
    plan = P.Plan(w.n, w.n, inp.wu[0], inp.wv[0], inp.block_off)
    perm = plan.permutation()
    y = dev(pb.y[perm].astype(np.complex64), torch.complex64)
    xt = dev(pb.x_true.astype(np.float32), torch.float32)
    T, step = ref["iterations"], 25
    for method, U, eta in [("ppd", pb.U, ref["eta_ppd"]), ("pd", np.ones_like(pb.U), ref["eta_pd"])]:
        announce(f"{name} {method} {T} iterations")
        Ud = dev(U[perm], torch.float64)
        st = P.PPDState(plan, y)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(T // step):
            s = P.ppd_iterate(plan, st, y, Ud, pb.eps, step, eta=eta, mu=1.0 / U.max(), x_true=xt)
            o = ref[method]["snr_db"][(k + 1) * step - 1]
            assert abs(s["snr_db"] - o) < 0.05, (name, method, (k + 1) * step, s["snr_db"], o)
        dt = time.perf_counter() - t0
        print(f"[ggd] {name} {method}: final GPU SNR {s['snr_db']:.3f} dB (oracle {o:.3f}), "
              f"{T / dt:.0f} iterations/s with statistics every {step}", flush=True)
