"""The 2048x2048, 20M-visibility, 64-block workload (on-the-fly
Kaiser-Bessel weights): sampled operator outputs against the FP64 oracle at
full size, the adjoint identity at full size, elementwise iteration parity on
the 512x512 crop problem at the same visibility density (oracle), the crop
problem's 200-iteration SNR trajectory against the oracle's
(tests/golden/make_crop2048.py), and a 200-iteration PPD run at full size."""
import json
import math
import os
import time

import numpy as np
import pytest

import synth
from oracle import nufft as onf
from oracle import ppd as O
from oracle import problem as oprob
from oracle import sara as osara

from gpu_util import announce, assert_op_close, check_trajectory, dev, host, rel_err, require_gpu

pytestmark = pytest.mark.gpu

CROP_GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "crop2048_traj.json")
CROP_SEED = 901
_BIG = {}


def _big():
    if "inp" not in _BIG:
        _BIG["inp"] = synth.make_inputs(synth.WORKLOADS["ppd2048"])
    return _BIG["inp"]


def _crop():
    """The 512^2 crop problem's inputs and oracle problem (built once)."""
    if "crop" not in _BIG:
        c = synth.crop_inputs(_big(), 512, 16, seed=CROP_SEED)
        _BIG["crop"] = (c, oprob.problem_from_inputs(c, with_eta=False))
    return _BIG["crop"]


def test_phi_sampled_and_adjoint_full_size():
    P = require_gpu()
    import torch
    announce("ppd2048 phi sampled + adjoint identity")
    inp = _big()
    n = inp.workload.n
    plan = P.Plan(n, n, inp.wu[0], inp.wv[0], inp.block_off)
    perm = plan.permutation()
    x = inp.x_true.astype(np.float32)
    y = P.ppd_phi(plan, dev(x, torch.float32))
    yu = np.empty(plan.M, np.complex64)
    yu[perm] = host(y)
    rng = np.random.default_rng(3)
    pick = np.sort(rng.choice(plan.M, 2000, replace=False))
    op = onf.Nufft(inp.wu[0][pick], inp.wv[0][pick], n, n)
    ref = op.phi(x.astype(np.float64))
    assert rel_err(yu[pick], ref) < 1e-5, rel_err(yu[pick], ref)
    assert np.abs(yu[pick] - ref).max() < 1e-5 * np.abs(ref).max()
    # <Phi x, r> = <x, Re Phi^H r> for a random r, FP64 dot products
    r = torch.randn(plan.M, dtype=torch.complex64, device="cuda", generator=torch.Generator("cuda").manual_seed(5))
    xb = P.ppd_phit(plan, r)
    lhs = float((y.to(torch.complex128).conj() * r.to(torch.complex128)).real.sum())
    rhs = float((dev(x, torch.float64) * xb.double()).sum())
    scale = float(y.abs().double().norm() * r.abs().double().norm())
    assert abs(lhs - rhs) <= 1e-5 * scale, (lhs, rhs, scale)


def test_crop_problem_iterations_match_oracle():
    """512^2 crop of the 2048^2 sky with a 1/16 subset of the points (the
    same points per grid cell): three fused iterations against the oracle."""
    P = require_gpu()
    import torch
    announce("ppd2048 crop 512 parity")
    c, pb = _crop()
    n = 512
    plan = P.Plan(n, n, c.wu[0], c.wv[0], c.block_off)
    perm = plan.permutation()
    y = dev(pb.y[perm].astype(np.complex64), torch.complex64)
    U = dev(pb.U[perm], torch.float64)
    # the step size from the oracle's own power iteration (any value serves
    # parity, as long as both sides use the same)
    eta = 1.0 / oprob.power_norm(pb.op, pb.U, c.power_start, tol=1e-3, max_iter=20)
    st = P.PPDState(plan, y)
    ost = O.init_state(n, n, pb.y)
    O.iterate(pb.op, pb.y, pb.U, pb.eps, pb.block_off, O.Params(eta=eta), ost, 3)
    P.ppd_iterate(plan, st, y, U, pb.eps, 3, eta=eta)
    assert_op_close(host(st.x), ost.x, what="x")
    assert_op_close(host(st.v), ost.v[perm], what="v")
    u_scale = np.abs(osara.analysis(ost.xt)).max()
    assert np.abs(host(st.u) - ost.u).max() <= 1e-5 * u_scale


def test_crop_problem_200_iterations_vs_oracle_trajectory():
    """200 fused iterations of the crop problem with the oracle's step size:
    SNR within 0.05 dB of the oracle's every 25 iterations."""
    P = require_gpu()
    import torch
    if not os.path.exists(CROP_GOLDEN):
        pytest.fail("missing golden file: run tests/golden/make_crop2048.py")
    with open(CROP_GOLDEN) as f:
        ref = json.load(f)
    assert ref["crop_seed"] == CROP_SEED
    announce("ppd2048 crop 512, 200 iterations vs oracle trajectory")
    c, pb = _crop()
    assert np.allclose(pb.eps, ref["eps"], rtol=1e-12) and ref["M"] == pb.y.size
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        plan = P.Plan(512, 512, c.wu[0], c.wv[0], c.block_off, stream=stream)
        check_trajectory(P, plan, pb, plan.permutation(), ref, False, "crop2048")


def test_ppd2048_200_iterations():
    P = require_gpu()
    import torch
    announce("ppd2048 200 iterations")
    inp = _big()
    w = inp.workload
    n = w.n
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        plan = P.Plan(n, n, inp.wu[0], inp.wv[0], inp.block_off, stream=stream)
        perm = plan.permutation()
        U = P.ppd_uniform_weights(plan)
        xt = dev(inp.x_true.astype(np.float32), torch.float32)
        y0 = P.ppd_phi(plan, xt)
        sigma = math.sqrt(float((y0.abs().double() ** 2).sum()) / w.M * 10.0 ** (-w.isnr_db / 10.0))
        y = (y0 + sigma * dev(inp.noise[0][perm].astype(np.complex64), torch.complex64)).contiguous()
        Mj = np.diff(inp.block_off).astype(np.float64)
        eps = sigma * np.sqrt(Mj + 2.0 * np.sqrt(Mj))
        norm2, _ = P.ppd_op_norm(plan, U, dev(inp.power_start.astype(np.float32), torch.float32), 300, 1e-7)
        st = P.PPDState(plan, y)
        snr = []
        stream.synchronize()
        t0 = time.perf_counter()
        for k in range(8):
            s = P.ppd_iterate(plan, st, y, U, eps, 25, eta=1.0 / norm2, use_graph=True, x_true=xt)
            snr.append(s["snr_db"])
        dt = time.perf_counter() - t0
    print(f"[scale] ppd2048: SNR every 25 iterations {' '.join(f'{v:.2f}' for v in snr)}; "
          f"{200 / dt:.1f} iterations/s including statistics", flush=True)
    assert all(np.isfinite(snr))
    assert snr[-1] > snr[0] + 3.0
    assert all(b >= a - 0.05 for a, b in zip(snr, snr[1:]))
