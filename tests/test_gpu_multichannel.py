"""The 8-channel workload at full size (512^2, 1M points per channel,
channel frequencies scaled by nu/nu0 in [0.9, 1.1]): sampled Phi outputs of
every channel against the FP64 oracle, the adjoint identity per channel,
and the gradients of the multi-channel data fidelity and of K = 10 unrolled
PPD iterations (timed; their parity is the small-size oracle tests')."""
import math
import time

import numpy as np
import pytest

import synth
from oracle import nufft as onf

from gpu_util import announce, dev, host, rel_err, require_gpu

pytestmark = pytest.mark.gpu


def test_multichannel_full_size():
    P = require_gpu()
    import torch
    from paper_1701_01748_amd import autograd as A
    announce("multichan512 full size")
    w = synth.WORKLOADS["multichan512"]
    inp = synth.make_inputs(w)
    n, C = w.n, w.n_chan
    x = dev(inp.x_true.astype(np.float32), torch.float32)
    rng = np.random.default_rng(11)
    plans, ys = [], []
    for c in range(C):
        plan = P.Plan(n, n, inp.wu[c], inp.wv[c], inp.block_off)
        perm = plan.permutation()
        y0 = P.ppd_phi(plan, x)
        yu = np.empty(plan.M, np.complex64)
        yu[perm] = host(y0)
        pick = np.sort(rng.choice(plan.M, 500, replace=False))
        ref = onf.Nufft(inp.wu[c][pick], inp.wv[c][pick], n, n).phi(inp.x_true.astype(np.float32).astype(np.float64))
        assert rel_err(yu[pick], ref) < 1e-5, (c, rel_err(yu[pick], ref))
        r = torch.randn(plan.M, dtype=torch.complex64, device="cuda",
                        generator=torch.Generator("cuda").manual_seed(c))
        xb = P.ppd_phit(plan, r)
        lhs = float((y0.to(torch.complex128).conj() * r.to(torch.complex128)).real.sum())
        rhs = float((x.double() * xb.double()).sum())
        assert abs(lhs - rhs) <= 1e-5 * float(y0.abs().double().norm() * r.abs().double().norm())
        sigma = math.sqrt(float((y0.abs().double() ** 2).sum()) / plan.M * 10.0 ** (-w.isnr_db / 10.0))
        ys.append((y0 + sigma * dev(inp.noise[c][perm].astype(np.complex64), torch.complex64)).contiguous())
        plans.append(plan)
    # gradient of sum_c ||Phi_c x - y_c||^2 at x = 0.9 x_true
    xg = (0.9 * x).clone().requires_grad_(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(5):
        xg.grad = None
        A.multichannel_fidelity(plans, xg, ys).backward()
    torch.cuda.synchronize()
    t_mc = (time.perf_counter() - t0) / 5
    g = xg.grad.detach()
    # the gradient is 2 Re sum_c Phi_c^H (Phi_c x - y_c): check it along a random direction
    # against the FP64 difference quotient of the loss (the loss is quadratic: exact up to rounding)
    d = torch.randn_like(x, generator=torch.Generator("cuda").manual_seed(99))
    h = 1e-2 * float(x.abs().max())

    def loss64(xv):
        s = 0.0
        for p, y in zip(plans, ys):
            rr = P.ppd_phi(p, xv).to(torch.complex128) - y.to(torch.complex128)
            s += float((rr.abs() ** 2).sum())
        return s
    fd = (loss64((0.9 * x + h * d).contiguous()) - loss64((0.9 * x - h * d).contiguous())) / (2 * h)
    ad = float((g.double() * d.double()).sum())
    assert abs(ad - fd) <= 1e-3 * abs(fd) + 1e-6 * float(g.double().norm() * d.double().norm()), (ad, fd)
    # K = 10 unrolled PPD iterations on channel 0, gradient w.r.t. x0 and y
    plan = plans[0]
    U = P.ppd_uniform_weights(plan)
    Mj = np.diff(inp.block_off).astype(np.float64)
    sigma0 = math.sqrt(float((P.ppd_phi(plan, x).abs().double() ** 2).sum()) / plan.M * 10.0 ** (-w.isnr_db / 10.0))
    eps = sigma0 * np.sqrt(Mj + 2.0 * np.sqrt(Mj))
    norm2, _ = P.ppd_op_norm(plan, U, dev(inp.power_start.astype(np.float32), torch.float32), 200, 1e-6)
    x0 = torch.zeros_like(x).requires_grad_(True)
    yd = ys[0].clone().requires_grad_(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    xT = A.unrolled_ppd(plan, inp.block_off, yd, U, eps, x0, 10, checkpoint=True, tau=0.49, eta=1.0 / norm2,
                        mu=1.0, n_itr=1)
    ((xT - x) ** 2).sum().backward()
    torch.cuda.synchronize()
    t_un = time.perf_counter() - t0
    assert torch.isfinite(x0.grad).all() and torch.isfinite(yd.grad.real).all()
    assert float(yd.grad.abs().max()) > 0.0
    print(f"[multichannel] 8 x 1M fidelity forward+backward {1e3 * t_mc:.2f} ms; "
          f"unrolled PPD K=10 (1M points) forward+backward {1e3 * t_un:.1f} ms", flush=True)
