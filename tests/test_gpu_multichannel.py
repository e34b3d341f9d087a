"""The 8-channel workload at full size (512^2, 1M points per channel,
channel frequencies scaled by nu/nu0 in [0.9, 1.1]): sampled Phi outputs of
every channel against the FP64 oracle, the adjoint identity per channel,
the gradient of the multi-channel data fidelity (timed) and its parity with
the oracle's on sampled points (closed form and FP64 difference quotient),
and the gradients of K = 10 unrolled PPD iterations (timed; their parity is
the small-size oracle tests')."""
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
    assert torch.isfinite(g).all()
    # Parity of the gradient with the oracle, on the fidelity restricted to a
    # sampled subset S_c of each channel's points (the full 8 x 1M oracle is
    # out of reach): L_S(x) = sum_c sum_{e in S_c} |(Phi_c x)_e - y_ce|^2.
    # GPU: forward Phi and backward Re Phi^H on the masked residual (the
    # library's kernels through autograd).  Oracle: its closed form
    # 2 Re sum_c Phi_Sc^H (Phi_Sc x - y_Sc) element by element, and the FP64
    # central difference of its own L_S (quadratic, so exact up to rounding)
    # along a random direction with h = 1e-3.  Tolerance: the operator bar
    # 1e-5 carried through the residual, 1e-5 (1 + ||Phi_S x|| / ||Phi_S x - y_S||).
    xs = (0.9 * x).clone().requires_grad_(True)
    xs64 = host(0.9 * x).astype(np.float64)
    g_or = np.zeros((n, n))
    r_norm2, px_norm2 = 0.0, 0.0
    ops = []
    total = 0.0
    for c, (p, yc) in enumerate(zip(plans, ys)):
        perm = p.permutation()
        pick = np.sort(np.random.default_rng(200 + c).choice(p.M, 2000, replace=False))   # user order
        inv = np.empty(p.M, np.int64)
        inv[perm] = np.arange(p.M)
        mask = torch.zeros(p.M, dtype=torch.float32, device="cuda")
        mask[torch.as_tensor(inv[pick], device="cuda")] = 1.0
        r = A.phi(p, xs) - yc
        total = total + ((r.real ** 2 + r.imag ** 2) * mask).sum()
        yu = np.empty(p.M, np.complex64)
        yu[perm] = host(yc)
        op = onf.Nufft(inp.wu[c][pick], inp.wv[c][pick], n, n)
        yS = yu[pick].astype(np.complex128)
        res = op.phi(xs64) - yS
        g_or += 2.0 * op.phit(res)
        r_norm2 += float(np.sum(np.abs(res) ** 2))
        px_norm2 += float(np.sum(np.abs(op.phi(xs64)) ** 2))
        ops.append((op, yS))
    total.backward()
    g_gpu = host(xs.grad).astype(np.float64)
    tol = 1e-5 * (1.0 + math.sqrt(px_norm2 / r_norm2))
    e_g = rel_err(g_gpu, g_or)
    assert e_g <= tol, (e_g, tol)
    dirn = np.random.default_rng(98).standard_normal((n, n))
    hfd = 1e-3

    def loss_or(xv):
        return sum(float(np.sum(np.abs(op.phi(xv) - yS) ** 2)) for op, yS in ops)
    fd = (loss_or(xs64 + hfd * dirn) - loss_or(xs64 - hfd * dirn)) / (2.0 * hfd)
    ad = float(np.sum(g_gpu * dirn))
    assert abs(ad - fd) <= tol * np.linalg.norm(g_or) * np.linalg.norm(dirn), (ad, fd)
    print(f"[multichannel] sampled-fidelity gradient vs oracle: rel err {e_g:.2e} (tol {tol:.2e}); "
          f"directional derivative {ad:.6e} vs oracle difference quotient {fd:.6e}", flush=True)
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
