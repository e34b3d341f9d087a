"""Differentiable measurement and sparsity operators, and unrolled PPD.

The forward and backward passes of the linear operators are the library's
HIP kernels: the adjoint of `Phi` (Sec. 2) is the gridding path
`Re Phi^H`, and the SARA analysis and synthesis (Sec. 5.1) are each other's
adjoint (Psi Psi^H = I, real).  Torch's convention for a real loss L of a
complex tensor y is grad = dL/dRe(y) + i dL/dIm(y); with it

    y = Phi x (x real)   ->  grad_x = Re(Phi^H grad_y)
    x = Re(Phi^H y)      ->  grad_y = Phi grad_x

`unrolled_ppd` composes K iterations of Algorithm 3 from these operators and
torch element-wise operations (the proximity operators are piecewise smooth:
clip, max(0, .) and the l2-ball projection), optionally checkpointing each
iteration so memory stays at one iteration's activations.
"""
from __future__ import annotations

from typing import Optional, Sequence

import torch
import torch.utils.checkpoint

from . import ppd as P


class PhiFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, plan):
        ctx.plan = plan
        return P.ppd_phi(plan, x.detach().contiguous().to(torch.float32))

    @staticmethod
    def backward(ctx, g):
        return P.ppd_phit(ctx.plan, g.contiguous().to(torch.complex64)), None


class PhitFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, y, plan):
        ctx.plan = plan
        return P.ppd_phit(plan, y.detach().contiguous().to(torch.complex64))

    @staticmethod
    def backward(ctx, g):
        return P.ppd_phi(ctx.plan, g.contiguous().to(torch.float32)), None


class SaraAnalysisFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, plan):
        ctx.plan = plan
        return P.ppd_sara(plan, P.SARA_ANALYSIS, x.detach().contiguous().to(torch.float32))

    @staticmethod
    def backward(ctx, g):
        return P.ppd_sara(ctx.plan, P.SARA_SYNTHESIS, g.contiguous().to(torch.float32)), None


class SaraSynthesisFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u, plan):
        ctx.plan = plan
        return P.ppd_sara(plan, P.SARA_SYNTHESIS, u.detach().contiguous().to(torch.float32))

    @staticmethod
    def backward(ctx, g):
        return P.ppd_sara(ctx.plan, P.SARA_ANALYSIS, g.contiguous().to(torch.float32)), None


def phi(plan, x):
    """y = Theta G F Z x, differentiable (plan order)."""
    return PhiFn.apply(x, plan)


def phit(plan, y):
    """x = Re Phi^H y, differentiable."""
    return PhitFn.apply(y, plan)


def sara_analysis(plan, x):
    return SaraAnalysisFn.apply(x, plan)


def sara_synthesis(plan, u):
    return SaraSynthesisFn.apply(u, plan)


def data_fidelity(plan, x, y):
    """||Phi x - y||_2^2."""
    r = phi(plan, x) - y
    return (r.real ** 2 + r.imag ** 2).sum()


def multichannel_fidelity(plans: Sequence, x, ys: Sequence):
    """sum_c ||Phi_c x - y_c||^2 over frequency channels sharing one sky."""
    return sum(data_fidelity(p, x, y) for p, y in zip(plans, ys))


def _proj_ball(q, y, eps: float):
    """P_B (Sec. 3.3, eq. proj-L2) for one block, differentiable."""
    d = q - y
    r = torch.sqrt((d.real ** 2 + d.imag ** 2).sum())
    scale = torch.clamp(eps / r, max=1.0)
    return y + d * scale


def ppd_iteration(plan, block_off, y, U, eps, x, xt, v, u, z, *, tau: float, eta: float, zeta: float = 1.0,
                  lam: float = 1.0, alpha: float = 1e-4, mu: float = 1.0, n_itr: int = 1):
    """One iteration of Algorithm 3 as differentiable torch code (plan order).

    x, xt: (ny, nx) float32; v: (M,) complex64; u: (9, ny, nx) float32;
    z: (M,) complex128; y: (M,) complex64; U: (M,) float64; eps: (d,) floats.
    Returns the new (x, xt, v, u, z)."""
    g = phi(plan, xt).to(torch.complex128)                          # step 4 + Theta G
    w = v.to(torch.complex128) / U + g                              # step 10 argument
    yd = y.to(torch.complex128)
    zs, vs = [], []
    for j in range(len(block_off) - 1):
        s = slice(int(block_off[j]), int(block_off[j + 1]))
        zj = z[s]
        for _ in range(n_itr):                                      # Algorithm 2
            zj = _proj_ball(zj - mu * U[s] * (zj - w[s]), yd[s], float(eps[j]))
        vbar = U[s] * (w[s] - zj)                                   # step 10
        vs.append(v[s].to(torch.complex128) + lam * (vbar - v[s].to(torch.complex128)))  # step 11
        zs.append(zj)
    v_new = torch.cat(vs).to(torch.complex64)
    z_new = torch.cat(zs)
    ubar = torch.clamp(u + sara_analysis(plan, xt), -alpha, alpha)  # step 19
    u_new = u + lam * (ubar - u)                                    # step 20
    grad = eta * phit(plan, v_new) + zeta * sara_synthesis(plan, u_new)   # steps 12, 21
    xbar = torch.relu(x - tau * grad)                               # step 28
    x_new = x + lam * (xbar - x)                                    # step 29
    xt_new = 2.0 * xbar - x                                         # step 30
    return x_new, xt_new, v_new, u_new, z_new


def unrolled_ppd(plan, block_off, y, U, eps, x0, K: int, *, checkpoint: bool = True, state=None, **params):
    """K differentiable PPD iterations from x = x~ = x0 (v = 0, u = 0, z = y
    unless `state` = (x, xt, v, u, z) is given).  Returns the final x."""
    if state is None:
        x, xt = x0, x0
        v = torch.zeros_like(y)
        u = torch.zeros((9,) + tuple(x0.shape), dtype=torch.float32, device=x0.device)
        z = y.to(torch.complex128)
    else:
        x, xt, v, u, z = state
    for _ in range(K):
        if checkpoint:
            x, xt, v, u, z = torch.utils.checkpoint.checkpoint(
                lambda *s: ppd_iteration(plan, block_off, y, U, eps, *s, **params),
                x, xt, v, u, z, use_reentrant=False)
        else:
            x, xt, v, u, z = ppd_iteration(plan, block_off, y, U, eps, x, xt, v, u, z, **params)
    return x
