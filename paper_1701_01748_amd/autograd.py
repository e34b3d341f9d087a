"""Differentiable measurement and sparsity operators, and unrolled PPD.

The forward and backward passes of the linear operators are the library's
HIP kernels: the adjoint of `Phi` (Sec. 2) is the gridding path
`Re Phi^H`, and the SARA analysis and synthesis (Sec. 5.1) are each other's
adjoint (Psi Psi^H = I, real).  Torch's convention for a real loss L of a
complex tensor y is grad = dL/dRe(y) + i dL/dIm(y); with it

    y = Phi x (x real)   ->  grad_x = Re(Phi^H grad_y)
    x = Re(Phi^H y)      ->  grad_y = Phi grad_x

`unrolled_ppd` composes K iterations of Algorithm 3 from these operators and
the library's three updates (data dual, sparsity dual, primal), whose
backward passes are the library's VJP kernels: the l2-ball projection's
Jacobian per block, the clip mask and the positivity mask (the proximity
operators are piecewise smooth).  Each iteration can be checkpointed, so
memory stays at one iteration's activations.
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


class DualUpdateFn(torch.autograd.Function):
    """(v', z') of the data-dual update from g = Theta G F Z x~, v, z and y;
    backward: the library's VJP kernels (the P_B Jacobian per block)."""

    @staticmethod
    def forward(ctx, g, v, z, y, plan, U, eps, n_itr, mu, lam):
        g, v, z, y = (t.detach().contiguous() for t in (g, v, z, y))
        v_out, z_out, zs = P.ppd_dual_update(plan, g, y, U, eps, v, z, n_itr, mu, lam, keep=True)
        ctx.save_for_backward(g, v, z, y, zs)
        ctx.args = (plan, U, eps, n_itr, mu, lam)
        return v_out, z_out

    @staticmethod
    def backward(ctx, gv, gz):
        g, v, z, y, zs = ctx.saved_tensors
        plan, U, eps, n_itr, mu, lam = ctx.args
        gv = None if gv is None else gv.contiguous().to(torch.complex64)
        gz = None if gz is None else gz.contiguous().to(torch.complex128)
        g_g, g_v, g_z, g_y = P.ppd_dual_update_vjp(plan, g, y, U, eps, v, z, n_itr, mu, lam, zs, gv, gz)
        return g_g, g_v, g_z, g_y, None, None, None, None, None, None


class SparsityUpdateFn(torch.autograd.Function):
    """u' = u + lambda (clip(u + c, +-alpha) - u); backward: the clip mask."""

    @staticmethod
    def forward(ctx, u, c, plan, alpha, lam):
        u, c = u.detach().contiguous(), c.detach().contiguous()
        ctx.save_for_backward(u, c)
        ctx.args = (plan, alpha, lam)
        return P.ppd_sparsity_update(plan, u, c, alpha, lam)

    @staticmethod
    def backward(ctx, g):
        u, c = ctx.saved_tensors
        plan, alpha, lam = ctx.args
        g_u, g_c = P.ppd_sparsity_update_vjp(plan, u, c, alpha, lam, g.contiguous().to(torch.float32))
        return g_u, g_c, None, None, None


class PrimalUpdateFn(torch.autograd.Function):
    """(x', x~') of the primal update from x, a = Re Phi^H v', b = Psi u';
    backward: the P_C mask."""

    @staticmethod
    def forward(ctx, x, a, b, plan, tau, eta, zeta, lam):
        x, a, b = (t.detach().contiguous() for t in (x, a, b))
        ctx.save_for_backward(x, a, b)
        ctx.args = (plan, tau, eta, zeta, lam)
        return P.ppd_primal_update(plan, x, a, b, tau, eta, zeta, lam)

    @staticmethod
    def backward(ctx, gx, gxt):
        x, a, b = ctx.saved_tensors
        plan, tau, eta, zeta, lam = ctx.args
        gx = None if gx is None else gx.contiguous().to(torch.float32)
        gxt = None if gxt is None else gxt.contiguous().to(torch.float32)
        g_x, g_a, g_b = P.ppd_primal_update_vjp(plan, x, a, b, tau, eta, zeta, lam, gx, gxt)
        return g_x, g_a, g_b, None, None, None, None, None


def ppd_iteration(plan, y, U, eps, x, xt, v, u, z, *, tau: float, eta: float, zeta: float = 1.0,
                  lam: float = 1.0, alpha: float = 1e-4, mu: float = 1.0, n_itr: int = 1):
    """One differentiable iteration of Algorithm 3 in the library's data flow
    (plan order): the data-dual update of every block on Theta G F Z x~, the
    sparsity dual update on Psi^H x~, and the primal update on
    Re Phi^H v' and Psi u'; every forward and backward step is a HIP kernel.

    x, xt: (ny, nx) float32; v: (M,) complex64; u: (9, ny, nx) float32;
    z: (M,) complex128; y: (M,) complex64; U: (M,) float64; eps: (d,).
    Returns the new (x, xt, v, u, z)."""
    g = phi(plan, xt)
    v_new, z_new = DualUpdateFn.apply(g, v, z, y, plan, U, eps, n_itr, mu, lam)
    u_new = SparsityUpdateFn.apply(u, sara_analysis(plan, xt), plan, alpha, lam)
    x_new, xt_new = PrimalUpdateFn.apply(x, phit(plan, v_new), sara_synthesis(plan, u_new), plan, tau, eta, zeta, lam)
    return x_new, xt_new, v_new, u_new, z_new


def unrolled_ppd(plan, block_off, y, U, eps, x0, K: int, *, checkpoint: bool = True, state=None, **params):
    """K differentiable PPD iterations from x = x~ = x0 (v = 0, u = 0, z = y
    unless `state` = (x, xt, v, u, z) is given).  Returns the final x.
    block_off is accepted for compatibility (the plan holds the blocks)."""
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
                lambda *s: ppd_iteration(plan, y, U, eps, *s, **params),
                x, xt, v, u, z, use_reentrant=False)
        else:
            x, xt, v, u, z = ppd_iteration(plan, y, U, eps, x, xt, v, u, z, **params)
    return x
