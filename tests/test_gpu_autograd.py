"""GPU tests of the differentiable operators and unrolled PPD against the
FP64 oracle (closed-form gradients and central finite differences)."""
import numpy as np
import pytest

import synth
from oracle import nufft as onf
from oracle import ppd as O
from oracle import problem as oprob
from oracle import sara as osara

from gpu_util import announce, assert_op_close, dev, host, rel_err, require_gpu

pytestmark = pytest.mark.gpu


def _setup(n=64, M=5000, d=2, seed=31):
    P = require_gpu()
    x, wu, wv, off = synth.small_case(n, M, seed=seed, d=d)
    plan = P.Plan(n, n, wu, wv, off)
    perm = plan.permutation()
    return P, plan, perm, x, wu, wv, off


def test_data_fidelity_gradient_matches_closed_form():
    P, plan, perm, x, wu, wv, off = _setup()
    import torch
    from paper_1701_01748_amd import autograd as A
    announce("autograd data fidelity")
    op = onf.Nufft(wu, wv, 64, 64)
    rng = np.random.default_rng(1)
    x32 = (x + 0.1 * rng.standard_normal(x.shape)).astype(np.float32)
    y = (op.phi(x) + 0.05 * (rng.standard_normal(wu.size) + 1j * rng.standard_normal(wu.size))).astype(np.complex64)
    xd = dev(x32, torch.float32).requires_grad_(True)
    yd = dev(y[perm], torch.complex64).requires_grad_(True)
    loss = A.data_fidelity(plan, xd, yd)
    loss.backward()
    r = op.phi(x32.astype(np.float64)) - y.astype(np.complex128)
    gx = 2.0 * op.phit(r)                         # grad_x ||Phi x - y||^2 = 2 Re Phi^H (Phi x - y)
    gy = -2.0 * r                                 # torch's complex gradient convention
    assert_op_close(host(xd.grad), gx, what="grad x")
    assert_op_close(host(yd.grad), gy[perm], what="grad y")
    assert float(loss) == pytest.approx(float(np.sum(np.abs(r) ** 2)), rel=1e-5)


def test_adjoint_pairs_backpropagate():
    P, plan, perm, x, wu, wv, off = _setup(seed=32)
    import torch
    from paper_1701_01748_amd import autograd as A
    announce("autograd phit and SARA")
    op = onf.Nufft(wu, wv, 64, 64)
    rng = np.random.default_rng(2)
    c = rng.standard_normal((64, 64)).astype(np.float32)
    yv = (rng.standard_normal(wu.size) + 1j * rng.standard_normal(wu.size)).astype(np.complex64)
    yd = dev(yv[perm], torch.complex64).requires_grad_(True)
    (A.phit(plan, yd) * dev(c, torch.float32)).sum().backward()
    assert_op_close(host(yd.grad), op.phi(c.astype(np.float64))[perm], what="grad of <c, Re Phi^H y>")
    xd = dev(c, torch.float32).requires_grad_(True)
    cc = rng.standard_normal((9, 64, 64)).astype(np.float32)
    (A.sara_analysis(plan, xd) * dev(cc, torch.float32)).sum().backward()
    assert_op_close(host(xd.grad), osara.synthesis(cc.astype(np.float64)), what="grad of <c, Psi^H x>")
    ud = dev(cc, torch.float32).requires_grad_(True)
    (A.sara_synthesis(plan, ud) * dev(c, torch.float32)).sum().backward()
    assert_op_close(host(ud.grad), osara.analysis(c.astype(np.float64)), what="grad of <c, Psi u>")


def _oracle_loss(pb, x0, y, K, prm, trace=None):
    st = O.State(x0.copy(), x0.copy(), np.zeros(y.size, complex), np.zeros((9,) + x0.shape), y.copy(), 0)
    O.iterate(pb.op, y, pb.U, pb.eps, pb.block_off, prm, st, K, trace=trace)
    return float(np.sum((st.x - pb.x_true) ** 2))


def _same_sets(ta, t0):
    """Same active sets as the base point, ignoring exact ties there (a dual
    coefficient at +-alpha whose new coefficient is zero up to rounding, a
    pixel whose P_C argument is zero up to rounding): their decision is
    rounding noise and the argument does not move to first order."""
    for a, b in zip(ta, t0):
        if a["proj"] != b["proj"]:
            return False
        for key in ("clip", "pos"):
            tie = np.abs(b[key]) <= 1e-13 * max(np.abs(b[key]).max(), 1e-300)
            if np.any(((a[key] > 0) != (b[key] > 0)) & ~tie):
                return False
    return True


@pytest.mark.parametrize("checkpoint", [True, False])
def test_unrolled_ppd_gradient_matches_finite_differences(checkpoint):
    """K = 10 unrolled PPD iterations: d||x^(K) - x_true||^2 along random
    unit directions of x^(0) and y, GPU autograd vs FP64 oracle central
    differences, on pieces where the active sets agree.  The iteration makes
    ~10^5 clip / positivity / projection decisions, so the step is small
    (h = 1e-6 on unit directions; FP64 keeps the difference quotient to
    ~1e-9)."""
    P = require_gpu()
    import torch
    from paper_1701_01748_amd import autograd as A
    announce(f"unrolled PPD gradient checkpoint={checkpoint}")
    n, M, K = 32, 2500, 10
    x, wu, wv, off = synth.small_case(n, M, seed=33, d=2)
    pb = oprob.make_problem(x, wu, wv, off, synth.noise_unit(M, 233), 30.0, np.ones((n, n)), power_tol=1e-9)
    prm = O.Params(eta=pb.eta, mu=1.0, n_itr=2)
    rng = np.random.default_rng(5)
    x0 = np.abs(0.5 * x + 0.02 * rng.standard_normal(x.shape))
    x0 = x0.astype(np.float32).astype(np.float64)
    plan = P.Plan(n, n, wu, wv, off)
    perm = plan.permutation()
    xd = dev(x0.astype(np.float32), torch.float32).requires_grad_(True)
    yd = dev(pb.y[perm].astype(np.complex64), torch.complex64).requires_grad_(True)
    Ud = dev(pb.U[perm], torch.float64)
    xT = A.unrolled_ppd(plan, off, yd, Ud, pb.eps, xd, K, checkpoint=checkpoint, tau=0.49, eta=pb.eta,
                        mu=1.0, n_itr=2)
    loss = ((xT - dev(pb.x_true.astype(np.float32), torch.float32)) ** 2).sum()
    loss.backward()
    gx, gy_plan = host(xd.grad).astype(np.float64), host(yd.grad).astype(np.complex128)
    gy = np.empty_like(gy_plan)
    gy[perm] = gy_plan
    # forward parity of the unrolled composition against the oracle
    assert float(loss) == pytest.approx(_oracle_loss(pb, x0, pb.y, K, prm), rel=1e-4)
    h = 1e-6
    checked = 0
    for trial in range(4):
        dx = rng.standard_normal(x.shape)
        dx /= np.linalg.norm(dx)
        dy = rng.standard_normal(M) + 1j * rng.standard_normal(M)
        dy /= np.linalg.norm(dy)
        for which in ("x", "y"):
            ta, tb, t0 = [], [], []
            if which == "x":
                fp = _oracle_loss(pb, x0 + h * dx, pb.y, K, prm, ta)
                fm = _oracle_loss(pb, x0 - h * dx, pb.y, K, prm, tb)
                _oracle_loss(pb, x0, pb.y, K, prm, t0)
                ad = float(np.sum(gx * dx))
            else:
                fp = _oracle_loss(pb, x0, pb.y + h * dy, K, prm, ta)
                fm = _oracle_loss(pb, x0, pb.y - h * dy, K, prm, tb)
                _oracle_loss(pb, x0, pb.y, K, prm, t0)
                ad = float(np.sum(gy.real * dy.real + gy.imag * dy.imag))
            if not (_same_sets(ta, t0) and _same_sets(tb, t0)):
                continue                     # a kink between x - h d and x + h d: skip
            fd = (fp - fm) / (2 * h)
            scale = np.linalg.norm(gx) if which == "x" else np.linalg.norm(gy)
            assert abs(ad - fd) <= 2e-3 * abs(fd) + 1e-4 * scale, (which, trial, ad, fd, scale)
            checked += 1
    print(f"[autograd] {checked} of 8 directions on a smooth piece", flush=True)
    assert checked >= 4, "too few directions on a smooth piece"


def test_multichannel_fidelity_gradient():
    P = require_gpu()
    import torch
    from paper_1701_01748_amd import autograd as A
    announce("multichannel gradient")
    n, M, C = 64, 3000, 8
    x, wu, wv, off = synth.small_case(n, M, seed=34)
    plans, ys, ops, perms, yo = [], [], [], [], []
    rng = np.random.default_rng(8)
    for c, f in enumerate(np.linspace(0.9, 1.1, C)):
        cu = (wu.astype(np.float64) * f / 1.1).astype(np.float32)
        cv = (wv.astype(np.float64) * f / 1.1).astype(np.float32)
        p = P.Plan(n, n, cu, cv, off)
        op = onf.Nufft(cu, cv, n, n)
        yc = (op.phi(x) + 0.05 * (rng.standard_normal(M) + 1j * rng.standard_normal(M))).astype(np.complex64)
        plans.append(p); ops.append(op); perms.append(p.permutation()); yo.append(yc)
        ys.append(dev(yc[perms[-1]], torch.complex64))
    x32 = (0.9 * x).astype(np.float32)
    xd = dev(x32, torch.float32).requires_grad_(True)
    A.multichannel_fidelity(plans, xd, ys).backward()
    g = sum(2.0 * op.phit(op.phi(x32.astype(np.float64)) - yc.astype(np.complex128)) for op, yc in zip(ops, yo))
    assert_op_close(host(xd.grad), g, what="multichannel grad")
