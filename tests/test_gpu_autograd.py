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


@pytest.mark.parametrize("n_itr", [1, 3])
def test_dual_update_vjp_matches_oracle_differences(n_itr):
    """The data-dual update's forward against the oracle's (Algorithm 2 per
    block, then the generalised Moreau step), and its VJP kernels against
    FP64 central differences of the oracle's update along random directions
    of g, v, z and y (blocks away from the ball boundary: smooth)."""
    P = require_gpu()
    import torch
    from oracle import prox as oprox
    announce(f"dual update VJP n_itr={n_itr}")
    n, M, d = 64, 6000, 3
    x, wu, wv, off = synth.small_case(n, M, seed=36, d=d)
    plan = P.Plan(n, n, wu, wv, off)
    perm = plan.permutation()
    rng = np.random.default_rng(12)

    def cplx(k, s=1.0):
        return s * (rng.standard_normal(k) + 1j * rng.standard_normal(k))
    y = cplx(M).astype(np.complex64).astype(np.complex128)
    g = cplx(M, 0.5).astype(np.complex64).astype(np.complex128)
    v = cplx(M, 0.2).astype(np.complex64).astype(np.complex128)
    z = y + cplx(M, 0.1)
    U = np.exp(rng.uniform(np.log(0.05), 0.0, M))
    mu, lam = 1.0, 0.8
    w0 = v / U + g
    eps = np.array([0.5, 3.0, 0.7]) * np.array([np.linalg.norm((w0 - y)[off[j]:off[j + 1]]) for j in range(d)])

    def oracle(g, v, z, y):
        w = v / U + g
        zn = np.empty_like(z)
        for j in range(d):
            s = slice(off[j], off[j + 1])
            zn[s] = oprox.fb_ellipsoid(w[s], y[s], eps[j], U[s], mu, n_itr, z[s])
        return v + lam * (U * (w - zn) - v), zn

    vo, zo = oracle(g, v, z, y)
    dg = lambda a, dt: dev(a[perm].astype(dt), getattr(torch, dt.__name__))
    gd, vd, yd = dg(g, np.complex64), dg(v, np.complex64), dg(y, np.complex64)
    zd, Ud = dev(z[perm], torch.complex128), dev(U[perm], torch.float64)
    v1, z1, zs = P.ppd_dual_update(plan, gd, yd, Ud, eps, vd, zd, n_itr, mu, lam, keep=True)
    assert_op_close(host(v1), vo[perm], what="v'")
    assert_op_close(host(z1), zo[perm], what="z'")
    # L = Re <a, v'> + Re <b, z'>: its gradients from the VJP kernels
    a, b = cplx(M), cplx(M)
    g_g, g_v, g_z, g_y = P.ppd_dual_update_vjp(plan, gd, yd, Ud, eps, vd, zd, n_itr, mu, lam, zs,
                                               dev(a[perm].astype(np.complex64), torch.complex64),
                                               dev(b[perm], torch.complex128))
    grads = {}
    for name, t in (("g", g_g), ("v", g_v), ("z", g_z), ("y", g_y)):
        gu = np.empty(M, np.complex128)
        gu[perm] = host(t)
        grads[name] = gu
    a64 = a.astype(np.complex64).astype(np.complex128)

    def L(g_, v_, z_, y_):
        vv, zz = oracle(g_, v_, z_, y_)
        return float(np.sum((a64.conj() * vv).real) + np.sum((b.conj() * zz).real))
    h = 1e-6
    for name in ("g", "v", "z", "y"):
        dirn = cplx(M)
        dirn /= np.linalg.norm(dirn)
        args_p = dict(g_=g, v_=v, z_=z, y_=y)
        args_m = dict(args_p)
        args_p[name + "_"] = args_p[name + "_"] + h * dirn
        args_m[name + "_"] = args_m[name + "_"] - h * dirn
        fd = (L(**args_p) - L(**args_m)) / (2 * h)
        ad = float(np.sum(grads[name].real * dirn.real + grads[name].imag * dirn.imag))
        assert abs(ad - fd) <= 1e-5 * np.linalg.norm(grads[name]) + 1e-6 * abs(fd), (name, ad, fd)
