"""GPU parity of the operators behind the C ABI against the FP64 oracle."""
import math

import numpy as np
import pytest

import synth
from oracle import nufft as onf
from oracle import problem as oprob
from oracle import prox as oprox
from oracle import sara as osara

from gpu_util import announce, assert_op_close, dev, host, peak_err, rel_err, require_gpu

pytestmark = pytest.mark.gpu

# (ny, nx, M, d, tile, chunk, theta): multi-tile grids, ragged chunk tails,
# non-square images, several blocks, every tile size
OP_CASES = [
    (64, 64, 4096, 1, 32, 1024, False),
    (64, 64, 5000, 3, 16, 100, True),
    (32, 64, 2999, 2, 64, 64, False),
    (128, 128, 20000, 4, 32, 777, True),
    (16, 16, 37, 1, 32, 64, False),
    (64, 64, 5000, 3, 8, 100, True),
    (128, 128, 20000, 4, 8, 777, False),
    (16, 32, 37, 1, 8, 64, True),
]


def _case(ny, nx, M, d, seed):
    x, wu, wv, off = synth.small_case(ny, M, seed=seed, nx=nx, d=d)
    return x, wu, wv, off


@pytest.mark.parametrize("case", OP_CASES)
def test_phi_phit_parity(case):
    P = require_gpu()
    import torch
    ny, nx, M, d, tile, chunk, with_theta = case
    announce(f"phi/phit {case}")
    x, wu, wv, off = _case(ny, nx, M, d, seed=ny + M)
    theta = np.random.default_rng(5).uniform(0.5, 2.0, M).astype(np.float32) if with_theta else None
    plan = P.Plan(nx, ny, wu, wv, off, theta=theta, tile=tile, chunk=chunk)
    op = onf.Nufft(wu, wv, ny, nx, theta=None if theta is None else theta.astype(np.float64))
    x32 = x.astype(np.float32)
    ref = op.phi(x32.astype(np.float64))
    perm = plan.permutation()
    y_plan = host(P.ppd_phi(plan, dev(x32, torch.float32)))
    y_user = host(P.ppd_phi(plan, dev(x32, torch.float32), order=P.ORDER_USER))
    torch.cuda.synchronize()
    assert_op_close(y_plan, ref[perm], what="phi plan order")
    assert np.array_equal(y_user, y_plan[np.argsort(perm)])
    rng = np.random.default_rng(7)
    v = (rng.standard_normal(M) + 1j * rng.standard_normal(M)).astype(np.complex64)
    xr = op.phit(v.astype(np.complex128))
    xg = host(P.ppd_phit(plan, dev(v, torch.complex64), order=P.ORDER_USER))
    xg2 = host(P.ppd_phit(plan, dev(v[perm], torch.complex64)))
    assert_op_close(xg, xr, what="phit")
    assert_op_close(xg2, xr, what="phit plan order")


def test_phi_matches_direct_nudft_on_gpu():
    P = require_gpu()
    import torch
    announce("phi vs NUDFT 32x32")
    x, wu, wv, off = synth.small_case(32, 500, seed=3, coverage="uniform")
    plan = P.Plan(32, 32, wu, wv, off)
    y = host(P.ppd_phi(plan, dev(x.astype(np.float32), torch.float32), order=P.ORDER_USER))
    yd = onf.nudft(x.astype(np.float32).astype(np.float64), wu, wv)
    assert rel_err(y, yd) < 1e-5


def test_adjoint_dot_product_on_gpu():
    P = require_gpu()
    import torch
    announce("adjoint dot 128x128")
    x, wu, wv, off = synth.small_case(128, 30000, seed=8, d=2)
    plan = P.Plan(128, 128, wu, wv, off)
    rng = np.random.default_rng(1)
    xr = rng.standard_normal((128, 128)).astype(np.float32)
    v = (rng.standard_normal(30000) + 1j * rng.standard_normal(30000)).astype(np.complex64)
    y = host(P.ppd_phi(plan, dev(xr, torch.float32)))
    xt = host(P.ppd_phit(plan, dev(v, torch.complex64)))
    lhs = float(np.real(np.vdot(v.astype(np.complex128), y.astype(np.complex128))))
    rhs = float(np.sum(xr.astype(np.float64) * xt))
    assert abs(lhs - rhs) / (np.linalg.norm(y) * np.linalg.norm(v)) < 1e-5


@pytest.mark.parametrize("shape,levels", [((64, 64), 3), ((32, 64), 3), ((128, 128), 3), ((64, 32), 1),
                                          ((16, 16), 3), ((256, 256), 4)])
def test_sara_parity(shape, levels):
    P = require_gpu()
    import torch
    ny, nx = shape
    announce(f"sara {shape} L={levels}")
    M = 64
    _, wu, wv, off = synth.small_case(16, M, seed=1)
    plan = P.Plan(nx, ny, wu, wv, off, levels=levels)
    rng = np.random.default_rng(ny + nx)
    x = rng.standard_normal((ny, nx)).astype(np.float32)
    ref = osara.analysis(x.astype(np.float64), levels)
    c = host(P.ppd_sara(plan, P.SARA_ANALYSIS, dev(x, torch.float32)))
    for b in range(9):
        assert_op_close(c[b], ref[b], what=f"analysis basis {b}")
    u = rng.standard_normal((9, ny, nx)).astype(np.float32)
    s_ref = osara.synthesis(u.astype(np.float64), levels)
    s = host(P.ppd_sara(plan, P.SARA_SYNTHESIS, dev(u, torch.float32)))
    assert_op_close(s, s_ref, what="synthesis")
    # perfect reconstruction through the GPU
    rec = host(P.ppd_sara(plan, P.SARA_SYNTHESIS, dev(c, torch.float32)))
    assert rel_err(rec, x) < 1e-5
    # dual mode: u <- u + lam (clip(u + Psi^H x, a) - u), out = Psi u
    alpha, lam = 0.05, 0.8
    u0 = 0.05 * rng.standard_normal((9, ny, nx)).astype(np.float32)
    ud = dev(u0, torch.float32)
    out = host(P.ppd_sara(plan, P.SARA_DUAL, dev(x, torch.float32), u=ud, alpha=alpha, lam=lam))
    u0d = u0.astype(np.float64)
    u_ref = u0d + lam * (oprox.clip_dual(u0d + ref, alpha) - u0d)
    assert_op_close(host(ud), u_ref, what="dual u")
    assert_op_close(out, osara.synthesis(u_ref, levels), what="dual synthesis")


@pytest.mark.parametrize("n_itr", [1, 5, 50])
def test_ellipsoid_projection_parity(n_itr):
    P = require_gpu()
    import torch
    announce(f"ellipsoid proj n_itr={n_itr}")
    ny = nx = 64
    M, d = 6000, 3
    x, wu, wv, off = synth.small_case(ny, M, seed=4, d=d)
    plan = P.Plan(nx, ny, wu, wv, off, chunk=256)
    perm = plan.permutation()
    rng = np.random.default_rng(3)
    y = (rng.standard_normal(M) + 1j * rng.standard_normal(M)).astype(np.complex64)
    w = y.astype(np.complex128) + rng.standard_normal(M) + 1j * rng.standard_normal(M)
    U = oprob.uniform_weights(wu, wv, ny, nx)
    z0 = y.astype(np.complex128) + 0.1 * (rng.standard_normal(M) + 1j * rng.standard_normal(M))
    eps = np.array([0.6 * np.linalg.norm((w - y)[off[j]:off[j + 1]]) for j in range(d)])
    eps[1] = 10 * np.linalg.norm((w - y)[off[1]:off[2]])   # one block already feasible
    ref = np.empty(M, np.complex128)
    for j in range(d):
        s = slice(off[j], off[j + 1])
        ref[s] = oprox.fb_ellipsoid(w[s], y[s].astype(np.complex128), eps[j], U[s], 1.0, n_itr, z0[s])
    # plan order inside each block
    zd = dev(z0[perm], torch.complex128)
    P.ppd_ellipsoid_proj(plan, dev(w[perm], torch.complex128), dev(y[perm], torch.complex64),
                         dev(U[perm], torch.float64), eps, n_itr, 1.0, zd)
    assert rel_err(host(zd), ref[perm]) < 1e-12
    # U = 1, mu = 1: one step is the l2-ball projection from any start
    if n_itr == 1:
        zd = dev(z0[perm], torch.complex128)
        P.ppd_ellipsoid_proj(plan, dev(w[perm], torch.complex128), dev(y[perm], torch.complex64),
                             dev(np.ones(M), torch.float64), eps, 1, 1.0, zd)
        zb = np.empty(M, np.complex128)
        for j in range(d):
            s = slice(off[j], off[j + 1])
            zb[s] = oprox.proj_B(w[s], y[s].astype(np.complex128), eps[j])
        assert rel_err(host(zd), zb[perm]) < 1e-14


def test_uniform_weights_bit_exact():
    P = require_gpu()
    announce("uniform weights")
    for (n, M, seed) in [(64, 4096, 1), (256, 65536, 2)]:
        _, wu, wv, off = synth.small_case(n, M, seed=seed, d=2)
        plan = P.Plan(n, n, wu, wv, off)
        U = host(P.ppd_uniform_weights(plan))
        ref = oprob.uniform_weights(wu, wv, n, n)
        assert np.array_equal(U, ref[plan.permutation()])


def test_operator_norm_matches_oracle():
    P = require_gpu()
    import torch
    announce("op norm 64x64")
    inp = synth.make_inputs(synth.WORKLOADS["ppd64"])
    wu, wv = inp.wu[0], inp.wv[0]
    op = onf.Nufft(wu, wv, 64, 64)
    U = oprob.uniform_weights(wu, wv, 64, 64)
    ref = oprob.power_norm(op, U, inp.power_start, tol=1e-10, max_iter=2000)
    plan = P.Plan(64, 64, wu, wv, inp.block_off)
    Ud = dev(U[plan.permutation()], torch.float64)
    g, it = P.ppd_op_norm(plan, Ud, dev(inp.power_start.astype(np.float32), torch.float32), 2000, 1e-10)
    assert abs(g - ref) / ref < 1e-5, (g, ref, it)


@pytest.mark.parametrize("M", [1, 63, 64, 65, 127, 128, 129, 300, 4000])
def test_tile8_item_boundaries(M):
    """All points in one 8 x 8 tile whose halo wraps around the grid edge
    (first taps in the last tile row and column), so that one tile's item
    split (128-point pieces plus a remainder), the batch tails (64-point
    batches), the run pipeline of the matrix-core gridding and the fold's
    wrapped halos are exercised at their boundaries; two blocks share the
    tile when M > 1.  With 4000 points the tile holds 32 items: its fold and
    its neighbours' take a whole workgroup each (heavy tiles)."""
    P = require_gpu()
    import torch
    announce(f"tile-8 boundaries M={M}")
    n = 32
    K = 2 * n
    rng = np.random.default_rng(M)
    # first-tap cell floor(omega K / 2 pi) - 3 in [K - 8, K): floor in [-5, 3)
    wu = (rng.uniform(-4.95, 2.95, M) * 2 * np.pi / K).astype(np.float32)
    wv = (rng.uniform(-4.95, 2.95, M) * 2 * np.pi / K).astype(np.float32)
    off = np.array([0, M], np.int64) if M == 1 else np.array([0, M // 2, M], np.int64)
    plan = P.Plan(n, n, wu, wv, off, tile=8)
    info = plan.info
    assert info.tile == 8 and info.n_chunks == -(-M // 128)
    op = onf.Nufft(wu, wv, n, n)
    x = rng.standard_normal((n, n)).astype(np.float32)
    perm = plan.permutation()
    y = host(P.ppd_phi(plan, dev(x, torch.float32)))
    assert_op_close(y, op.phi(x.astype(np.float64))[perm], what="phi")
    v = (rng.standard_normal(M) + 1j * rng.standard_normal(M)).astype(np.complex64)
    xg = host(P.ppd_phit(plan, dev(v, torch.complex64), order=P.ORDER_USER))
    assert_op_close(xg, op.phit(v.astype(np.complex128)), what="phit")


def test_workspace_plan_matches_allocated_plan():
    """A plan carved from a PyTorch workspace computes exactly what a plan
    with library-allocated buffers computes; a too small or misaligned
    workspace is rejected before any device work."""
    P = require_gpu()
    import ctypes
    import torch
    announce("workspace plan vs allocated plan")
    x, wu, wv, off = synth.small_case(64, 5000, seed=21, d=3)
    pa = P.Plan(64, 64, wu, wv, off, workspace=False)
    pw = P.Plan(64, 64, wu, wv, off)
    assert pa.info.device_bytes == pw.info.device_bytes
    assert pw._ws.numel() >= pw.info.device_bytes
    assert np.array_equal(pa.permutation(), pw.permutation())
    x32 = dev(x.astype(np.float32), torch.float32)
    ya, yw = P.ppd_phi(pa, x32), P.ppd_phi(pw, x32)
    assert np.array_equal(host(ya), host(yw))
    assert np.array_equal(host(P.ppd_phit(pa, ya)), host(P.ppd_phit(pw, ya)))
    eps = 0.5 * np.array([np.linalg.norm(host(ya)[off[j]:off[j + 1]]) for j in range(3)])
    xs = []
    for plan in (pa, pw):
        U = P.ppd_uniform_weights(plan)
        st = P.PPDState(plan, ya)
        P.ppd_iterate(plan, st, ya, U, eps, 3, eta=1e-3, mu=1.0)
        xs.append((host(st.x), host(st.v), host(st.z)))
    for a, b in zip(*xs):
        assert np.array_equal(a, b)
    L = P.lib()
    wu32, wv32 = np.ascontiguousarray(wu, np.float32), np.ascontiguousarray(wv, np.float32)
    off64 = np.ascontiguousarray(off, np.int64)
    desc = P.PlanDesc(64, 64, wu32.size, off64.size - 1, off64.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                      wu32.ctypes.data, wv32.ctypes.data, None, 0.0, 3, 0, 0)
    need = P.plan_workspace_size(64, 64, wu, wv, off)
    buf = torch.empty(need + 256, dtype=torch.uint8, device="cuda")
    for ptr, size in ((buf.data_ptr(), need - 256), (buf.data_ptr() + 16, need)):
        h = ctypes.c_void_p()
        st = L.ppd_plan_create_ws(ctypes.byref(h), ctypes.byref(desc), ctypes.c_void_p(ptr), size,
                                  ctypes.c_void_p(0))
        assert st == P.PPD_EINVAL and not h.value
    h = ctypes.c_void_p()
    assert L.ppd_plan_create_ws(ctypes.byref(h), ctypes.byref(desc), ctypes.c_void_p(buf.data_ptr()), need,
                                ctypes.c_void_p(0)) == 0
    assert L.ppd_plan_destroy(h) == 0
