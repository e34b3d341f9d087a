"""ppd_ellipsoid_proj_noalloc (no plan, no device allocation) against
ppd_ellipsoid_proj on the same plan-order inputs: FP64, the same Algorithm 2
arithmetic with the block norms summed in another order, so within 1e-12
relative.  Two calls in a row, the second with a smaller input (fewer
points and blocks) on the same GPU's fixed array; an oversized call is
rejected before any launch."""
import ctypes

import numpy as np
import pytest

import synth
from oracle import problem as oprob

from gpu_util import announce, dev, host, rel_err, require_gpu

pytestmark = pytest.mark.gpu


def _case(P, seed, n, M, d, n_itr):
    import torch
    x, wu, wv, off = synth.small_case(n, M, seed=seed, d=d)
    plan = P.Plan(n, n, wu, wv, off, chunk=256)
    perm = plan.permutation()
    rng = np.random.default_rng(seed)
    y = (rng.standard_normal(M) + 1j * rng.standard_normal(M)).astype(np.complex64)
    w = y.astype(np.complex128) + rng.standard_normal(M) + 1j * rng.standard_normal(M)
    U = oprob.uniform_weights(wu, wv, n, n)
    z0 = y.astype(np.complex128) + 0.1 * (rng.standard_normal(M) + 1j * rng.standard_normal(M))
    eps = np.array([0.6 * np.linalg.norm((w - y)[off[j]:off[j + 1]]) for j in range(d)])
    eps[d // 2] = 10 * np.linalg.norm((w - y)[off[d // 2]:off[d // 2 + 1]])   # one block already inside
    wd, yd, Ud = dev(w[perm], torch.complex128), dev(y[perm], torch.complex64), dev(U[perm], torch.float64)
    z_ref = dev(z0[perm], torch.complex128)
    P.ppd_ellipsoid_proj(plan, wd, yd, Ud, eps, n_itr, 1.0, z_ref)
    z_na = dev(z0[perm], torch.complex128)
    # plan order keeps every block in its own range, so the same offsets apply
    P.ppd_ellipsoid_proj_noalloc(wd, yd, Ud, off, eps, n_itr, 1.0, z_na)
    torch.cuda.synchronize()
    return host(z_na), host(z_ref), (wd, yd, Ud, off, eps)


@pytest.mark.parametrize("n_itr", [1, 5])
def test_noalloc_matches_plan_entry_point(n_itr):
    P = require_gpu()
    announce(f"ellipsoid proj noalloc n_itr={n_itr}")
    big = _case(P, 61, 64, 40000, 5, n_itr)      # one block spans several 8192-point chunks
    assert rel_err(big[0], big[1]) < 1e-12, rel_err(big[0], big[1])
    small = _case(P, 62, 32, 3000, 2, n_itr)     # fewer points and blocks on the same array
    assert rel_err(small[0], small[1]) < 1e-12, rel_err(small[0], small[1])


def test_noalloc_rejects_oversized_inputs():
    P = require_gpu()
    import torch
    announce("ellipsoid proj noalloc limits")
    w = torch.zeros(8, dtype=torch.complex128, device="cuda")
    y = torch.zeros(8, dtype=torch.complex64, device="cuda")
    U = torch.ones(8, dtype=torch.float64, device="cuda")
    z = torch.zeros(8, dtype=torch.complex128, device="cuda")
    off = np.arange(0, 4097 * 8 + 1, 8, dtype=np.int64)[: 4098]   # 4097 blocks > 4096
    L = P.lib()
    status = L.ppd_ellipsoid_proj_noalloc(
        w.data_ptr(), y.data_ptr(), U.data_ptr(), 4097, off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
        np.ones(4097).ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 1, 1.0, z.data_ptr(), None)
    assert status == P.PPD_EINVAL
    assert "d must be in" in L.ppd_last_error().decode()
