"""Degenerate and edge cases of Algorithm 3 (ppd_iterate) against the FP64
oracle: a single visibility, the smallest images (square and not) on both
tile kernels, and l2 radii shrunk towards zero (Sec. 3: the data-fidelity
ball collapses onto the data, so every projection returns y)."""
import numpy as np
import pytest

import synth
from oracle import ppd as O
from oracle import problem as oprob
from oracle import sara as osara

from gpu_util import announce, assert_op_close, dev, host, require_gpu

pytestmark = pytest.mark.gpu

# (ny, nx, M, d, tile): one visibility; 37 visibilities on a 16 x 16 image;
# a non-square 16 x 32 image with two blocks; tile 8 (matrix-core gridding)
# and tile 16 (LDS gridding)
EDGE_CASES = [(16, 16, 1, 1, 8), (16, 16, 1, 1, 16), (16, 16, 37, 1, 8), (16, 32, 300, 2, 8),
              (16, 32, 300, 2, 16)]


def _problem(ny, nx, M, d, seed):
    x, wu, wv, off = synth.small_case(ny, M, seed=seed, nx=nx, d=d)
    noise = synth.noise_unit(M, 200 + seed)
    pb = oprob.make_problem(x, wu, wv, off, noise, 30.0, np.ones((ny, nx)), power_tol=1e-9)
    return pb, wu, wv


def _check(P, plan, st, ost, perm, what):
    assert_op_close(host(st.x), ost.x, what=f"x {what}")
    assert_op_close(host(st.xt), ost.xt, what=f"x tilde {what}")
    assert_op_close(host(st.v), ost.v[perm], what=f"v {what}")
    assert_op_close(host(st.z), ost.z[perm], what=f"z {what}")
    u_scale = max(np.abs(osara.analysis(ost.xt)).max(), 1e-30)
    assert np.abs(host(st.u) - ost.u).max() <= 1e-5 * u_scale, f"u {what}"


@pytest.mark.parametrize("n_itr", [1, 3])
@pytest.mark.parametrize("case", EDGE_CASES)
def test_edge_iterations_match_oracle(case, n_itr):
    P = require_gpu()
    import torch
    ny, nx, M, d, tile = case
    announce(f"edge iterate {case} n_itr={n_itr}")
    pb, wu, wv = _problem(ny, nx, M, d, seed=ny + nx + M)
    plan = P.Plan(nx, ny, wu, wv, pb.block_off, tile=tile)
    perm = plan.permutation()
    y = dev(pb.y[perm].astype(np.complex64), torch.complex64)
    U = dev(pb.U[perm], torch.float64)
    st = P.PPDState(plan, y)
    ost = O.init_state(ny, nx, pb.y)
    prm = O.Params(eta=pb.eta, mu=1.0, n_itr=n_itr)
    for T in (1, 3):
        O.iterate(pb.op, pb.y, pb.U, pb.eps, pb.block_off, prm, ost, T)
        s = P.ppd_iterate(plan, st, y, U, pb.eps, T, eta=pb.eta, mu=1.0, n_itr=n_itr)
        assert s["iter"] == ost.it
        _check(P, plan, st, ost, perm, f"after {ost.it}")


@pytest.mark.parametrize("n_itr", [1, 4])
def test_vanishing_radius_projects_onto_the_data(n_itr):
    """eps_j = 1e-30 ||y_j||: every projection onto the ball lands on y_j
    (the offset eps / r (q - y) is far below an ulp of y), so the
    Algorithm 2 iterate is the data bitwise after every iteration, and the
    iterates match the oracle run with the same radii.  A zero radius is
    rejected (eps must be > 0)."""
    P = require_gpu()
    import torch
    announce(f"edge vanishing radius n_itr={n_itr}")
    pb, wu, wv = _problem(32, 32, 3000, 3, seed=5)
    off = pb.block_off
    eps = np.array([1e-30 * np.linalg.norm(pb.y[off[j]:off[j + 1]]) for j in range(len(off) - 1)])
    plan = P.Plan(32, 32, wu, wv, off, tile=8)
    perm = plan.permutation()
    y = dev(pb.y[perm].astype(np.complex64), torch.complex64)
    U = dev(pb.U[perm], torch.float64)
    st = P.PPDState(plan, y)
    ost = O.init_state(32, 32, pb.y)
    O.iterate(pb.op, pb.y, pb.U, eps, off, O.Params(eta=pb.eta, mu=1.0, n_itr=n_itr), ost, 3)
    P.ppd_iterate(plan, st, y, U, eps, 3, eta=pb.eta, mu=1.0, n_itr=n_itr, stats=False)
    torch.cuda.synchronize()
    assert np.array_equal(ost.z, pb.y)
    assert np.array_equal(host(st.z), pb.y[perm])
    _check(P, plan, st, ost, perm, "vanishing radius")
    with pytest.raises(P.PPDError) as err:
        P.ppd_iterate(plan, st, y, U, np.zeros_like(eps), 1, eta=pb.eta)
    assert err.value.status == P.PPD_EINVAL
