"""Several frequency channels of one sky solved together (the batched form):
each channel's coverage is the base coverage scaled by nu / nu0, and its
visibilities become blocks of one plan, so one iteration runs every
channel's and every block's dual update, Algorithm 2's middle steps of all
of them in one persistent launch, and one gridding into the common image.
Iterates against the FP64 oracle run on the same stacked problem (the
oracle takes the blocks as they come), eagerly and replayed from a graph."""
import math

import numpy as np
import pytest

import synth
from oracle import ppd as O
from oracle import problem as oprob
from oracle import sara as osara

from gpu_util import announce, assert_op_close, dev, host, require_gpu

pytestmark = pytest.mark.gpu


def _stacked(n=64, M=3000, d=2, n_chan=4, seed=7):
    x = synth.sky(n, seed=seed)
    wu, wv = synth.coverage_radial(M, seed=100 + seed, rmax=math.pi / 1.1)
    sizes = synth.block_sizes_loguniform(M, d, M // (4 * d), 4 * M // d, 300 + seed)
    wu, wv, off, _ = synth.radial_blocks(wu, wv, sizes)
    us, vs, offs, noise = [], [], [0], []
    for c, f in enumerate(np.linspace(0.9, 1.1, n_chan)):
        u, v = synth._to_f32_coverage(wu.astype(np.float64) * f, wv.astype(np.float64) * f)
        us.append(u)
        vs.append(v)
        offs.extend(int(o) + c * M for o in off[1:])
        noise.append(synth.noise_unit(M, 200 + seed + 1000 * c))
    return x, np.concatenate(us), np.concatenate(vs), np.array(offs, np.int64), np.concatenate(noise)


@pytest.mark.parametrize("graph", [False, True])
def test_stacked_channels_match_oracle(graph):
    P = require_gpu()
    import torch
    announce(f"stacked channels as blocks, n_itr=3, graph={graph}")
    x, wu, wv, off, noise = _stacked()
    n = x.shape[0]
    pb = oprob.make_problem(x, wu, wv, off, noise, 30.0, np.ones((n, n)), power_tol=1e-8)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        plan = P.Plan(n, n, wu, wv, off, stream=stream)
        assert plan.d == 8 and plan.info.persistent == 1
        perm = plan.permutation()
        y = dev(pb.y[perm].astype(np.complex64), torch.complex64)
        U = dev(pb.U[perm], torch.float64)
        st = P.PPDState(plan, y)
        ost = O.init_state(n, n, pb.y)
        prm = O.Params(eta=pb.eta, mu=1.0, n_itr=3)
        for T in (2, 3):
            O.iterate(pb.op, pb.y, pb.U, pb.eps, off, prm, ost, T)
            s = P.ppd_iterate(plan, st, y, U, pb.eps, T, eta=pb.eta, mu=1.0, n_itr=3, use_graph=graph)
            stream.synchronize()
            assert s["iter"] == ost.it
            assert_op_close(host(st.x), ost.x, what=f"x after {ost.it}")
            assert_op_close(host(st.v), ost.v[perm], what=f"v after {ost.it}")
            assert_op_close(host(st.z), ost.z[perm], what=f"z after {ost.it}")
            u_scale = np.abs(osara.analysis(ost.xt)).max()
            assert np.abs(host(st.u) - ost.u).max() <= 1e-5 * u_scale
