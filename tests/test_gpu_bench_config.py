"""The benchmark's own workload at full size and in its launch
configuration: 512^2 image, 1.3M visibilities in 16 uneven blocks, plan
defaults (8 x 8 tiles, 128-point items), one Algorithm 2 step per iteration.
Fused iterations, first launched eagerly on the two streams and then
replayed from a HIP graph, are compared element by element with the FP64
oracle (Algorithm 3)."""
import numpy as np
import pytest

import synth
from oracle import ppd as O
from oracle import problem as oprob
from oracle import sara as osara

from gpu_util import announce, assert_op_close, dev, host, require_gpu

pytestmark = pytest.mark.gpu


def test_ppd512_bench_configuration_matches_oracle():
    P = require_gpu()
    import torch
    announce("ppd512 full size, plan defaults, eager then graph")
    inp = synth.make_inputs(synth.WORKLOADS["ppd512"])
    n = inp.workload.n
    pb = oprob.problem_from_inputs(inp, with_eta=False)
    # a step size from a few oracle power iterations: parity does not depend
    # on its exact value, only on both sides using the same one
    eta = 1.0 / oprob.power_norm(pb.op, pb.U, inp.power_start, tol=1e-3, max_iter=10)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        plan = P.Plan(n, n, inp.wu[0], inp.wv[0], inp.block_off, stream=stream)
        assert (plan.info.tile, plan.info.chunk) == (8, 128)
        perm = plan.permutation()
        y = dev(pb.y[perm].astype(np.complex64), torch.complex64)
        U = dev(pb.U[perm], torch.float64)
        st = P.PPDState(plan, y)
        ost = O.init_state(n, n, pb.y)
        prm = O.Params(eta=eta, mu=1.0, n_itr=1)
        for graph in (False, True):
            O.iterate(pb.op, pb.y, pb.U, pb.eps, pb.block_off, prm, ost, 2)
            s = P.ppd_iterate(plan, st, y, U, pb.eps, 2, eta=eta, mu=1.0, n_itr=1, use_graph=graph)
            stream.synchronize()
            assert s["iter"] == ost.it
            mode = "graph" if graph else "eager"
            assert_op_close(host(st.x), ost.x, what=f"x after {ost.it} ({mode})")
            assert_op_close(host(st.xt), ost.xt, what=f"x tilde after {ost.it} ({mode})")
            assert_op_close(host(st.v), ost.v[perm], what=f"v after {ost.it} ({mode})")
            assert_op_close(host(st.z), ost.z[perm], what=f"z after {ost.it} ({mode})")
            u_scale = np.abs(osara.analysis(ost.xt)).max()
            du = np.abs(host(st.u) - ost.u).max()
            assert du <= 1e-5 * u_scale, f"u after {ost.it} ({mode}): {du:.3e} vs scale {u_scale:.3e}"
