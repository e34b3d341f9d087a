"""The gridding-tile autotuner (tune.autotune): it times every candidate
(tile, chunk) plan by graph replay of one fused iteration, returns the
fastest, and caches the result per coverage and device, so that a second
call reads the cache instead of timing again; the plan it picks matches the
FP64 oracle like any other."""
import json

import numpy as np
import pytest

import synth
from oracle import ppd as O
from oracle import problem as oprob

from gpu_util import announce, assert_op_close, dev, host, require_gpu

pytestmark = pytest.mark.gpu


def test_autotune_picks_times_and_caches(tmp_path, monkeypatch):
    P = require_gpu()
    import torch
    from paper_1701_01748_amd import tune
    announce("autotune 64x64, three candidates")
    n, M = 64, 20000
    x, wu, wv, off = synth.small_case(n, M, seed=31, d=3)
    cache = str(tmp_path / "tune.json")
    cands = ((8, 128), (8, 256), (16, 512))
    stream = torch.cuda.Stream()
    best, timings = tune.autotune(n, n, wu, wv, off, stream, candidates=cands, cache=cache)
    assert best in cands and set(timings) == set(cands)
    assert all(np.isfinite(v) and v > 0 for v in timings.values())
    assert timings[best] == min(timings.values())
    with open(cache) as f:
        table = json.load(f)
    assert len(table) == 1 and tuple(next(iter(table.values()))["best"]) == best

    # a second call reads the cache: timing again would fail here
    def no_timing(plan, reps=20):
        raise AssertionError("cache not used")
    monkeypatch.setattr(tune, "time_iteration", no_timing)
    best2, timings2 = tune.autotune(n, n, wu, wv, off, stream, candidates=cands, cache=cache)
    assert best2 == best and timings2 == timings

    # the chosen decomposition computes the same iteration as the oracle
    pb = oprob.make_problem(x, wu, wv, off, synth.noise_unit(M, 231), 30.0, np.ones((n, n)), power_tol=1e-6)
    plan = P.Plan(n, n, wu, wv, off, tile=best[0], chunk=best[1])
    perm = plan.permutation()
    y = dev(pb.y[perm].astype(np.complex64), torch.complex64)
    st = P.PPDState(plan, y)
    P.ppd_iterate(plan, st, y, dev(pb.U[perm], torch.float64), pb.eps, 3, eta=pb.eta)
    ost = O.init_state(n, n, pb.y)
    O.iterate(pb.op, pb.y, pb.U, pb.eps, pb.block_off, O.Params(eta=pb.eta), ost, 3)
    assert_op_close(host(st.x), ost.x, what=f"x with tile {best[0]}, chunk {best[1]}")
