"""The benchmark's own workload at full size and in its launch
configuration: 512^2 image, 1.3M visibilities in 16 uneven blocks, plan
defaults (8 x 8 tiles, 128-point items), one Algorithm 2 step per iteration.

* Fused iterations, first launched eagerly on the two streams and then
  replayed from a HIP graph, element by element against the FP64 oracle
  (Algorithm 3), with the statistics of every iteration against the
  oracle's records.
* The error of every result against the FP64 oracle, reported per result
  (Phi, Phi^H, SARA analysis and synthesis, and x, x~, v, z, u, SNR after
  two iterations of the fused and of the plain per-block FP64 form).
* 200 iterations (the length the reconstruction SNR bar is stated for)
  against the oracle's stored trajectory (tests/golden/make_ppd512.py): SNR
  within 0.05 dB every 25 iterations, eagerly and replayed from a graph,
  with the statistics reduced on the device every 25 iterations as in the
  benchmark."""
import json
import os

import numpy as np
import pytest

import synth
from oracle import ppd as O
from oracle import problem as oprob
from oracle import sara as osara

from gpu_util import announce, assert_op_close, check_stats, check_trajectory, dev, host, require_gpu

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "ppd512_traj.json")
_CACHE = {}


def _problem():
    """The ppd512 inputs and the oracle's problem (built once per module)."""
    if "pb" not in _CACHE:
        inp = synth.make_inputs(synth.WORKLOADS["ppd512"])
        _CACHE["inp"] = inp
        _CACHE["pb"] = oprob.problem_from_inputs(inp, with_eta=False)
    return _CACHE["inp"], _CACHE["pb"]


def test_ppd512_bench_configuration_matches_oracle():
    P = require_gpu()
    import torch
    announce("ppd512 full size, plan defaults, eager then graph")
    inp, pb = _problem()
    n = inp.workload.n
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
        xt = dev(pb.x_true.astype(np.float32), torch.float32)
        st = P.PPDState(plan, y)
        ost = O.init_state(n, n, pb.y)
        prm = O.Params(eta=eta, mu=1.0, n_itr=1)
        for graph in (False, True):
            recs = O.iterate(pb.op, pb.y, pb.U, pb.eps, pb.block_off, prm, ost, 2, x_true=pb.x_true)
            hist = torch.zeros(2 * (8 + plan.d), dtype=torch.float64, device="cuda")
            s = P.ppd_iterate(plan, st, y, U, pb.eps, 2, eta=eta, mu=1.0, n_itr=1, use_graph=graph, x_true=xt,
                              stats_every=1, stats_history=hist)
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
            check_stats(host(hist).reshape(2, 8 + plan.d), recs, pb.y, pb.block_off, pb.eps, f"ppd512 {mode}")


@pytest.mark.parametrize("graph", [False, True])
def test_ppd512_200_iterations_vs_oracle_trajectory(graph):
    P = require_gpu()
    import torch
    if not os.path.exists(GOLDEN):
        pytest.fail("missing golden file: run tests/golden/make_ppd512.py")
    with open(GOLDEN) as f:
        ref = json.load(f)
    announce(f"ppd512 200 iterations vs oracle trajectory graph={graph}")
    inp, pb = _problem()
    assert np.allclose(pb.eps, ref["eps"], rtol=1e-12) and ref["M"] == pb.y.size
    n = inp.workload.n
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        plan = P.Plan(n, n, inp.wu[0], inp.wv[0], inp.block_off, stream=stream)
        check_trajectory(P, plan, pb, plan.permutation(), ref, graph, f"ppd512 graph={graph}")


def test_ppd512_precision_report():
    """Relative (norm) and peak-relative error of each result against the
    FP64 oracle at the benchmark's size, printed as one table; every entry
    within the parity bar (1e-5; u against its coefficient scale)."""
    P = require_gpu()
    import torch
    announce("ppd512 precision report")
    inp, pb = _problem()
    n = inp.workload.n
    eta = 1.0 / oprob.power_norm(pb.op, pb.U, inp.power_start, tol=1e-3, max_iter=10)
    rows = []

    def row(name, gpu, ref, bar=1e-5, scale=None):
        g, r = np.asarray(gpu, np.complex128 if np.iscomplexobj(gpu) else np.float64), np.asarray(ref)
        rel = float(np.linalg.norm((g - r).ravel()) / max(np.linalg.norm(r.ravel()), 1e-300))
        peak = float(np.abs(g - r).max() / (scale if scale is not None else max(np.abs(r).max(), 1e-300)))
        rows.append((name, rel, peak))
        assert peak <= bar and (scale is not None or rel <= bar), (name, rel, peak)

    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        plan = P.Plan(n, n, inp.wu[0], inp.wv[0], inp.block_off, stream=stream)
        perm = plan.permutation()
        x32 = pb.x_true.astype(np.float32)
        yg = host(P.ppd_phi(plan, dev(x32, torch.float32)))
        row("Phi x", yg, pb.op.phi(x32.astype(np.float64))[perm])
        y32 = pb.y.astype(np.complex64)
        yd = dev(y32[perm], torch.complex64)
        row("Phi^H y", host(P.ppd_phit(plan, yd)), pb.op.phit(y32.astype(np.complex128)))
        c = host(P.ppd_sara(plan, P.SARA_ANALYSIS, dev(x32, torch.float32)))
        row("Psi^H x", c, osara.analysis(x32.astype(np.float64)))
        row("Psi c", host(P.ppd_sara(plan, P.SARA_SYNTHESIS, dev(c, torch.float32))),
            osara.synthesis(c.astype(np.float64)))
        U = dev(pb.U[perm], torch.float64)
        xt_dev = dev(x32, torch.float32)
        ost = O.init_state(n, n, pb.y)
        recs = O.iterate(pb.op, pb.y, pb.U, pb.eps, pb.block_off, O.Params(eta=eta, mu=1.0), ost, 2,
                         x_true=pb.x_true)
        u_scale = np.abs(osara.analysis(ost.xt)).max()
        for form, fname in ((P.FORM_FUSED, "fused"), (P.FORM_PLAIN, "plain")):
            st = P.PPDState(plan, yd)
            s = P.ppd_iterate(plan, st, yd, U, pb.eps, 2, eta=eta, mu=1.0, form=form, x_true=xt_dev)
            stream.synchronize()
            row(f"x ({fname})", host(st.x), ost.x)
            row(f"x~ ({fname})", host(st.xt), ost.xt)
            row(f"v ({fname})", host(st.v), ost.v[perm])
            row(f"z ({fname})", host(st.z), ost.z[perm])
            row(f"u ({fname}, peak over coefficient scale)", host(st.u), ost.u, scale=u_scale)
            d_snr = abs(s["snr_db"] - recs[-1]["snr"])
            rows.append((f"SNR dB ({fname}, absolute)", d_snr, d_snr))
            assert d_snr <= 0.05
    lines = [f"{name:42s} {rel:10.2e} {peak:10.2e}" for name, rel, peak in rows]
    print("[precision] ppd512, error against the FP64 oracle (relative norm, peak-relative):\n" +
          "\n".join(lines), flush=True)


def test_bench_line_with_fewer_steps_than_the_statistics_period():
    """bench.py's one JSON line, in a child process, for a run shorter than
    the statistics period and than one call of the untimed warm-up phase
    (3 timed steps, 1 warm-up step): the keys of the line's contract and a
    positive value."""
    import subprocess
    import sys
    announce("bench.py --steps 3 --warmup 1")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--steps", "3", "--warmup", "1", "--quick",
                        "--no-cpu-baseline"], capture_output=True, text=True, timeout=300, cwd=root)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [ln for ln in r.stdout.splitlines() if ln.startswith("{")]
    assert len(lines) == 1, r.stdout[-2000:]
    d = json.loads(lines[0])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
              "vs_baseline", "dtype", "data", "config", "roofline"):
        assert k in d, k
    assert d["steps"] == 3 and d["warmup"] == 1 and d["n_gpus"] == 1
    assert d["value"] > 0 and d["config"]["workload"] == "ppd512"
