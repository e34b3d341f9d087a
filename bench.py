#!/usr/bin/env python3
"""Benchmark of the PPD hot path on one MI355X.

Workload (default): 512 x 512 image, M = 1.3M visibilities on a 1/r-dense
radial coverage in 16 uneven blocks (20k..200k), 30 dB input SNR, SARA with
3 levels, one Algorithm 2 sub-iteration.  A step is one full iteration of
Algorithm 3 (forward FFT, degridding with the fused dual update, gridding,
inverse FFT, SARA analysis + dual clip + synthesis, primal update), replayed
from a captured HIP graph or launched eagerly on two streams (both timed,
the faster is the value), inputs resident in HBM; the statistics (relative
change, SNR, block residuals) of every --stats-every-th (10th) iteration
are reduced on the device during the timed call, as a stopping test would,
and the call ends by reading back the last ones.

Prints one JSON line: PPD iterations/s (value), Phi / Phi^H visibilities/s,
the plain (unfused, per-block FP64) form for comparison, the roofline of the
dominant kernel (per-launch HIP events) and the FP64 oracle timed on the
host's cores on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "PPD iters/s + Phi/Phi^T vis/s at 512^2, M=1.3M; batched vs plain, HBM GB/s"
PREHEAT_S = 0.15   # minimum length of the untimed warm-up phase (seconds)
PREHEAT_CALL = 10  # iterations per call of that phase
HBM_PEAK_GBS = 8000.0
CRITICAL_PATH = ("fft_rows_fwd", "fft_cols_fwd", "degrid", "grid", "fold", "fft_cols_inv", "fft_rows_inv")
# kernel kind -> source file that defines it (traffic figures are only used
# while that file is unchanged since the counters were taken)
KIND_SOURCE = {"degrid": "nufft.hip", "grid": "nufft.hip", "fold": "nufft.hip",
               "fft_rows_fwd": "fft.hip", "fft_cols_fwd": "fft.hip", "fft_cols_inv": "fft.hip",
               "fft_rows_inv": "fft.hip", "dwt": "sara.hip", "idwt": "sara.hip", "subiter": "dual.hip"}


def source_sha(name: str) -> str:
    """Hash of a kernel source's code lines (comments and blank lines
    dropped, so that editing a comment keeps the recorded counters valid)."""
    import hashlib
    with open(os.path.join(ROOT, "paper_1701_01748_amd", "csrc", name)) as f:
        code = [ln.split("//", 1)[0].rstrip() for ln in f]
    return hashlib.sha1("\n".join(ln for ln in code if ln).encode()).hexdigest()[:12]


def measured_traffic(kind: str, workload: str, tile: int, chunk: int):
    """HBM bytes per launch of `kind` from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE scaled by the copy-kernel factors),
    or None if absent or taken on a different kernel source / configuration."""
    path = os.path.join(ROOT, "profiles", f"pmc_{workload}.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as f:
        for line in f:
            line = line.strip()
            if "=" in line and not line.startswith("#"):
                k, v = line.split("=", 1)
                vals[k.strip()] = v.strip()
    src = KIND_SOURCE.get(kind)
    if not src or vals.get(f"sha.{src}") != source_sha(src):
        return None
    if vals.get("tile") != str(tile) or vals.get("chunk") != str(chunk):
        return None
    try:
        fetch = float(vals[f"{kind}.fetch_kib"]) * float(vals["fetch_factor"])
        write = float(vals[f"{kind}.write_kib"]) * float(vals["write_factor"])
    except KeyError:
        return None
    return (fetch + write) * 1024.0


# kernel kind -> the kernel's name in a rocprofv3 summary (fused iteration, 8 x 8 tiles)
KIND_KERNEL = {"degrid": "k_degrid<8, true>", "grid": "k_grid_mfma<true>", "fold": "k_fold8",
               "fft_rows_fwd": "k_fft_rows_fwd", "fft_cols_fwd": "k_fft_cols_fwd", "fft_cols_inv": "k_fft_cols_inv",
               "fft_rows_inv": "k_fft_rows_inv<true, true>"}


def rocprof_avg_us(kind: str, workload: str, tile: int, chunk: int):
    """Average duration of the kernel of `kind` in the committed rocprofv3
    kernel statistics of this workload, or None if absent or taken on a
    different kernel source / configuration."""
    path = os.path.join(ROOT, "profiles", f"kernel_stats_{workload}.txt")
    name = KIND_KERNEL.get(kind)
    if not os.path.exists(path) or name is None or tile != 8:
        return None
    vals, avg = {}, None
    with open(path) as f:
        for line in f:
            t = line.strip()
            if t.startswith("#") or not t:
                continue
            if "=" in t and " " not in t.split("=", 1)[0]:
                k, v = t.split("=", 1)
                vals[k] = v
            elif t.startswith(name + " "):
                avg = float(t[len(name):].split()[1])
    src = KIND_SOURCE.get(kind)
    if not src or vals.get(f"sha.{src}") != source_sha(src) or vals.get("chunk") != str(chunk):
        return None
    return avg


def algorithmic_bytes(kind: str, M: int, N: int, K: int, ny: int, Kx: int) -> float:
    """Bytes each kernel kind must move per launch (fused PPD iteration)."""
    if kind == "degrid":      # omega 8, v 8, U 8, z 16, y 8 in; Theta G a 8 out; grid read once
        return 56.0 * M + 8.0 * K
    if kind == "grid":        # omega 8, Theta G a 8, z 16, U 8, y 8, v 8 in; z 16, v 8 out; grid written once
        return 80.0 * M + 8.0 * K
    if kind == "fft_rows_fwd":
        return 4.0 * N + 8.0 * ny * Kx
    if kind in ("fft_cols_fwd", "fft_cols_inv"):
        return 8.0 * ny * Kx + 8.0 * K
    if kind == "fft_rows_inv":  # half in; x, u~ in; x, x~ out
        return 8.0 * ny * Kx + 16.0 * N
    if kind == "zero":
        return 8.0 * K
    if kind == "dwt":          # per level on average: x / low-pass in, 9 duals read+written
        return (4.0 * N + 72.0 * N) / 3.0
    if kind == "idwt":
        return (36.0 * N + 4.0 * N) / 3.0
    return 0.0


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="ppd512")
    ap.add_argument("--n-itr", type=int, default=1)
    ap.add_argument("--stats-every", type=int, default=10,
                    help="the statistics (relative change, SNR, block residuals) of every this-many-th "
                         "iteration are reduced on the device during the timed call, as a stopping test")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=5)
    ap.add_argument("--quick", action="store_true", help="skip the secondary measurements (profiling runs)")
    ap.add_argument("--tile", type=int, default=0, help="gridding tile edge (0: library default)")
    ap.add_argument("--chunk", type=int, default=0, help="visibilities per work item (0: library default)")
    ap.add_argument("--autotune", action="store_true", help="pick tile / chunk by timing candidates first")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a 256 MiB device copy from an L2/MALL-evicted source (counter calibration)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this build measures one GPU; multi-GPU runs are not part of it "
              f"(asked for --gpus {args.gpus}, WORLD_SIZE={world})", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    from paper_1701_01748_amd import ppd as P

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    if args.calibrate_copy:
        nbytes = 256 << 20
        src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        sweep = torch.empty(1 << 28, dtype=torch.float32, device="cuda")   # 1 GiB
        sweep.fill_(2.0)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibration": "device copy", "bytes_read": nbytes, "bytes_written": nbytes}))
        return
    w = synth.WORKLOADS[args.workload]
    inp = synth.make_inputs(w)
    n = w.n
    wu, wv, off = inp.wu[0], inp.wv[0], inp.block_off
    M, N = w.M, n * n
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)
    tuned = None
    if args.autotune:
        from paper_1701_01748_amd import tune
        (args.tile, args.chunk), tuned = tune.autotune(n, n, wu, wv, off, stream)
    plan = P.Plan(n, n, wu, wv, off, stream=stream, tile=args.tile, chunk=args.chunk)
    info = plan.info
    K, Kx = info.Kx * info.Ky, info.Kx
    perm = plan.permutation()

    # ---- problem setup on the GPU (not timed) --------------------------------
    U = P.ppd_uniform_weights(plan)
    x_true = torch.as_tensor(inp.x_true.astype(np.float32)).cuda()
    y0 = P.ppd_phi(plan, x_true)
    sigma = math.sqrt(float((y0.abs().double() ** 2).sum()) / M * 10.0 ** (-w.isnr_db / 10.0))
    noise = torch.as_tensor(inp.noise[0][perm].astype(np.complex64)).cuda()
    y = (y0 + sigma * noise).contiguous()
    Mj = np.diff(off).astype(np.float64)
    eps = sigma * np.sqrt(Mj + 2.0 * np.sqrt(Mj))
    norm2, it_pow = P.ppd_op_norm(plan, U, torch.as_tensor(inp.power_start.astype(np.float32)).cuda(),
                                  300, 1e-7)
    eta = 1.0 / norm2
    kw = dict(eta=eta, tau=0.49, zeta=1.0, lam=1.0, alpha=1e-4, mu=1.0, n_itr=args.n_itr)
    state = P.PPDState(plan, y)

    # ---- timed region: the fused iteration, replayed from a HIP graph and
    # launched eagerly (two streams); the faster of the two is the value ----
    # The statistics (step a12: relative change, SNR, block residuals over
    # eps) are part of the step: those of every `stats_every`-th iteration are
    # reduced on the device during the call into a history, as a stopping
    # test would, and the call ends by reading back the last ones.
    every = max(1, args.stats_every)
    rows = max(args.steps, args.warmup, PREHEAT_CALL) // every
    hist = torch.zeros(rows * (8 + len(off) - 1), dtype=torch.float64, device="cuda")

    def timed(graph: bool):
        # arguments checked and marshalled once, outside the timed region, as
        # a serving loop would hold them
        it = P.Iteration(plan, state, y, U, eps, use_graph=graph, x_true=x_true, stats_every=every,
                         stats_history=hist, **kw)
        t_w = time.perf_counter()
        it.run(args.warmup)   # also captures the graphs
        torch.cuda.synchronize()
        # The GPU's clocks take tens of milliseconds of continuous work to
        # settle after idle (eight back-to-back 20-iteration calls measured
        # 149.5 -> 138.5 us per iteration; with 50 ms of idle before each
        # call, 150-153 us).  So that a short timed region measures the same
        # steady state as a long one, untimed iterations continue until the
        # warm-up phase has lasted PREHEAT_S; their count is reported.
        extra = 0
        while time.perf_counter() - t_w < PREHEAT_S:
            it.run(PREHEAT_CALL, stats=False)
            extra += PREHEAT_CALL
            torch.cuda.synchronize()
        preheat[graph] = extra
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record(stream)
        st = it.run(args.steps)
        e1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        # checked after the timed region: the copy of the history is not part of a step
        h = hist.view(-1, 8 + len(off) - 1)[: args.steps // every].cpu().numpy()
        assert np.isfinite(st["rel_change"]) and np.all(np.isfinite(h[:, :2]))
        return wall, e0.elapsed_time(e1)

    preheat = {}
    wall_g, ev_g = timed(True)
    wall_e, ev_e = timed(False)
    use_graph = wall_g <= wall_e
    wall_s, ev_ms = (wall_g, ev_g) if use_graph else (wall_e, ev_e)
    value = args.steps / wall_s
    st = P.ppd_iterate(plan, state, y, U, eps, 1, use_graph=use_graph, x_true=x_true, **kw)

    out = {
        "metric": METRIC, "value": round(value, 3), "unit": "PPD iterations/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(1000.0 * wall_s / args.steps, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "image": f"{n}x{n}", "M": M, "blocks": int(len(off) - 1),
                   "n_itr": args.n_itr, "levels": 3,
                   "form": "fused, hip graph" if use_graph else "fused, eager two-stream", "tile": info.tile,
                   "chunk": info.chunk},
        "stats_every": every,
        "event_ms_per_step": round(ev_ms / args.steps, 4),
        "graph_iters_per_s": round(args.steps / wall_g, 2), "eager_iters_per_s": round(args.steps / wall_e, 2),
        "preheat_iterations": {"graph": preheat[True], "eager": preheat[False], "seconds": PREHEAT_S},
        "snr_db_after": round(st["snr_db"], 3), "iterations_done": st["iter"],
        "residual_max_over_eps": round(st["residual_max"], 4),
        "op_norm_power_iters": it_pow,
    }

    # ---- per-kernel HIP events: eager pass of the same iteration ------------------
    n_prof = 10
    plan.timing(True)
    plan.timing_reset()
    P.ppd_iterate(plan, state, y, U, eps, n_prof, use_graph=False, x_true=x_true, **kw)
    tk = plan.timing_read()
    plan.timing(False)
    per_kind = {k: {"launches": c, "avg_us": round(1000.0 * ms / c, 3)} for k, (c, ms) in tk.items()}
    # dominant kernel: the largest total time on the data-fidelity chain, the
    # iteration's critical path (SARA runs beside it on a second stream, so
    # its event times include waiting for the shared compute units)
    dom = max((kv for kv in tk.items() if kv[0] in CRITICAL_PATH), key=lambda kv: kv[1][1])[0]
    cnt, ms = tk[dom]
    avg_s = ms / cnt / 1000.0
    algo = algorithmic_bytes(dom, M, N, K, n, Kx)
    achieved = algo / avg_s / 1e9
    out["kernels"] = per_kind
    traffic = measured_traffic(dom, args.workload, info.tile, info.chunk)
    rp = rocprof_avg_us(dom, args.workload, info.tile, info.chunk)
    out["roofline"] = {"kernel": dom, "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                       "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                       "traffic": None if traffic is None else round(traffic),
                       "algorithmic_bytes_per_launch": algo, "avg_launch_us": round(avg_s * 1e6, 3),
                       "rocprof_avg_us": rp,
                       "rocprof_frac": None if rp is None else round(algo / (rp * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)}
    if tuned:
        out["autotune_us_per_iteration"] = {f"tile{t}_chunk{c}": round(v, 1) for (t, c), v in tuned.items()}

    if not args.quick:
        # ---- Phi / Phi^H visibilities per second (plan order) ------------------------
        def time_calls(fn, reps=100):
            for _ in range(10):
                fn()
            ts = []
            for _ in range(reps):
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record(stream)
                fn()
                b.record(stream)
                torch.cuda.synchronize()
                ts.append(a.elapsed_time(b))
            return sorted(ts)[len(ts) // 2] / 1000.0

        yb = torch.empty(M, dtype=torch.complex64, device="cuda")
        xb = torch.empty((n, n), dtype=torch.float32, device="cuda")
        t_phi = time_calls(lambda: P.ppd_phi(plan, x_true, yb))
        t_phit = time_calls(lambda: P.ppd_phit(plan, y, xb))
        phi_bytes = 4.0 * N + 16.0 * M + 8.0 * n * Kx + 16.0 * K
        out["phi_vis_per_s"] = round(M / t_phi, 1)
        out["phit_vis_per_s"] = round(M / t_phit, 1)
        out["phi_us"] = round(t_phi * 1e6, 2)
        out["phit_us"] = round(t_phit * 1e6, 2)
        out["phi_algorithmic_GBps"] = round(phi_bytes / t_phi / 1e9, 1)
        out["phit_algorithmic_GBps"] = round(phi_bytes / t_phit / 1e9, 1)

        # ---- cold caches: a 1 GiB sweep (4x the 256 MB Infinity Cache) before
        # each timed call evicts every input of the call from the caches ------------
        sweep = torch.empty(1 << 28, dtype=torch.float32, device="cuda")

        def cold_and_warm(fn, reps=10):
            res = []
            for flush in (True, False):
                ts = []
                for k in range(reps):
                    if flush:
                        sweep.fill_(float(k))
                    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    a.record(stream)
                    fn()
                    b.record(stream)
                    torch.cuda.synchronize()
                    ts.append(a.elapsed_time(b))
                res.append(round(1000.0 * sorted(ts)[len(ts) // 2], 2))
            return res

        one = P.Iteration(plan, state.clone(), y, U, eps, use_graph=False, **kw)
        c_phi, w_phi = cold_and_warm(lambda: P.ppd_phi(plan, x_true, yb))
        c_phit, w_phit = cold_and_warm(lambda: P.ppd_phit(plan, y, xb))
        c_it, w_it = cold_and_warm(lambda: one.run(1, stats=False))
        out["cold"] = {"what": "median of 10 calls, each after a 1 GiB device sweep (us); warm: the same "
                               "calls back to back", "phi_us": c_phi, "phit_us": c_phit,
                       "iteration_call_us": c_it, "warm_phi_us": w_phi, "warm_phit_us": w_phit,
                       "warm_iteration_call_us": w_it}
        del sweep

        # ---- batched (fused) eager and plain per-block FP64 forms --------------------
        def iters_per_s(form, graph, T):
            # same statistics cadence as the headline
            s2 = state.clone()
            P.ppd_iterate(plan, s2, y, U, eps, 2, form=form, use_graph=graph, x_true=x_true, **kw)
            torch.cuda.synchronize()
            ta = time.perf_counter()
            P.ppd_iterate(plan, s2, y, U, eps, T, form=form, use_graph=graph, x_true=x_true, stats_every=every, **kw)
            torch.cuda.synchronize()
            return T / (time.perf_counter() - ta)

        out["plain_iters_per_s"] = round(iters_per_s(P.FORM_PLAIN, False, 20), 2)

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(inp, args.cpu_iters)
    print(json.dumps(out), flush=True)


def cpu_baseline(inp, iters: int) -> dict:
    """The FP64 oracle (untuned) timed on the host on a bounded sample:
    `iters` full PPD iterations of the same workload, setup excluded, with the
    sparse products split by rows over a thread pool and scipy.fft running
    on the same number of threads (at most the 16 cores a one-GPU machine
    shares); plus per-operator medians and the 64x64 workload's 200
    iterations end to end, and the 256^2 tracks workload's per-iteration
    median (n_itr = 5) with its 500-iteration run estimated from it."""
    import numpy as np

    import synth
    from oracle import nufft as onf
    from oracle import ppd as O
    from oracle import problem as oprob
    from oracle import prox as oprox
    from oracle import sara as osara

    workers = max(1, min(16, os.cpu_count() or 1))
    w = inp.workload
    wu, wv, off = inp.wu[0], inp.wv[0], inp.block_off
    op = onf.Nufft(wu, wv, w.n, w.n, workers=workers)
    y0 = op.phi(inp.x_true)
    sigma = math.sqrt(np.sum(np.abs(y0) ** 2) / w.M * 10.0 ** (-w.isnr_db / 10.0))
    y = (y0 + sigma * inp.noise[0]).astype(np.complex64).astype(np.complex128)
    U = oprob.uniform_weights(wu, wv, w.n, w.n)
    eps = oprob.l2_bounds(sigma, off)
    # the step size value does not change the arithmetic being timed
    prm = O.Params(eta=1e-3, mu=1.0, n_itr=1)
    st = O.init_state(w.n, w.n, y)
    O.iterate(op, y, U, eps, off, prm, st, 1)   # warm-up; leaves a non-trivial state

    def median_ms(fn, reps=3):
        fn()
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            fn()
            ts.append(time.perf_counter() - t0)
        return round(1e3 * sorted(ts)[len(ts) // 2], 2)

    wv_arg = st.v / U + op.degrid(op.fft_grid(st.xt))

    def alg2_step():
        for j in range(off.size - 1):
            s_ = slice(int(off[j]), int(off[j + 1]))
            oprox.fb_ellipsoid(wv_arg[s_], y[s_], eps[j], U[s_], 1.0, 1, st.z[s_])

    img, ut = op.phit(st.v), osara.synthesis(st.u, 3)

    def primal_update(img, ut):
        xbar = oprox.proj_C(st.x - prm.tau * (prm.eta * img + prm.zeta * ut))
        return st.x + prm.lam * (xbar - st.x), 2.0 * xbar - st.x

    ops = {"phi_ms": median_ms(lambda: op.phi(st.xt)), "phit_ms": median_ms(lambda: op.phit(st.v)),
           "sara_analysis_ms": median_ms(lambda: osara.analysis(st.xt, 3)),
           "sara_synthesis_ms": median_ms(lambda: osara.synthesis(st.u, 3)),
           "alg2_step_ms": median_ms(alg2_step),
           "primal_update_ms": median_ms(lambda: primal_update(img, ut))}
    t0 = time.perf_counter()
    O.iterate(op, y, U, eps, off, prm, st, iters)
    dt = time.perf_counter() - t0
    # the 64x64 workload end to end (200 iterations, problem setup excluded)
    w64 = synth.WORKLOADS["ppd64"]
    i64 = synth.make_inputs(w64)
    pb64 = oprob.problem_from_inputs(i64, with_eta=False)
    s64 = O.init_state(64, 64, pb64.y)
    t1 = time.perf_counter()
    O.iterate(pb64.op, pb64.y, pb64.U, pb64.eps, pb64.block_off, O.Params(eta=1e-3), s64, 200)
    ops["ppd64_200_iterations_s"] = round(time.perf_counter() - t1, 3)
    # the 256^2 tracks workload (4 blocks, n_itr = 5 as in its PD / PPD
    # comparison): median of 5 iterations, and that times its 500 iterations
    w256 = synth.WORKLOADS["tracks256"]
    i256 = synth.make_inputs(w256)
    pb256 = oprob.problem_from_inputs(i256, with_eta=False)
    s256 = O.init_state(w256.n, w256.n, pb256.y)
    p256 = O.Params(eta=1e-3, mu=1.0 / pb256.U.max(), n_itr=5)

    def one256():
        O.iterate(pb256.op, pb256.y, pb256.U, pb256.eps, pb256.block_off, p256, s256, 1)

    it256 = median_ms(one256, reps=5)
    ops["tracks256_iteration_ms"] = it256
    ops["tracks256_500_iterations_s_estimate"] = round(500 * it256 / 1e3, 1)
    return {"value": round(iters / dt, 5), "unit": "PPD iterations/s", "cores": workers, "kind": "oracle",
            "host_cpus": os.cpu_count(), "per_operator": ops,
            "sample": f"{iters} full FP64 oracle iterations of {w.name} (setup excluded), {dt:.1f} s; sparse "
                      f"products split by rows over {workers} threads and scipy.fft with {workers} workers; "
                      "SARA, Algorithm 2 and the primal update single-threaded NumPy; per-operator medians of 3"}


if __name__ == "__main__":
    main()
