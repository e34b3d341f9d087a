"""Helpers shared by the GPU parity tests (no method arithmetic)."""
import sys

import numpy as np
import pytest


def require_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    from paper_1701_01748_amd import ppd
    ppd.lib()
    return ppd


def announce(msg: str):
    """Name the GPU case before it runs (flushed, in case the device faults)."""
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def dev(a, dtype):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def host(t):
    return t.detach().cpu().numpy()


def rel_err(a, b) -> float:
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def peak_err(a, b) -> float:
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


# Operator outputs (float32 path against the float64 oracle): norm-wise and
# peak-relative element-wise bound of the stated parity tolerance.
OP_TOL = 1e-5


def assert_op_close(gpu, ref, tol=OP_TOL, what=""):
    r, p = rel_err(gpu, ref), peak_err(gpu, ref)
    assert r <= tol and p <= tol, f"{what}: rel {r:.3e}, peak-rel {p:.3e} > {tol:g}"


def check_stats(rows, recs, y, block_off, eps, what: str):
    """rows: GPU history rows [8 + d] (one per iteration); recs: oracle records."""
    assert len(rows) == len(recs)
    yj = np.array([np.linalg.norm(y[block_off[j]:block_off[j + 1]]) for j in range(len(eps))])
    worst = {"rel": 0.0, "xn": 0.0, "r": 0.0, "snr": 0.0}
    for t, (h, rec) in enumerate(zip(rows, recs)):
        rel, xn, snr, rmax = h[0], h[1], h[2], h[3]
        r = h[8:]
        ro = np.asarray(rec["residual"])
        d_rel = abs(rel - rec["rel_change"])
        assert d_rel <= 3e-5 + 1e-5 * rec["rel_change"], (what, t + 1, "rel_change", rel, rec["rel_change"])
        d_xn = abs(xn - rec["x_norm"])
        assert d_xn <= 1e-5 * rec["x_norm"], (what, t + 1, "x_norm", xn, rec["x_norm"])
        bound = 1e-5 * (yj + ro)
        assert np.all(np.abs(r - ro) <= bound), (what, t + 1, "residual", r, ro)
        assert abs(rmax - np.max(ro / eps)) <= np.max(bound / eps), (what, t + 1, "residual_max", rmax)
        assert abs(snr - rec["snr"]) <= 0.05, (what, t + 1, "snr", snr, rec["snr"])
        worst["rel"] = max(worst["rel"], d_rel)
        worst["xn"] = max(worst["xn"], d_xn / rec["x_norm"])
        worst["r"] = max(worst["r"], float(np.max(np.abs(r - ro) / (yj + ro))))
        worst["snr"] = max(worst["snr"], abs(snr - rec["snr"]))
    print(f"[stats] {what}: max |d rel_change| {worst['rel']:.2e}, max rel d||x|| {worst['xn']:.2e}, "
          f"max |d r_j|/(||y_j|| + r_j) {worst['r']:.2e}, max |d SNR| {worst['snr']:.2e} dB", flush=True)


def check_trajectory(P, plan, pb, perm, ref, graph: bool, what: str, every: int = 25):
    """ref["iterations"] fused iterations from the zero state with the
    oracle's step size; statistics of every `every`-th iteration reduced on
    the device into a history; SNR within 0.05 dB of the oracle's at each."""
    import torch
    T = ref["iterations"]
    d = plan.d
    y = dev(pb.y[perm].astype(np.complex64), torch.complex64)
    U = dev(pb.U[perm], torch.float64)
    xt = dev(pb.x_true.astype(np.float32), torch.float32)
    st = P.PPDState(plan, y)
    hist = torch.zeros((T // every) * (8 + d), dtype=torch.float64, device="cuda")
    P.ppd_iterate(plan, st, y, U, pb.eps, T, eta=ref["eta"], mu=1.0 / pb.U.max(), n_itr=ref["n_itr"],
                  x_true=xt, use_graph=graph, stats_every=every, stats_history=hist)
    torch.cuda.synchronize()
    h = host(hist).reshape(T // every, 8 + d)
    yj = np.array([np.linalg.norm(pb.y[pb.block_off[j]:pb.block_off[j + 1]]) for j in range(d)])
    lines = []
    for k in range(T // every):
        t = (k + 1) * every - 1
        snr_o = ref["snr_db"][t]
        assert abs(h[k, 2] - snr_o) <= 0.05, (what, t + 1, h[k, 2], snr_o)
        # the residuals of the stopping test: the iterates drift apart by at
        # most ~1e-3 relative over 200 float32 iterations
        ro = np.asarray(ref["residual"][t])
        assert np.all(np.abs(h[k, 8:] - ro) <= 1e-3 * (yj + ro)), (what, t + 1, h[k, 8:], ro)
        lines.append(f"{t + 1}:{h[k, 2]:.3f}/{snr_o:.3f}")
    print(f"[trajectory] {what}: SNR GPU/oracle " + " ".join(lines), flush=True)
    return st
