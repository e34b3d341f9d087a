"""Write the FP64 oracle's trajectory for the ppd512 workload, the
configuration the benchmark is quoted on.

    python tests/golden/make_ppd512.py

512 x 512 image, 1.3M points on the radial 1/r coverage in 16 uneven blocks
(20k..200k), 30 dB input SNR; PPD (Algorithm 3, one Algorithm 2 iteration),
200 iterations from the zero state, statistics recorded every iteration:
SNR (Sec. 5), the relative change ||x_t - x_{t-1}|| / ||x_t||, ||x_t|| and
the block residuals ||Phi_j x~ - y_j|| of the stopping test.  The step size
eta = 1 / ||U^1/2 Phi||^2 comes from the oracle's own power iteration and is
stored with the trajectory, so the GPU run uses the same value.  Calls only
the oracle and the seeded input generators.  Output: ppd512_traj.json.
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import synth  # noqa: E402
from oracle import ppd as O  # noqa: E402
from oracle import problem as P  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def trajectory(inp, T: int, n_itr: int = 1, power_tol: float = 1e-7, power_max_iter: int = 300) -> dict:
    """T oracle PPD iterations on the problem of `inp`; returns the stored record."""
    w = inp.workload
    t0 = time.perf_counter()
    pb = P.problem_from_inputs(inp, with_eta=False)
    eta = 1.0 / P.power_norm(pb.op, pb.U, inp.power_start, power_tol, power_max_iter)
    print(f"{w.name}: problem and eta in {time.perf_counter() - t0:.1f} s", flush=True)
    st = O.init_state(w.n, w.n, pb.y)
    prm = O.Params(eta=eta, mu=1.0 / pb.U.max(), n_itr=n_itr)
    t0 = time.perf_counter()
    hist = O.iterate(pb.op, pb.y, pb.U, pb.eps, pb.block_off, prm, st, T, x_true=pb.x_true)
    print(f"{w.name}: {T} iterations in {time.perf_counter() - t0:.1f} s, final SNR {hist[-1]['snr']:.4f} dB",
          flush=True)
    return {"workload": w.name, "n": w.n, "M": int(pb.y.size), "iterations": T, "n_itr": n_itr,
            "eta": eta, "sigma": pb.sigma, "eps": pb.eps.tolist(),
            "snr_db": [h["snr"] for h in hist],
            "rel_change": [h["rel_change"] for h in hist],
            "x_norm": [h["x_norm"] for h in hist],
            "residual": [list(map(float, h["residual"])) for h in hist]}


def main(T: int = 200):
    out = trajectory(synth.make_inputs(synth.WORKLOADS["ppd512"]), T)
    with open(os.path.join(HERE, "ppd512_traj.json"), "w") as f:
        json.dump(out, f)


if __name__ == "__main__":
    main()
