"""Write the FP64 oracle's SNR trajectories for the generalised-Gaussian
coverage workloads (Sec. 5.2: shape beta = 2, 0.5, 0.25 at 30 dB input SNR,
and beta = 0.25 at 50 dB).

    python tests/golden/make_ggd256.py

256 x 256 image, 65536 points, 4 blocks; PPD (one Algorithm 2 iteration)
and PD (U = 1), 300 iterations each, SNR recorded every iteration.  Calls
only the oracle and the seeded input generators (one process per
workload).  Output: ggd256_snr.json.
"""
import json
import os
import sys
from concurrent.futures import ProcessPoolExecutor

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import synth  # noqa: E402
from oracle import ppd as O  # noqa: E402
from oracle import problem as P  # noqa: E402

NAMES = ("ggd256_b2", "ggd256_b05", "ggd256_b025", "ggd256_b025_50db")


def run(name: str):
    w = synth.WORKLOADS[name]
    inp = synth.make_inputs(w)
    pb = P.problem_from_inputs(inp, power_tol=1e-9)
    out = {"workload": name, "iterations": w.iters, "beta": w.ggd_beta, "isnr_db": w.isnr_db,
           "eta_ppd": pb.eta, "eta_pd": pb.eta_pd, "eps": pb.eps.tolist(),
           "u_min": float(pb.U.min())}
    for method, U, eta in [("ppd", pb.U, pb.eta), ("pd", np.ones_like(pb.U), pb.eta_pd)]:
        st = O.init_state(w.n, w.n, pb.y)
        prm = O.Params(eta=eta, mu=1.0 / U.max(), n_itr=1)
        hist = O.iterate(pb.op, pb.y, U, pb.eps, pb.block_off, prm, st, w.iters, x_true=pb.x_true)
        out[method] = {"snr_db": [h["snr"] for h in hist]}
        print(name, method, "final SNR", hist[-1]["snr"], flush=True)
    return name, out


def main():
    with ProcessPoolExecutor(max_workers=len(NAMES)) as ex:
        res = dict(ex.map(run, NAMES))
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "ggd256_snr.json"), "w") as f:
        json.dump({k: res[k] for k in NAMES}, f)


if __name__ == "__main__":
    main()
