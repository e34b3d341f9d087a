"""Write the FP64 oracle's SNR trajectories for the tracks256 workload.

    python tests/golden/make_tracks256.py

256 x 256 image, 65536 points on 36 elliptical tracks, blocks of 8000, 12000,
20000 and 25536 points, 30 dB input SNR; PPD with 5 Algorithm 2 iterations
(Sec. 5.1 uses 1, 5 and 50), PPD with 50, and PD (U = 1), 500 iterations
each.  Calls only the oracle and the seeded input generators.  Output:
tracks256_snr.json (keys "ppd", "ppd_nitr50" and "pd").
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import synth  # noqa: E402
from oracle import ppd as O  # noqa: E402
from oracle import problem as P  # noqa: E402


def main(T: int = 500):
    w = synth.WORKLOADS["tracks256"]
    inp = synth.make_inputs(w)
    pb = P.problem_from_inputs(inp, power_tol=1e-9)
    out = {"workload": w.name, "iterations": T, "n_itr": w.n_itr, "eta_ppd": pb.eta, "eta_pd": pb.eta_pd,
           "sigma": pb.sigma, "eps": pb.eps.tolist()}
    runs = [("ppd", pb.U, pb.eta, w.n_itr), ("pd", np.ones_like(pb.U), pb.eta_pd, 1),
            ("ppd_nitr50", pb.U, pb.eta, 50)]
    for name, U, eta, n_itr in runs:
        st = O.init_state(w.n, w.n, pb.y)
        prm = O.Params(eta=eta, mu=1.0 / U.max(), n_itr=n_itr)
        hist = O.iterate(pb.op, pb.y, U, pb.eps, pb.block_off, prm, st, T, x_true=pb.x_true)
        out[name] = {"snr_db": [h["snr"] for h in hist],
                     "residual_over_eps_final": (np.array(hist[-1]["residual"]) / pb.eps).tolist(),
                     "n_itr": prm.n_itr}
        print(name, "final SNR", hist[-1]["snr"], flush=True)
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "tracks256_snr.json"), "w") as f:
        json.dump(out, f)


if __name__ == "__main__":
    main()
