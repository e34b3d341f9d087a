"""Write the FP64 oracle's trajectory for the 512 x 512 crop problem of the
ppd2048 workload.

    python tests/golden/make_crop2048.py

The crop problem keeps the central 512 x 512 part of the 2048 x 2048 sky and
a random 1/16 of each block's points (64 blocks, ~1.25M points), i.e. the
same visibilities per grid cell as the full 20M-point problem, small enough
for the oracle.  PPD with one Algorithm 2 iteration, 200 iterations,
statistics every iteration (as make_ppd512.py).  Calls only the oracle and
the seeded input generators.  Output: crop2048_traj.json.
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, HERE)

import synth  # noqa: E402
from make_ppd512 import trajectory  # noqa: E402

CROP_SEED = 901


def crop_inputs():
    """The crop problem's inputs (the GPU test builds the same ones)."""
    return synth.crop_inputs(synth.make_inputs(synth.WORKLOADS["ppd2048"]), 512, 16, seed=CROP_SEED)


def main(T: int = 200):
    out = trajectory(crop_inputs(), T)
    out["crop_seed"] = CROP_SEED
    with open(os.path.join(HERE, "crop2048_traj.json"), "w") as f:
        json.dump(out, f)


if __name__ == "__main__":
    main()
