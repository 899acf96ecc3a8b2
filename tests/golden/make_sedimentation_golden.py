"""Write the FP64 oracle trajectories of the many-body sedimentation workload
(stored expected values for the error-growth comparison of the GPU's FP32,
FP16 and BF16 storage at full size).

Workload: D2Q9 2048x4096 closed box, tau = 0.55, g = (0, -2e-6), 350 disks
R = 8 and 150 ellipses 12x6 (seeded placement), K = 1.  Stored: every body's
centre X and measured velocity U every 100 steps up to --steps, to 10
significant digits.

Calls only oracle/; writes tests/golden/sedimentation_2048x4096.json.
    python tests/golden/make_sedimentation_golden.py [--steps 4000]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_2511_01629_amd.workloads import workload  # noqa: E402  (inputs only)

NAME = "sedimentation_2048x4096"


def _round(rows):
    """10 significant digits: far below the reduced-precision errors compared
    against, and half the size of full FP64 text."""
    return [[[float(f"{v:.10g}") for v in body] for body in row] for row in rows]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=4000)
    ap.add_argument("--every", type=int, default=100)
    ap.add_argument("--out", default=os.path.join(os.path.dirname(os.path.abspath(__file__)), f"{NAME}.json"))
    args = ap.parse_args()
    cfg, parts, _, _ = workload(NAME)
    t0 = time.time()
    o = O.Oracle(cfg, parts)
    X, U, steps = [], [], []
    done = 0
    while done < args.steps:
        n = min(args.every, args.steps - done)
        r = o.step(n, record=True)
        done += n
        steps.append(done)
        X.append(r[-1, :, 0:2].tolist())
        U.append(r[-1, :, 4:6].tolist())
        print(f"{done} steps ({time.time() - t0:.0f} s)", flush=True)
    out = dict(workload=NAME, steps=args.steps, every=args.every, record_steps=steps, X=_round(X), U=_round(U),
               note="FP64 oracle; X and U of every body after each recorded step, 10 significant digits")
    with open(args.out, "w") as f:
        json.dump(out, f)
    print("wrote", args.out, f"({time.time() - t0:.0f} s)")


if __name__ == "__main__":
    main()
