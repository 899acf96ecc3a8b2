"""Write the FP64 oracle trajectories of the many-body sedimentation workload
(stored expected values for the error-growth comparison of the GPU's FP32,
FP16 and BF16 storage at full size).

Workload: D2Q9 2048x4096 closed box, tau = 0.55, g = (0, -2e-6), 350 disks
R = 8 and 150 ellipses 12x6 (seeded placement), K = 1.  Stored: every body's
centre X and measured velocity U every 100 steps up to --steps (the
workload's full 10000 by default), to 10 significant digits.  The run
resumes from --partial if interrupted (trajectory.py).

Calls only oracle/; writes tests/golden/sedimentation_2048x4096.json.
    python tests/golden/make_sedimentation_golden.py --partial DIR [--steps 10000]
"""
import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
sys.path.insert(0, HERE)

from paper_2511_01629_amd.workloads import workload  # noqa: E402  (inputs only)
from trajectory import rounded, run  # noqa: E402

NAME = "sedimentation_2048x4096"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=10000)
    ap.add_argument("--every", type=int, default=100)
    ap.add_argument("--save-every", type=int, default=1000)
    ap.add_argument("--partial", required=True, help="directory for the resumable record")
    ap.add_argument("--out", default=os.path.join(HERE, f"{NAME}.json"))
    args = ap.parse_args()
    cfg, parts, _, _ = workload(NAME)
    t0 = time.time()
    _, log = run(cfg, parts, args.steps, args.every, args.save_every, args.partial, 2)
    out = dict(workload=NAME, steps=args.steps, every=args.every, record_steps=log["record_steps"],
               X=rounded(log["X"]), U=rounded(log["U"]),
               note="FP64 oracle; X and U of every body after each recorded step, 10 significant digits")
    with open(args.out, "w") as f:
        json.dump(out, f)
    print("wrote", args.out, f"({time.time() - t0:.0f} s)")


if __name__ == "__main__":
    main()
