"""Write the FP64 oracle trajectories of a 3D sphere-settling workload
(stored expected values for the error-growth comparison of the GPU's FP32
and FP16 storage).

Workloads (paper_2511_01629_amd.workloads): spheres_256x256x512 (D3Q19
256x256x512 closed box, tau = 0.6, g = (0, 0, -1e-5), 64 spheres R = 8,
seeded placement in the upper half, densities in [1.2, 1.8], K = 1) and
spheres_64x64x128 (the same fluid, spheres and gravity, 8 spheres in a box
1/64 of the volume).  Stored: every sphere's centre X and measured velocity U
every --every steps up to --steps, to 10 significant digits, and the fluid
velocity on a fixed seeded sample of nodes after the last step.  The run
resumes from --partial if interrupted (trajectory.py); a later call with a
larger --steps continues the same record.

Calls only oracle/; writes tests/golden/<name>.json.
    python tests/golden/make_spheres_golden.py --partial DIR [--name NAME] [--steps 5000]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
sys.path.insert(0, HERE)

from paper_2511_01629_amd.workloads import workload  # noqa: E402  (inputs only)
from trajectory import rounded, run  # noqa: E402

N_SAMPLE = 4096  # fluid-velocity sample nodes (seeded, fixed)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--name", default="spheres_256x256x512", choices=["spheres_256x256x512", "spheres_64x64x128"])
    ap.add_argument("--steps", type=int, default=5000)
    ap.add_argument("--every", type=int, default=100)
    ap.add_argument("--save-every", type=int, default=500)
    ap.add_argument("--partial", required=True, help="directory for the resumable record")
    ap.add_argument("--out", default=None)
    args = ap.parse_args()
    NAME = args.name
    out_path = args.out or os.path.join(HERE, f"{NAME}.json")
    cfg, parts, _, _ = workload(NAME)
    t0 = time.time()
    o, log = run(cfg, parts, args.steps, args.every, args.save_every, args.partial, 3)
    u, _, _ = o.fields()
    N = int(np.prod(cfg["n"]))
    nodes = np.sort(np.random.default_rng(5000).choice(N, min(N_SAMPLE, N), replace=False))
    uf = u.reshape(N, 3)
    out = dict(workload=NAME, steps=args.steps, every=args.every, record_steps=log["record_steps"],
               X=rounded(log["X"]), U=rounded(log["U"]), nodes=nodes.tolist(),
               u_nodes=[[float(f"{v:.10g}") for v in row] for row in uf[nodes]],
               u_max=float(np.abs(uf).max()),
               note="FP64 oracle; X and U of every sphere after each recorded step, fluid u on sampled "
                    "nodes after the last step, 10 significant digits")
    with open(out_path, "w") as f:
        json.dump(out, f)
    print("wrote", out_path, f"({time.time() - t0:.0f} s)")


if __name__ == "__main__":
    main()
