"""Write the oracle gradient of the differentiated workload (stored expected values).

Workload: 512x1024 D2Q9 closed box, tau = 0.7, |g| = 1e-5 along -y, 16 disks
of radius 10 (seeded placement, densities in [1.2, 1.6]), 5000 steps.
Loss: L = (1/16) sum_i Y_i after the last step (the mean final height).
Parameters: the 16 densities rho_s, tau (alpha = 1/tau follows it) and |g|.

Two oracle gradients, both FP64 and both with the indicator sequence of the
base run (a binary indicator makes L piecewise smooth; the derivative is the
one of the step map with the indicator frozen):
  * complex step, for every parameter: one run of the complex-valued oracle
    with an imaginary perturbation 1e-30 (exact to rounding);
  * central differences with h_k = 1e-6 |theta_k|, the indicator replayed from
    the centres and orientations recorded in the base run, for every
    parameter (--fd all, the default, or a comma-separated subset): two real
    runs per parameter, an independent check of the complex step.

--cs-from takes the complex-step values of an earlier output of this script
instead of recomputing them (they do not depend on the central differences).

Each parameter is one job, run in a child process, whose result is kept in
--partial so that an interrupted run resumes where it stopped.

Calls only oracle/; writes tests/golden/adjoint_512x1024_grad.json.
    python tests/golden/make_adjoint_golden.py --partial DIR [--jobs 3 --threads 2]
        [--cs-from tests/golden/adjoint_512x1024_grad.json]
"""
import argparse
import json
import os
import subprocess
import sys
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

NAME = "adjoint_512x1024"
FD_DEFAULT = "all"


def _setup():
    from paper_2511_01629_amd.workloads import workload  # inputs only

    cfg, parts, _, _ = workload(NAME)
    gmag = float(np.linalg.norm(cfg["g"]))
    names = [f"rho_s[{i}]" for i in range(len(parts))] + ["tau", "gmag"]
    values = [p["rho_s"] for p in parts] + [cfg["tau"], gmag]
    return cfg, parts, gmag, names, values


def _mean_height(o, imag=False):
    return float(o.particles(imag=imag)["X"][:, 1].mean())


def run_one(k, steps, partial, do_fd, cs_from=None):
    """Complex-step (and optionally central-difference) derivative for parameter k."""
    from oracle import oracle as O

    cfg, parts, gmag, names, values = _setup()
    name, npart = names[k], len(parts)
    seed = dict(d_rho_s=[0.0] * npart, d_tau=0.0, d_gmag=0.0, h=1e-30)
    if k < npart:
        seed["d_rho_s"][k] = 1.0
    elif name == "tau":
        seed["d_tau"] = 1.0
    else:
        seed["d_gmag"] = 1.0
    t0 = time.time()
    if cs_from:
        prev = json.load(open(cs_from))
        assert prev["steps"] == steps and prev["params"][k] == name
        cs = prev["grad_complex_step"][k]
    else:
        oc = O.Oracle(cfg, parts, complex_step=seed)
        oc.step(steps)
        cs = _mean_height(oc, imag=True) / seed["h"]
        del oc
    fd = None
    if do_fd:
        base = np.load(os.path.join(partial, "base.npz"))
        replay = (np.ascontiguousarray(base["X"]), np.ascontiguousarray(base["theta"]))
        h = 1e-6 * abs(values[k])
        Ls = []
        for sgn in (+1, -1):
            p2 = [dict(q) for q in parts]
            c2 = dict(cfg)
            if k < npart:
                p2[k]["rho_s"] += sgn * h
            elif name == "tau":
                c2["tau"] += sgn * h
            else:
                c2["g"] = tuple(np.asarray(cfg["g"]) * (gmag + sgn * h) / gmag)
            o = O.Oracle(c2, p2)
            o.set_replay(0, *replay)
            o.step(steps)
            Ls.append(_mean_height(o))
            del o
        fd = (Ls[0] - Ls[1]) / (2 * h)
    out = dict(k=k, name=name, complex_step=cs, central_diff=fd, seconds=time.time() - t0)
    tmp = os.path.join(partial, f"p{k:02d}.json.tmp")
    with open(tmp, "w") as f:
        json.dump(out, f)
    os.replace(tmp, os.path.join(partial, f"p{k:02d}.json"))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=5000)
    ap.add_argument("--partial", required=True, help="directory for per-parameter results")
    ap.add_argument("--jobs", type=int, default=3)
    ap.add_argument("--threads", type=int, default=2, help="OpenMP threads per job")
    ap.add_argument("--fd", default=FD_DEFAULT, help="'all' or the parameters that get central differences")
    ap.add_argument("--cs-from", default=None, help="reuse the complex-step values of this earlier output")
    ap.add_argument("--one", type=int, default=None, help=argparse.SUPPRESS)
    ap.add_argument("--out", default=os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                                  f"{NAME}_grad.json"))
    args = ap.parse_args()
    os.makedirs(args.partial, exist_ok=True)
    cfg, parts, gmag, names, values = _setup()
    fd_names = set(names) if args.fd == "all" else set(s for s in args.fd.split(",") if s)
    if args.one is not None:
        run_one(args.one, args.steps, args.partial, names[args.one] in fd_names, args.cs_from)
        return

    from oracle import oracle as O

    t0 = time.time()
    meta = os.path.join(args.partial, "base.json")
    if os.path.exists(meta) and json.load(open(meta))["steps"] == args.steps:
        L0 = json.load(open(meta))["loss"]
    else:
        base = O.Oracle(cfg, parts)
        rec = base.step(args.steps, record=True)
        L0 = _mean_height(base)
        np.savez(os.path.join(args.partial, "base.npz"), X=rec[:, :, 0:3].copy(), theta=rec[:, :, 3].copy())
        with open(meta, "w") as f:
            json.dump(dict(steps=args.steps, loss=L0), f)
        del base
    print(f"base run done ({time.time() - t0:.0f} s), L = {L0!r}", flush=True)

    todo = [k for k in range(len(names)) if not os.path.exists(os.path.join(args.partial, f"p{k:02d}.json"))]
    env = dict(os.environ, OMP_NUM_THREADS=str(args.threads))

    def job(k):
        cmd = [sys.executable, os.path.abspath(__file__), "--one", str(k), "--steps", str(args.steps),
               "--partial", args.partial, "--fd", args.fd] + (["--cs-from", args.cs_from] if args.cs_from else [])
        r = subprocess.run(cmd, env=env)
        res = json.load(open(os.path.join(args.partial, f"p{k:02d}.json"))) if r.returncode == 0 else None
        print(f"{names[k]}: rc {r.returncode} {res} ({time.time() - t0:.0f} s)", flush=True)
        return r.returncode

    with ThreadPoolExecutor(args.jobs) as ex:
        rcs = list(ex.map(job, todo))
    if any(rcs):
        sys.exit("some parameter jobs failed; run again to resume")

    res = [json.load(open(os.path.join(args.partial, f"p{k:02d}.json"))) for k in range(len(names))]
    out = dict(workload=NAME, steps=args.steps, loss="mean final Y of the 16 disks", loss_value=L0,
               params=names, values=values, grad_complex_step=[r["complex_step"] for r in res],
               grad_central_diff=[r["central_diff"] for r in res], fd_rel_step=1e-6, complex_step_h=1e-30,
               note="FP64 oracle; indicator frozen at the base run (replayed for the differences); "
                    "central differences only where not null")
    with open(args.out, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", args.out)


if __name__ == "__main__":
    main()
