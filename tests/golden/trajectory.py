"""Resumable FP64 oracle trajectory runs for the stored expected values.

run(cfg, parts, steps, every, save_every, partial) advances the oracle in
blocks of `every` steps, keeping each body's centre X and measured velocity U
after every block.  Every `save_every` steps the populations and particle
state go to the `partial` directory (the log that names them is replaced
atomically), so an interrupted run continues from the last saved step with
the same results as an uninterrupted one: the saved state is exactly what
the next step starts from (populations f^n; X, theta, U^{n-1}, omega^{n-1},
A^n of every body).

Calls only oracle/.
"""
import json
import os
import time

import numpy as np

from oracle import oracle as O


def run(cfg, parts, steps, every, save_every, partial, d):
    os.makedirs(partial, exist_ok=True)
    t0 = time.time()
    o = O.Oracle(cfg, parts)
    log_path = os.path.join(partial, "log.json")
    log = dict(record_steps=[], X=[], U=[], saved=0)
    if os.path.exists(log_path):
        log = json.load(open(log_path))
        step0 = log["saved"]
        o.set_f(np.load(os.path.join(partial, f"f_{step0}.npy")))
        o.load_particles(np.load(os.path.join(partial, f"p_{step0}.npy")), step0)
        print(f"resumed at step {step0}", flush=True)
    done = log["saved"]
    while done < steps:
        n = min(every, steps - done)
        r = o.step(n, record=True)
        done += n
        log["record_steps"].append(done)
        log["X"].append(r[-1, :, 0:d].tolist())
        log["U"].append(r[-1, :, 4:4 + d].tolist())
        if done % save_every == 0 or done == steps:
            np.save(os.path.join(partial, f"f_{done}.npy"), o.f())
            np.save(os.path.join(partial, f"p_{done}.npy"), o.particles()["raw"])
            prev = log["saved"]
            log["saved"] = done
            with open(log_path + ".tmp", "w") as f:
                json.dump(log, f)
            os.replace(log_path + ".tmp", log_path)
            for k in ("f", "p"):
                old = os.path.join(partial, f"{k}_{prev}.npy")
                if prev and os.path.exists(old):
                    os.remove(old)
        print(f"{done} steps ({time.time() - t0:.0f} s)", flush=True)
    return o, log


def rounded(rows):
    """10 significant digits: far below the reduced-precision errors compared
    against, and half the size of full FP64 text."""
    return [[[float(f"{v:.10g}") for v in body] for body in row] for row in rows]
