"""Shared helpers of the GPU parity tests (HIP library vs FP64 oracle)."""
import math
import sys

import numpy as np

from oracle import oracle as O
from paper_2511_01629_amd import lbm


def banner(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def rel(a, b):
    den = np.abs(b).max()
    return float(np.abs(a - b).max() / (den if den > 0 else 1.0))


def pair(cfg, parts, storage="f64", f0=None, max_particles=None):
    """A library simulation and an oracle run from the same state.  With f0
    (shape (nz, ny, nx, Q)) both start from those populations."""
    sim = lbm.Simulation(cfg, parts, storage=storage, device=0, max_particles=max_particles)
    ora = O.Oracle(cfg, parts)
    if f0 is not None:
        sim.set_populations(f0)
        ora.set_f(f0)
        if parts:
            sim.set_particles(parts)
            ora.reset_particles(parts)
    return sim, ora


def shape_margin(p, X, theta, node):
    """Signed distance-like margin of `node` to the boundary of particle p at
    centre X (positive inside).  Used to accept indicator differences only at
    nodes that sit on a boundary to round-off."""
    r = np.asarray(node, dtype=float) - np.asarray(X)[: len(node)]
    if p["shape"] in ("disk", "sphere"):
        return (p["a"] ** 2 - float(r @ r)) / p["a"] ** 2
    c, s = math.cos(theta), math.sin(theta)
    xi = c * r[0] + s * r[1]
    eta = -s * r[0] + c * r[1]
    a, b = p["a"], p["b"]
    return (a * a * b * b - b * b * xi * xi - a * a * eta * eta) / (a * a * b * b)


def check_owner(own_g, own_o, parts, P, periodic=(0, 0, 0), tol=1e-9):
    """Indicators equal, except at nodes on a boundary to within `tol`."""
    diff = np.argwhere(own_g != own_o)
    shp = own_o.shape  # (nz, ny, nx)
    n = (shp[2], shp[1], shp[0])
    for z, y, x in diff:
        ids = {int(own_g[z, y, x]), int(own_o[z, y, x])} - {-1}
        ok = False
        for i in ids:
            node = [x, y, z][: 3 if parts[i]["shape"] == "sphere" else 2]
            node = np.array(node, dtype=float)
            for k in range(len(node)):
                if periodic[k]:
                    dlt = node[k] - P["X"][i][k]
                    node[k] -= n[k] * round(dlt / n[k])
            if abs(shape_margin(parts[i], P["X"][i], P["theta"][i], node)) < tol:
                ok = True
        assert ok, f"indicator differs away from a boundary at {(x, y, z)}: {own_g[z, y, x]} vs {own_o[z, y, x]}"
    return len(diff)
