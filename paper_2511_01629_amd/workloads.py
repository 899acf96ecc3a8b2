"""Seeded synthetic workloads (configurations and particle lists).

This module holds inputs only -- no step of the method.  Both the GPU path and
the oracle take what it returns (plain dicts), so neither has to import the
other.

The five workloads are shaped like the paper's sedimentation cases
(sec. 3.2-3.5: disks and ellipses settling in closed boxes, tau near 1/2,
small gravity in lattice units) plus a floating disk in uniform flow (sec. 3.1
uses a neutrally buoyant disk).  The paper's own initial particle patterns and
literature comparison data are not available; the bodies here are placed by
seeded rejection sampling:

  * centres uniform in the upper half of the box along the gravity axis,
  * a wall margin of (bounding radius + 2) lattice units,
  * a gap of at least 2 lattice units between bounding circles/spheres,
  * densities uniform in the stated range, ellipse angles uniform in [0, pi),
  * the order of shapes shuffled by the same generator.

Lattice units: node (i, j[, k]) sits at (i, j[, k]); walls at -0.5 and n-0.5.
"""
import numpy as np

BASE = dict(alpha=0.0, rho_f=1.0, u0=(0.0, 0.0, 0.0), p0=0.0, eps_p=2.0, eps_w=1.0, delta=1.0, K=1,
            collision_form=0, gravity_form=0, fluid_accel=(0.0, 0.0, 0.0), penalize_all=0)


def _cfg(**kw):
    c = dict(BASE)
    c.update(kw)
    return c


def place(n, kinds, seed, rho_range, upper_axis, gap=2.0, margin=2.0, max_tries=200000):
    """Rejection-sample non-overlapping bodies.  kinds: list of
    (shape, a, b) tuples, drawn in a seeded shuffled order.  Returns a list of
    particle dicts."""
    rng = np.random.default_rng(seed)
    order = np.arange(len(kinds))
    rng.shuffle(order)
    d = len(n)
    out, centres, radii = [], [], []
    for idx in order:
        shape, a, b = kinds[idx]
        Rb = a
        lo = np.array([-0.5 + Rb + margin] * d)
        hi = np.array([n[k] - 0.5 - Rb - margin for k in range(d)])
        lo[upper_axis] = max(lo[upper_axis], n[upper_axis] / 2.0)
        for _ in range(max_tries):
            x = rng.uniform(lo, hi)
            if centres:
                dist = np.linalg.norm(np.asarray(centres) - x, axis=1)
                if np.any(dist < np.asarray(radii) + Rb + gap):
                    continue
            break
        else:
            raise RuntimeError("placement failed")
        rho = float(rng.uniform(*rho_range))
        theta = float(rng.uniform(0.0, np.pi)) if shape == "ellipse" else 0.0
        centres.append(x)
        radii.append(Rb)
        out.append(dict(shape=shape, rho_s=rho, a=float(a), b=float(b), x=tuple(float(v) for v in x) + (0.0,) * (3 - d),
                        theta=theta))
    return out


def workload(name):
    """Return (cfg, particles, steps, info) for one of the named workloads."""
    if name == "floating_disk_200x400":
        cfg = _cfg(lattice="D2Q9", n=(200, 400, 1), periodic=(1, 0, 0), tau=0.8, g=(0.0, 0.0, 0.0),
                   u0=(0.02, 0.0, 0.0), storage="f64")
        parts = [dict(shape="disk", rho_s=1.0, a=10.0, b=10.0, x=(100.0, 200.0, 0.0), theta=0.0)]
        return cfg, parts, 2000, dict(desc="floating disk R=10 in uniform flow 0.02, x periodic, y walls")
    if name == "disk_settling_400x1600":
        cfg = _cfg(lattice="D2Q9", n=(400, 1600, 1), periodic=(0, 0, 0), tau=0.6, g=(0.0, -1e-5, 0.0),
                   storage="f32")
        parts = [dict(shape="disk", rho_s=1.5, a=12.0, b=12.0, x=(200.0, 1400.0, 0.0), theta=0.0)]
        return cfg, parts, 20000, dict(desc="single disk R=12 settling in a closed 400x1600 channel")
    if name == "sedimentation_2048x4096":
        cfg = _cfg(lattice="D2Q9", n=(2048, 4096, 1), periodic=(0, 0, 0), tau=0.55, g=(0.0, -2e-6, 0.0),
                   storage="f32")
        kinds = [("disk", 8.0, 8.0)] * 350 + [("ellipse", 12.0, 6.0)] * 150
        parts = place((2048, 4096), kinds, 1629, (1.1, 1.5), upper_axis=1)
        return cfg, parts, 10000, dict(desc="500 bodies (350 disks R=8, 150 ellipses 12x6) settling in 2048x4096")
    if name == "spheres_256x256x512":
        cfg = _cfg(lattice="D3Q19", n=(256, 256, 512), periodic=(0, 0, 0), tau=0.6, g=(0.0, 0.0, -1e-5),
                   storage="f32")
        kinds = [("sphere", 8.0, 8.0)] * 64
        parts = place((256, 256, 512), kinds, 1630, (1.2, 1.8), upper_axis=2)
        return cfg, parts, 5000, dict(desc="64 spheres R=8 settling in a closed 256x256x512 box (D3Q19)")
    if name == "spheres_64x64x128":
        # the sphere workload's spheres, fluid and gravity in a box 1/64 of its
        # volume with 8 spheres (8 times its solid fraction, so that they meet):
        # the full 5000-step horizon within reach of the FP64 oracle
        cfg = _cfg(lattice="D3Q19", n=(64, 64, 128), periodic=(0, 0, 0), tau=0.6, g=(0.0, 0.0, -1e-5),
                   storage="f32")
        kinds = [("sphere", 8.0, 8.0)] * 8
        parts = place((64, 64, 128), kinds, 1632, (1.2, 1.8), upper_axis=2)
        return cfg, parts, 5000, dict(desc="8 spheres R=8 settling in a closed 64x64x128 box (D3Q19)")
    if name == "adjoint_512x1024":
        cfg = _cfg(lattice="D2Q9", n=(512, 1024, 1), periodic=(0, 0, 0), tau=0.7, g=(0.0, -1e-5, 0.0),
                   storage="f32")
        kinds = [("disk", 10.0, 10.0)] * 16
        parts = place((512, 1024), kinds, 1631, (1.2, 1.6), upper_axis=1)
        return cfg, parts, 5000, dict(desc="16 disks R=10 in 512x1024; loss = mean final height", checkpoint=100)
    if name == "couette_migration_5000x200":
        # plane Couette flow, H = 4D, L = 100D, walls at -U_w/2 and +U_w/2 with
        # U_w = 1/60, tau = 1; a neutrally buoyant disk of diameter D = 50
        # released at (15D, D)
        H, D, Uw = 200, 50.0, 1.0 / 60.0
        cfg = _cfg(lattice="D2Q9", n=(100 * int(D), H, 1), periodic=(1, 0, 0), tau=1.0, g=(0.0, 0.0, 0.0),
                   storage="f64",
                   wall_velocity=[[(0.0, 0.0, 0.0)] * 2, [(-Uw / 2, 0.0, 0.0), (Uw / 2, 0.0, 0.0)], [(0.0, 0.0, 0.0)] * 2])
        parts = [dict(shape="disk", rho_s=1.0, a=D / 2, b=D / 2, x=(15 * D, D, 0.0), theta=0.0)]
        return cfg, parts, 700000, dict(desc="lateral migration of a neutrally buoyant disk in plane Couette flow",
                                        shear_rate=Uw / H)
    raise KeyError(name)


NAMES = ["floating_disk_200x400", "disk_settling_400x1600", "sedimentation_2048x4096", "spheres_256x256x512",
         "spheres_64x64x128", "couette_migration_5000x200",
         "adjoint_512x1024"]


def random_state(shape, Q, scale, seed):
    """Seeded random population field of the given shape (..., Q), used to start
    both sides from an arbitrary non-equilibrium state."""
    rng = np.random.default_rng(seed)
    return rng.normal(0.0, scale, size=tuple(shape) + (Q,))
