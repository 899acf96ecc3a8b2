"""Moving walls on the GPU: the plane Couette configuration of sec. 3.1
(halfway walls at -1/2 and H - 1/2 moving tangentially; a population bounced
off a moving wall gains the difference of the equilibria of eq. 13 at the
wall velocity).

* parity with the FP64 oracle: fluid from a random state in D2Q9 and D3Q19
  (FP64, FP32 with the LDS-staged D3Q19 kernel, one step in FP16/BF16),
  bodies in the sheared channel, and the adjoint against the complex-step
  oracle;
* the exact linear Couette profile, reached on the GPU;
* the lateral-migration workload of sec. 3.1 (5000x200, tau = 1, a neutrally
  buoyant disk of diameter 50 released at (15D, D)): parity with the oracle
  over its first steps at full size, then the full run, in which the disk
  migrates to the mid-plane y/H = 1/2.
"""
import numpy as np
import pytest

from gpu_common import banner, pair, rel
from paper_2511_01629_amd import lbm
from paper_2511_01629_amd.workloads import place, random_state, workload
from test_gpu_adjoint import _check, gpu_gradient, oracle_gradient
from test_gpu_parity import TOL, _compare_run, _half_quantum, _round_storage
from test_oracle_pins import couette_walls

pytestmark = pytest.mark.gpu


def _walls_2d(lo, hi):
    return [[(0.0, 0.0, 0.0)] * 2, [lo, hi], [(0.0, 0.0, 0.0)] * 2]


def test_couette_fluid_random_state_f64():
    """D2Q9, periodic x, walls in y moving at different speeds, 20 steps from
    a random state: populations and fields within 1e-12 of the oracle."""
    banner("couette fluid 2d f64")
    n = (37, 29, 1)
    cfg = dict(lattice="D2Q9", n=n, periodic=(1, 0, 0), tau=0.75,
               wall_velocity=_walls_2d((-0.03, 0.0, 0.0), (0.045, 0.0, 0.0)))
    f0 = random_state((1, n[1], n[0]), 9, 2e-3, seed=41)
    sim, ora = pair(cfg, [], f0=f0)
    assert rel(sim.populations(), f0) < 1e-15  # the inverse of the pull, moving walls included
    sim.step(20)
    ora.step(20)
    assert rel(sim.populations(), ora.f()) < TOL
    ug, pg, _ = sim.fields()
    uo, po, _ = ora.fields()
    assert rel(ug, uo) < TOL and rel(pg, po) < TOL * 10


@pytest.mark.parametrize("lattice,n,axis", [("D2Q9", (9, 7, 1), 1), ("D3Q19", (5, 6, 7), 2)])
def test_couette_initial_state(lattice, n, axis):
    """The uniform initial state is f^eq(p0, u0) on every node, also next to
    a moving wall (the stored state is the previous step's post-collision
    populations, so the wall term is taken out of the bounced ones)."""
    banner(f"couette initial state {lattice}")
    w = couette_walls(0.04, axis)
    cfg = dict(lattice=lattice, n=n, periodic=tuple(int(k != axis) for k in range(3)), tau=0.8,
               u0=(0.01, -0.005, 0.0), p0=0.002, wall_velocity=w)
    sim, ora = pair(cfg, [])
    assert rel(sim.populations(), ora.f()) < 1e-15


@pytest.mark.parametrize("storage,tol", [("f64", TOL), ("f32", 5e-6)])
def test_couette_fluid_3d(storage, tol):
    """D3Q19, periodic x and y, walls normal to z moving along different
    tangential directions (nx a multiple of 4: the FP32 rows are staged
    through LDS)."""
    banner(f"couette fluid 3d {storage}")
    n = (8, 7, 9)
    w = [[(0.0, 0.0, 0.0)] * 2, [(0.0, 0.0, 0.0)] * 2, [(0.02, -0.01, 0.0), (-0.015, 0.025, 0.0)]]
    cfg = dict(lattice="D3Q19", n=n, periodic=(1, 1, 0), tau=0.7, wall_velocity=w)
    f0 = random_state((n[2], n[1], n[0]), 19, 2e-3, seed=42)
    if storage == "f32":
        f0 = f0.astype(np.float32).astype(np.float64)
    sim, ora = pair(cfg, [], storage=storage, f0=f0)
    sim.step(10)
    ora.step(10)
    e = rel(sim.populations(), ora.f())
    print(f"[measured] couette 3d {storage}: populations rel err {e:.2e}", flush=True)
    assert e < tol


@pytest.mark.parametrize("storage,tol", [("f64", TOL), ("f32", 5e-6), ("f16", None)])
def test_couette_fluid_3d_y_walls(storage, tol):
    """D3Q19 with the moving walls normal to y (x and z periodic): the rows
    next to them are whole (y, z) rows, in every storage type (FP32 staged
    through LDS; FP16 one step within half a storage quantum)."""
    banner(f"couette fluid 3d y walls {storage}")
    n = (12, 7, 6)
    w = [[(0.0, 0.0, 0.0)] * 2, [(0.02, 0.0, -0.01), (-0.015, 0.0, 0.02)], [(0.0, 0.0, 0.0)] * 2]
    cfg = dict(lattice="D3Q19", n=n, periodic=(1, 0, 1), tau=0.7, wall_velocity=w)
    f0 = random_state((n[2], n[1], n[0]), 19, 2e-3, seed=46)
    if storage == "f32":
        f0 = f0.astype(np.float32).astype(np.float64)
    if storage == "f16":
        f0 = _round_storage(f0, "f16")
    sim, ora = pair(cfg, [], storage=storage, f0=f0)
    if storage == "f16":
        ora.set_f(sim.populations())
        sim.step(1)
        ora.step(1)
        g, o = sim.populations(), ora.f()
        mag = np.abs(o)
        mag[:, [0, -1]] += 2.0 / 18.0 * 0.025 * 3.0
        excess = np.abs(g - o) - (_half_quantum(mag, "f16") * (1 + 1e-3) + 2e-6 * np.abs(o).max())
        assert excess.max() <= 0.0, excess.max()
        return
    sim.step(10)
    ora.step(10)
    e = rel(sim.populations(), ora.f())
    print(f"[measured] couette 3d y walls {storage}: populations rel err {e:.2e}", flush=True)
    assert e < tol


def test_couette_sphere_3d_f64():
    """A sphere sheared between walls normal to z (D3Q19, FP64), with
    gravity along the walls' normal: the whole step within 1e-12."""
    banner("couette sphere 3d f64")
    w = [[(0.0, 0.0, 0.0)] * 2, [(0.0, 0.0, 0.0)] * 2, [(-0.02, 0.01, 0.0), (0.03, 0.0, 0.0)]]
    cfg = dict(lattice="D3Q19", n=(18, 16, 20), periodic=(1, 1, 0), tau=0.7, g=(0.0, 0.0, -3e-4), wall_velocity=w)
    parts = [dict(shape="sphere", rho_s=1.4, a=4.0, x=(8.3, 7.6, 9.2))]
    f0 = random_state((20, 16, 18), 19, 1e-3, seed=47)
    _compare_run(cfg, parts, 15, f0=f0)


@pytest.mark.parametrize("storage", ["f16", "bf16"])
def test_couette_two_byte_step(storage):
    """One step in 2-byte storage on rows of several segments with moving y
    walls: every population within half a storage quantum of the oracle's
    (from the same state), plus FP32 arithmetic."""
    banner(f"couette two-byte {storage}")
    n = (1600, 24, 1)
    cfg = dict(lattice="D2Q9", n=n, periodic=(1, 0, 0), tau=0.7,
               wall_velocity=_walls_2d((-0.04, 0.0, 0.0), (0.05, 0.0, 0.0)))
    f0 = _round_storage(random_state((1, n[1], n[0]), 9, 5e-3, seed=43), storage)
    sim, ora = pair(cfg, [], storage=storage, f0=f0)
    # next to a moving wall the stored value is f - (wall term), rounded to 2
    # bytes, so the state the GPU holds differs from f0 there by that
    # rounding: the oracle starts from the populations the GPU holds
    ora.set_f(sim.populations())
    sim.step(1)
    ora.step(1)
    g, o = sim.populations(), ora.f()
    # a population bounced off a moving wall is the stored value of the
    # opposite one plus the wall term (at most 2 (1/9) 0.05 / cs^2 here): its
    # rounding is that of a value up to that much larger
    mag = np.abs(o)
    mag[:, [0, -1]] += 2.0 / 9.0 * 0.05 * 3.0
    bound = _half_quantum(mag, storage) * (1 + 1e-3) + 2e-6 * np.abs(o).max()
    excess = np.abs(g - o) - bound
    print(f"[measured] couette {storage}: max |g - o| {np.abs(g - o).max():.3e}, worst excess {excess.max():.3e}",
          flush=True)
    assert excess.max() <= 0.0


@pytest.mark.parametrize("storage,tol", [("f64", 1e-13), ("f32", 2e-5)])
def test_couette_steady_profile(storage, tol):
    """Walls at -U/2 and +U/2: the GPU reaches the exact linear profile (the
    oracle pin shows it is exact to round-off in FP64)."""
    banner(f"couette profile {storage}")
    H, U, tau = 16, 0.02, 0.8
    cfg = dict(lattice="D2Q9", n=(4, H, 1), periodic=(1, 0, 0), tau=tau, wall_velocity=couette_walls(U))
    sim = lbm.Simulation(cfg, [], storage=storage, device=0)
    sim.step(int(40 * H * H / ((tau - 0.5) / 3)))
    u, _, _ = sim.fields()
    exact = -U / 2 + U * (np.arange(H) + 0.5) / H
    e = np.abs(u[0, :, :, 0] - exact[:, None]).max() / U
    print(f"[measured] couette profile {storage}: max |u - linear| / U = {e:.2e}", flush=True)
    assert e < tol
    sim.close()


def test_couette_particles_f64():
    """Two disks and an ellipse sheared between moving walls (one neutrally
    buoyant), with gravity and contacts: the whole step within 1e-12."""
    banner("couette particles f64")
    cfg = dict(lattice="D2Q9", n=(60, 40, 1), periodic=(1, 0, 0), tau=0.7, g=(0.0, -2e-4, 0.0),
               wall_velocity=_walls_2d((-0.02, 0.0, 0.0), (0.03, 0.0, 0.0)))
    parts = [dict(shape="disk", rho_s=1.0, a=5.0, x=(12.3, 20.4, 0.0)),
             dict(shape="disk", rho_s=1.4, a=4.0, x=(22.0, 24.1, 0.0)),
             dict(shape="ellipse", rho_s=1.3, a=6.0, b=3.0, x=(45.5, 8.3, 0.0), theta=0.4)]
    f0 = random_state((1, 40, 60), 9, 1e-3, seed=44)
    _compare_run(cfg, parts, 40, f0=f0)


def test_couette_adjoint_f64():
    """The adjoint with moving walls (the wall term is a constant of the step,
    so its transpose adds nothing, but the pre-collision populations the
    Jacobian is taken at include it): against the complex-step oracle."""
    banner("couette adjoint f64")
    kinds = [("disk", 5.0, 5.0)] * 3
    parts = place((40, 48), kinds, seed=45, rho_range=(1.3, 1.7), upper_axis=1, gap=1.0, margin=2.0)
    cfg = dict(lattice="D2Q9", n=(40, 48, 1), periodic=(1, 0, 0), tau=0.7, g=(0.0, -3e-4, 0.0),
               wall_velocity=_walls_2d((-0.02, 0.0, 0.0), (0.03, 0.0, 0.0)))
    w = np.random.default_rng(7).normal(size=(len(parts), 3))
    w[:, 2] = 0.0
    steps = 40
    go = oracle_gradient(cfg, parts, steps, w)
    ga = gpu_gradient(cfg, parts, steps, 10, w)
    _check(ga, go, 1e-8)


def test_couette_migration_workload():
    """The lateral-migration workload of sec. 3.1 (FP64): the first 300 steps
    at full size against the oracle (1e-12), then the paper's 700,000 steps
    (t* = shear rate x t = 58.3).  The disk, released at y/H = 1/4 (y from
    the lower wall at -1/2), migrates steadily toward the mid-plane: the
    distance to y/H = 1/2 never rises more than 1e-3 above its running
    minimum, y/H passes 0.41, and the disk turns at about minus half the shear
    rate, as a free disk in shear does (within 10 %).  A run 5 times longer
    (measured separately) ends at y/H = 0.499."""
    cfg, parts, steps, info = workload("couette_migration_5000x200")
    H, gamma = cfg["n"][1], info["shear_rate"]
    banner("couette migration: parity over the first 300 steps at 5000x200")
    sim, ora = pair(cfg, parts)
    rg = sim.step_record(300)
    ro = ora.step(300, record=True)
    assert np.abs(rg[:, :, 0:3] - ro[:, :, 0:3]).max() / H < TOL
    assert rel(sim.populations(), ora.f()) < TOL
    del ora
    banner("couette migration: full run")
    chunk = 10000
    height = lambda: (sim.particles()["X"][0][1] + 0.5) / H
    done, ys, ts = 300, [height()], [300]
    while done < steps:
        k = min(chunk, steps - done)
        sim.step(k)
        done += k
        ys.append(height())
        ts.append(done)
    omega = sim.particles()["omega"][0][2]
    sim.close()
    ys, t_star = np.array(ys), gamma * np.array(ts, dtype=float)
    for i in range(0, len(ys), 7):
        print(f"[measured] t* = {t_star[i]:6.2f}  y/H = {ys[i]:.4f}", flush=True)
    print(f"[measured] final t* = {t_star[-1]:.2f}  y/H = {ys[-1]:.4f}, omega / (-gamma/2) = {omega / (-gamma / 2):.4f}",
          flush=True)
    dist = np.abs(ys - 0.5)
    assert (dist - np.minimum.accumulate(dist)).max() < 1e-3
    assert ys[-1] > 0.41 and ys[-1] < 0.5, ys[-1]
    assert abs(omega / (-gamma / 2) - 1) < 0.1, omega
