"""GPU parity: the HIP library through its C ABI against the FP64 oracle on the
same seeded inputs (FP64 storage: within 1e-12 relative).

Sizes span several 256-node workgroups with a ragged tail; walls, periodic
axes, corners, contacts and ellipses are all exercised.
"""
import numpy as np
import pytest

from gpu_common import banner, check_owner, pair, rel
from oracle import oracle as O
from paper_2511_01629_amd import lbm
from paper_2511_01629_amd.workloads import place, random_state, workload

pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.mark.parametrize("kind,n,periodic", [
    ("D2Q9", (37, 29, 1), (0, 0, 0)),
    ("D2Q9", (37, 29, 1), (1, 0, 0)),
    ("D2Q9", (33, 20, 1), (1, 1, 0)),
    ("D3Q19", (13, 11, 9), (0, 0, 0)),
    ("D3Q19", (13, 11, 9), (1, 0, 1)),
    ("D3Q19", (12, 11, 9), (1, 1, 0)),
])
def test_fluid_step_random_state(kind, n, periodic):
    """Pull streaming with bounce-back/wrap and the BGK collision from a random
    non-equilibrium state (eq. 10, 13, 15)."""
    banner(f"fluid random {kind} {n} {periodic}")
    cfg = dict(lattice=kind, n=n, periodic=periodic, tau=0.7, fluid_accel=(2e-5, -1e-5, 3e-6))
    Q = 9 if kind == "D2Q9" else 19
    shp = (n[2] if kind == "D3Q19" else 1, n[1], n[0])
    f0 = random_state(shp, Q, 2e-3, seed=11)
    sim, ora = pair(cfg, [], f0=f0)
    assert rel(sim.populations(), f0) < 1e-16  # set/get round trip through the inverse pull
    for steps in (1, 4):
        sim.step(steps)
        ora.step(steps)
        e = rel(sim.populations(), ora.f())
        assert e < TOL, e
    ug, pg, _ = sim.fields()
    uo, po, _ = ora.fields()
    assert rel(ug, uo) < TOL and rel(pg, po) < TOL


@pytest.mark.parametrize("n,periodic", [
    ((12, 11, 9), (0, 0, 0)),    # one partial segment, walls on every side
    ((12, 11, 9), (1, 1, 0)),
    ((520, 3, 4), (1, 0, 1)),    # three segments: the x halo across segment edges, periodic wrap
    ((520, 3, 4), (0, 1, 0)),
])
def test_fluid_step_random_state_f32_3d(n, periodic):
    """D3Q19 in FP32 storage, the rows staged through LDS (nx a multiple of 4):
    the same steps as the FP64 oracle, to FP32 rounding (a few ulp of the
    populations per step)."""
    banner(f"fluid random f32 D3Q19 {n} {periodic}")
    cfg = dict(lattice="D3Q19", n=n, periodic=periodic, tau=0.7, fluid_accel=(2e-5, -1e-5, 3e-6))
    f0 = random_state((n[2], n[1], n[0]), 19, 2e-3, seed=12).astype(np.float32).astype(np.float64)
    sim, ora = pair(cfg, [], storage="f32", f0=f0)
    for steps in (1, 4):
        sim.step(steps)
        ora.step(steps)
        e = rel(sim.populations(), ora.f())
        print(f"[measured] f32 3D {n} {periodic} after {steps}: {e:.2e}", flush=True)
        assert e < 5e-6, e


def _round_storage(f, storage):
    """The values 2-byte storage holds (round to nearest even)."""
    if storage == "f16":
        return f.astype(np.float16).astype(np.float64)
    u = f.astype(np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _half_quantum(o, storage):
    a = np.abs(o)
    if storage == "f16":
        return 0.5 * np.spacing(a.astype(np.float16)).astype(np.float64)
    return 0.5 * 2.0 ** (np.floor(np.log2(np.maximum(a, 1e-38))) - 7)


@pytest.mark.parametrize("storage", ["f16", "bf16"])
@pytest.mark.parametrize("periodic,with_parts", [((1, 0, 0), False), ((0, 1, 0), False), ((1, 0, 0), True)])
def test_two_byte_step_wide_rows(storage, periodic, with_parts):
    """D2Q9 in 2-byte storage on a lattice of several row segments (interior
    segments, whose sources come from uniform row pointers, and row-end and
    wall-row segments, which take per-node offsets).  One step from a random
    state against the FP64 oracle started from the same rounded populations:
    every population within half a storage quantum of the oracle's, plus
    FP32 arithmetic.  With bodies: some inside interior segments, one across
    a wavefront edge there, one wrapping the periodic x axis."""
    banner(f"two-byte wide rows {storage} {periodic} parts={with_parts}")
    n = (1600, 24, 1)
    cfg = dict(lattice="D2Q9", n=n, periodic=periodic, tau=0.7)
    parts = []
    if with_parts:
        cfg["g"] = (0.0, -3e-4, 0.0)
        parts = [dict(shape="disk", rho_s=1.5, a=5.0, x=(700.3, 12.2, 0.0)),
                 dict(shape="disk", rho_s=1.3, a=4.5, x=(1023.6, 10.7, 0.0)),
                 dict(shape="ellipse", rho_s=1.4, a=6.0, b=3.0, x=(1540.2, 12.5, 0.0), theta=0.7),
                 dict(shape="disk", rho_s=1.6, a=4.0, x=(2.1, 11.4, 0.0))]
    else:
        cfg["fluid_accel"] = (2e-5, -1e-5, 0.0)
    scale = 5e-3
    f0 = _round_storage(random_state((1, n[1], n[0]), 9, scale, seed=31), storage)
    sim, ora = pair(cfg, parts, storage=storage, f0=f0)
    assert np.array_equal(sim.populations(), f0)
    rg = sim.step_record(1) if with_parts else None
    ro = ora.step(1, record=True) if with_parts else None
    if not with_parts:
        sim.step(1)
        ora.step(1)
    g, o = sim.populations(), ora.f()
    bound = _half_quantum(o, storage) * (1 + 1e-3) + 2e-6 * np.abs(o).max()
    excess = np.abs(g - o) - bound
    print(f"[measured] {storage} {periodic} parts={with_parts}: max |g - o| {np.abs(g - o).max():.3e}, "
          f"worst excess over the bound {excess.max():.3e}", flush=True)
    assert excess.max() <= 0.0
    if with_parts:
        assert np.array_equal(rg[:, :, 13], ro[:, :, 13])  # node counts
        Usc = np.abs(ro[:, :, 4:6]).max()
        assert np.abs(rg[:, :, 4:6] - ro[:, :, 4:6]).max() <= 1e-4 * Usc
        _, _, og = sim.fields()
        _, _, oo = ora.fields()
        check_owner(og, oo, parts, ora.particles(), periodic)


def test_penalize_all_random_state():
    banner("penalize_all random")
    cfg = dict(lattice="D2Q9", n=(31, 27, 1), periodic=(1, 1, 0), tau=0.8, alpha=0.6, penalize_all=1)
    f0 = random_state((1, 27, 31), 9, 2e-3, seed=5)
    sim, ora = pair(cfg, [], f0=f0)
    sim.step(3)
    ora.step(3)
    assert rel(sim.populations(), ora.f()) < TOL


def _compare_run(cfg, parts, steps, f0=None, storage="f64", tol=TOL, xtol=TOL, fused=None):
    """fused: if not None, whether the step must take the momentum sums in the
    lattice kernel (no separate momentum-sum launches)."""
    sim, ora = pair(cfg, parts, storage=storage, f0=f0)
    if fused is not None:
        sim.profile(True)
    rg = sim.step_record(steps)
    if fused is not None:
        launches = sim.profile_read()["reduce_clear"][1]
        sim.profile(False)
        assert (launches == 0) == fused, launches
    ro = ora.step(steps, record=True)
    # per-step records: X theta U omega A N
    scaleX = max(np.abs(ro[:, :, 0:3]).max(), 1.0)
    assert np.abs(rg[:, :, 0:3] - ro[:, :, 0:3]).max() / scaleX < xtol
    assert rel(rg[:, :, 4:10], ro[:, :, 4:10]) < tol * 10
    eA = np.abs(rg[:, :, 10:13] - ro[:, :, 10:13]).max()
    assert eA <= max(tol * 10 * np.abs(ro[:, :, 10:13]).max(), 1e-13), eA
    assert np.array_equal(rg[:, :, 13], ro[:, :, 13])
    fg, fo = sim.populations(), ora.f()
    assert rel(fg, fo) < tol
    Pg, Po = sim.particles(), ora.particles()
    ug, pg, og = sim.fields()
    uo, po, oo = ora.fields()
    assert rel(ug, uo) < tol and rel(pg, po) < tol * 10
    check_owner(og, oo, parts, Po, cfg.get("periodic", (0, 0, 0)))
    # omega is a ratio whose numerator sum r x u cancels for near-uniform flow:
    # its error is measured on the scale |U|/R of an angular velocity
    Uscale = max(np.abs(Po["U"]).max(), np.abs(Po["U_prev"]).max(), 1e-30)
    Rmin = min(p["a"] for p in parts)
    for key in ("U", "U_prev"):
        assert np.abs(Pg[key] - Po[key]).max() / Uscale < tol * 10, key
    for key in ("omega", "omega_prev"):
        assert np.abs(Pg[key] - Po[key]).max() * Rmin / Uscale < tol * 10, key
    assert np.abs(Pg["theta"] - Po["theta"]).max() < 1e-12
    return sim, ora, rg, ro


def test_particles_random_state_2d():
    """The whole step with two disks and an ellipse in contact, walls in y,
    periodic x, from a random state (eq. 9-22, Algorithm 1)."""
    banner("particles random 2d")
    cfg = dict(lattice="D2Q9", n=(45, 37, 1), periodic=(1, 0, 0), tau=0.7, g=(0.0, -5e-4, 0.0), eps_p=2.0,
               eps_w=1.0, delta=1.0)
    parts = [dict(shape="disk", rho_s=1.5, a=4.0, x=(10.2, 14.7, 0.0)),
             dict(shape="disk", rho_s=1.2, a=5.0, x=(19.0, 17.1, 0.0)),
             dict(shape="ellipse", rho_s=1.4, a=6.0, b=3.0, x=(40.5, 6.3, 0.0), theta=0.9)]
    f0 = random_state((1, 37, 45), 9, 1e-3, seed=3)
    # boxes wider than the period less a wavefront: sums in a kernel of their own
    _, _, rg, _ = _compare_run(cfg, parts, 30, f0=f0, fused=False)
    assert np.abs(rg[:, :, 10:12]).max() > 1e-6  # contact forces acted


@pytest.mark.parametrize("nx,storage", [(17, "f64"), (20, "f32")])
def test_particles_3d(nx, storage):
    """Two spheres in D3Q19; in FP32 storage with nx a multiple of 4 the rows
    are staged through LDS."""
    banner(f"particles 3d nx={nx} {storage}")
    cfg = dict(lattice="D3Q19", n=(nx, 15, 19), periodic=(0, 1, 0), tau=0.65, g=(0.0, 0.0, -5e-4))
    parts = [dict(shape="sphere", rho_s=1.6, a=3.0, x=(7.0, 7.5, 9.0)),
             dict(shape="sphere", rho_s=1.3, a=3.5, x=(12.2, 8.0, 12.4))]
    f0 = random_state((19, 15, nx), 19, 1e-3, seed=4)
    if storage == "f64":
        _compare_run(cfg, parts, 12, f0=f0)
    else:
        _compare_run(cfg, parts, 12, f0=f0.astype(np.float32).astype(np.float64), storage="f32", tol=5e-6,
                     xtol=1e-7)


def test_floating_disk_workload():
    """The floating-disk workload in full (200x400, 2000 steps, FP64)."""
    banner("floating disk 200x400 2000 steps")
    cfg, parts, steps, _ = workload("floating_disk_200x400")
    sim, ora, rg, ro = _compare_run(cfg, parts, steps)
    assert np.abs(rg[:, 0, 4:6] - [0.02, 0.0]).max() <= 1e-3 * 0.02


def test_small_sedimentation_contacts():
    """Eight bodies settling in a closed 64x96 box with strong gravity, so that
    particle-particle and particle-wall forces act (sec. 2.3)."""
    banner("small sedimentation contacts")
    kinds = [("disk", 5.0, 5.0)] * 5 + [("ellipse", 6.0, 3.0)] * 3
    # gaps of 0.3 l.u. < delta: several pairs start inside the collision range
    parts = place((64, 96), kinds, seed=7, rho_range=(1.2, 1.8), upper_axis=1, gap=0.3, margin=0.3)
    cfg = dict(lattice="D2Q9", n=(64, 96, 1), periodic=(0, 0, 0), tau=0.6, g=(0.0, -2e-4, 0.0))
    _, _, rg, _ = _compare_run(cfg, parts, 400, xtol=1e-11)
    assert (np.abs(rg[:, :, 10:12]).max(axis=(1, 2)) > 0).sum() > 100  # contact forces in most steps


def test_determinism_bitwise():
    banner("determinism")
    cfg = dict(lattice="D2Q9", n=(80, 64, 1), periodic=(0, 0, 0), tau=0.6, g=(0.0, -1e-4, 0.0))
    parts = place((80, 64), [("disk", 5.0, 5.0)] * 4, seed=9, rho_range=(1.2, 1.5), upper_axis=1)
    out = []
    for _ in range(2):
        sim = lbm.Simulation(cfg, parts, storage="f32")
        sim.step(50)
        out.append((sim.populations(), sim.particles()["X"]))
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])


def test_unstable_sentinel():
    banner("sentinel")
    cfg = dict(lattice="D2Q9", n=(40, 30, 1), periodic=(1, 1, 0), tau=0.8, u0=(0.35, 0.0))
    sim = lbm.Simulation(cfg, [], storage="f32")
    sim.step(2)
    with pytest.raises(lbm.LbmError) as e:
        sim.sync()
    assert e.value.code == lbm.LBM_EUNSTABLE


def test_particle_validation():
    banner("validation")
    cfg = dict(lattice="D2Q9", n=(30, 60, 1), periodic=(1, 0, 0), tau=0.8)
    sim = lbm.Simulation(cfg, [], storage="f32", max_particles=2)
    for bad in ([dict(shape="disk", rho_s=1.2, a=5.0, x=(15.0, 3.0, 0.0))],       # crosses the y wall
                [dict(shape="sphere", rho_s=1.2, a=5.0, x=(15.0, 30.0, 0.0))],    # 3D shape on D2Q9
                [dict(shape="disk", rho_s=1.2, a=5.0, x=(15.0, 30.0, 0.0))] * 3,  # over capacity
                [dict(shape="disk", rho_s=1.2, a=14.0, x=(15.0, 30.0, 0.0))],     # a + 2 >= n/2 on the x period
                [dict(shape="ellipse", rho_s=1.2, a=3.0, b=4.0, x=(15.0, 30.0, 0.0))],  # b > a
                [dict(shape="disk", rho_s=-1.0, a=5.0, x=(15.0, 30.0, 0.0))]):    # negative density
        with pytest.raises(lbm.LbmError) as e:
            sim.set_particles(bad)
        assert e.value.code == lbm.LBM_EINVAL
    sim.set_particles([dict(shape="disk", rho_s=1.2, a=5.0, x=(15.0, 30.0, 0.0))])  # a valid one still works
    sim.step(2)
    sim.sync()


def test_substeps_k3():
    """Algorithm 1 with K = 3 sub-steps (all particles integrated together)."""
    banner("substeps K=3")
    kinds = [("disk", 5.0, 5.0)] * 5 + [("ellipse", 6.0, 3.0)] * 3
    parts = place((64, 96), kinds, seed=7, rho_range=(1.2, 1.8), upper_axis=1, gap=0.3, margin=0.3)
    cfg = dict(lattice="D2Q9", n=(64, 96, 1), periodic=(0, 0, 0), tau=0.6, g=(0.0, -2e-4, 0.0), K=3)
    _, _, rg, _ = _compare_run(cfg, parts, 200, xtol=1e-11)
    assert (np.abs(rg[:, :, 10:12]).max(axis=(1, 2)) > 0).sum() > 20


def test_many_bodies_contacts():
    """80 bodies, more than the one-workgroup particle kernel takes: the sums
    and Algorithm 1 run one workgroup per particle; contacts, x periodic, even
    width (two nodes per indicator claim)."""
    banner("many bodies 128x160")
    kinds = [("disk", 3.0, 3.0)] * 56 + [("ellipse", 4.0, 2.0)] * 24
    parts = place((128, 160), kinds, seed=11, rho_range=(1.2, 1.8), upper_axis=1, gap=0.3, margin=0.3)
    cfg = dict(lattice="D2Q9", n=(128, 160, 1), periodic=(1, 0, 0), tau=0.6, g=(0.0, -2e-4, 0.0))
    _, _, rg, _ = _compare_run(cfg, parts, 150, xtol=1e-11, fused=True)
    assert (np.abs(rg[:, :, 10:12]).max(axis=(1, 2)) > 0).sum() > 50


def test_fused_sums_periodic_wrap_2d():
    """Momentum sums taken by the lattice kernel, with scan boxes wrapping both
    periodic axes and a ragged last wavefront in x (200 = 3 x 64 + 8)."""
    banner("fused sums wrap 2d 200x128")
    cfg = dict(lattice="D2Q9", n=(200, 128, 1), periodic=(1, 1, 0), tau=0.7, g=(0.0, -3e-4, 0.0))
    parts = [dict(shape="disk", rho_s=1.5, a=6.0, x=(1.5, 60.0, 0.0)),
             dict(shape="disk", rho_s=1.3, a=5.0, x=(197.2, 20.3, 0.0)),
             dict(shape="ellipse", rho_s=1.4, a=7.0, b=3.5, x=(100.4, 1.2, 0.0), theta=0.4),
             dict(shape="disk", rho_s=1.6, a=4.0, x=(63.6, 126.5, 0.0)),
             dict(shape="disk", rho_s=1.2, a=4.5, x=(140.0, 70.0, 0.0))]
    f0 = random_state((1, 128, 200), 9, 1e-3, seed=21)
    _compare_run(cfg, parts, 40, f0=f0, fused=True)


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_fused_sums_periodic_wrap_3d(storage):
    """D3Q19 with every axis periodic, spheres wrapping each of them, a ragged
    last wavefront (132 = 2 x 64 + 4); in FP32 the rows are staged through
    LDS."""
    banner(f"fused sums wrap 3d 132x32x32 {storage}")
    cfg = dict(lattice="D3Q19", n=(132, 32, 32), periodic=(1, 1, 1), tau=0.65, g=(0.0, 0.0, -4e-4))
    parts = [dict(shape="sphere", rho_s=1.6, a=4.0, x=(1.0, 8.0, 8.0)),
             dict(shape="sphere", rho_s=1.3, a=3.5, x=(129.9, 24.0, 30.9)),
             dict(shape="sphere", rho_s=1.4, a=4.0, x=(65.0, 0.7, 16.0)),
             dict(shape="sphere", rho_s=1.5, a=3.0, x=(64.0, 20.0, 1.0))]
    f0 = random_state((32, 32, 132), 19, 1e-3, seed=22)
    if storage == "f64":
        _compare_run(cfg, parts, 8, f0=f0, fused=True)
    else:
        _compare_run(cfg, parts, 8, f0=f0.astype(np.float32).astype(np.float64), storage="f32", tol=5e-6,
                     xtol=1e-7, fused=True)


def test_many_bodies_substeps_k3():
    """The many-body path with K = 3 (one-workgroup sub-step integration, then
    the indicator), odd width (one node per claim)."""
    banner("many bodies K=3 127x160")
    kinds = [("disk", 3.0, 3.0)] * 70
    parts = place((127, 160), kinds, seed=13, rho_range=(1.2, 1.8), upper_axis=1, gap=0.3, margin=0.3)
    cfg = dict(lattice="D2Q9", n=(127, 160, 1), periodic=(0, 0, 0), tau=0.6, g=(0.0, -2e-4, 0.0), K=3)
    _, _, rg, _ = _compare_run(cfg, parts, 100, xtol=1e-11)
    assert (np.abs(rg[:, :, 10:12]).max(axis=(1, 2)) > 0).sum() > 20


def test_large_boxes_3d():
    """Six spheres of radius 6: few bodies, but scan boxes too large for the
    one-workgroup kernel; odd width, z periodic."""
    banner("large boxes 3d 41x48x40")
    parts = place((41, 48, 40), [("sphere", 6.0, 6.0)] * 6, seed=12, rho_range=(1.2, 1.6), upper_axis=1, gap=0.5,
                  margin=0.3)
    cfg = dict(lattice="D3Q19", n=(41, 48, 40), periodic=(0, 0, 1), tau=0.65, g=(0.0, -5e-4, 0.0))
    f0 = random_state((40, 48, 41), 19, 1e-3, seed=6)
    _compare_run(cfg, parts, 10, f0=f0)


TINY_2D = [((1, 1, 1), p) for p in ((0, 0, 0), (1, 1, 0))] + \
    [(n, p) for n in ((1, 5, 1), (5, 1, 1), (2, 2, 1), (3, 2, 1)) for p in ((0, 0, 0), (1, 0, 0), (0, 1, 0), (1, 1, 0))]
TINY_3D = [(n, p) for n in ((1, 1, 4), (2, 3, 1), (4, 1, 2), (4, 2, 3)) for p in ((0, 0, 0), (1, 1, 1), (1, 0, 1))]


@pytest.mark.parametrize("kind,n,periodic", [("D2Q9", n, p) for n, p in TINY_2D] + [("D3Q19", n, p) for n, p in TINY_3D])
def test_fluid_step_tiny_axes(kind, n, periodic):
    """Axes of one to five nodes, walls or periodic: a pulled source wraps onto
    the node itself or bounces on both sides of it.  FP64 storage within 1e-12
    of the oracle; D3Q19 rows of four nodes in FP32 storage (the LDS-staged
    kernel, whose halo elements wrap or bounce inside the row) to FP32
    rounding."""
    banner(f"fluid tiny axes {kind} {n} {periodic}")
    cfg = dict(lattice=kind, n=n, periodic=periodic, tau=0.7, fluid_accel=(2e-5, -1e-5, 3e-6 if kind == "D3Q19" else 0.0))
    Q = 9 if kind == "D2Q9" else 19
    f0 = random_state((n[2], n[1], n[0]), Q, 2e-3, seed=13)
    storages = ["f64"] + (["f32"] if kind == "D3Q19" and n[0] % 4 == 0 else [])
    for storage in storages:
        f = f0 if storage == "f64" else f0.astype(np.float32).astype(np.float64)
        sim, ora = pair(cfg, [], storage=storage, f0=f)
        for steps in (1, 5):
            sim.step(steps)
            ora.step(steps)
            e = rel(sim.populations(), ora.f())
            assert e < (TOL if storage == "f64" else 5e-6), (storage, steps, e)
        ug, pg, _ = sim.fields()
        uo, po, _ = ora.fields()
        tol = TOL if storage == "f64" else 5e-6
        assert rel(ug, uo) < tol * 10 and rel(pg, po) < tol * 10
        sim.close()
