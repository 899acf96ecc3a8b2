"""The lattice cut into slabs on one GPU (lbm_step_slabs: per-slab buffers with
halo rows exchanged by explicit copies, per-slab momentum-sum tables merged
before Algorithm 1) against the unsplit step: bit for bit, in D2Q9 and D3Q19,
every storage type, walls or a periodic split axis, moving walls, the fused
sums and the separate sums kernel, the fractional indicator, 2 to 5 slabs (the
one-GPU part of a multi-GPU slab decomposition)."""
import numpy as np
import pytest

from gpu_common import banner
from paper_2511_01629_amd import lbm
from paper_2511_01629_amd.workloads import place, random_state

pytestmark = pytest.mark.gpu


def _same(a, b):
    assert np.array_equal(a.populations(), b.populations())
    Pa, Pb = a.particles(), b.particles()
    for key in ("X", "theta", "U", "omega", "U_prev", "omega_prev", "A", "N"):
        assert np.array_equal(Pa[key], Pb[key]), key
    ua, pa, oa = a.fields()
    ub, pb, ob = b.fields()
    assert np.array_equal(ua, ub) and np.array_equal(pa, pb) and np.array_equal(oa, ob)


def _contacts(n=(64, 96), periodic=(0, 0, 0)):
    kinds = [("disk", 5.0, 5.0)] * 5 + [("ellipse", 6.0, 3.0)] * 3
    parts = place(n, kinds, seed=7, rho_range=(1.2, 1.8), upper_axis=1, gap=0.3, margin=0.3)
    cfg = dict(lattice="D2Q9", n=n + (1,), periodic=periodic, tau=0.6, g=(0.0, -2e-4, 0.0))
    return cfg, parts


def _run_pair(cfg, parts, storage, steps, nslabs, f0=None, fused=None):
    a = lbm.Simulation(cfg, parts, storage=storage)
    b = lbm.Simulation(cfg, parts, storage=storage)
    if f0 is not None:
        for s in (a, b):
            s.set_populations(f0)
            if parts:
                s.set_particles(parts)
    if fused is not None:
        a.profile(True)
        a.step(1)
        assert (a.profile_read()["reduce_clear"][1] == 0) == fused
        a.profile(False)
        b.step(1)
    a.step(steps)
    b.step_slabs(steps, nslabs)
    _same(a, b)
    # and onward: the unsplit step continues from the slabs' state
    a.step(5)
    b.step(5)
    _same(a, b)
    return a


@pytest.mark.parametrize("storage", ["f64", "f32", "f16", "bf16"])
@pytest.mark.parametrize("nslabs", [2, 3])
def test_slabs_contacts_2d(storage, nslabs):
    banner(f"slabs 2d contacts {storage} {nslabs}")
    cfg, parts = _contacts()
    _run_pair(cfg, parts, storage, 60, nslabs, fused=True)  # bodies start inside the collision range


@pytest.mark.parametrize("nslabs", [2, 5])
def test_slabs_periodic_split_axis(nslabs):
    """A periodic split axis: the first and last slabs exchange halos around
    the period; bodies whose scan boxes wrap it."""
    banner(f"slabs periodic {nslabs}")
    cfg = dict(lattice="D2Q9", n=(128, 64, 1), periodic=(1, 1, 0), tau=0.7, g=(0.0, -3e-4, 0.0))
    parts = [dict(shape="disk", rho_s=1.5, a=6.0, x=(20.5, 1.5, 0.0)),
             dict(shape="ellipse", rho_s=1.3, a=7.0, b=3.5, x=(80.4, 62.7, 0.0), theta=0.4),
             dict(shape="disk", rho_s=1.4, a=5.0, x=(60.0, 30.2, 0.0))]
    f0 = random_state((1, 64, 128), 9, 1e-3, seed=31)
    _run_pair(cfg, parts, "f64", 40, nslabs, f0=f0)


def test_slabs_separate_sums_kernel():
    """Boxes too wide for the slot layout of a short periodic x axis: the
    momentum sums run as a kernel of their own, reading the shared
    solid-node velocity the slab kernels write."""
    banner("slabs unfused")
    cfg = dict(lattice="D2Q9", n=(45, 37, 1), periodic=(1, 0, 0), tau=0.7, g=(0.0, -5e-4, 0.0))
    parts = [dict(shape="disk", rho_s=1.5, a=4.0, x=(10.2, 14.7, 0.0)),
             dict(shape="disk", rho_s=1.2, a=5.0, x=(19.0, 17.1, 0.0)),
             dict(shape="ellipse", rho_s=1.4, a=6.0, b=3.0, x=(40.5, 6.3, 0.0), theta=0.9)]
    f0 = random_state((1, 37, 45), 9, 1e-3, seed=3)
    _run_pair(cfg, parts, "f64", 30, 2, f0=f0, fused=False)


def test_slabs_moving_walls():
    banner("slabs couette")
    Uw = 0.02
    cfg = dict(lattice="D2Q9", n=(96, 48, 1), periodic=(1, 0, 0), tau=0.8,
               wall_velocity=[[(0.0, 0.0, 0.0)] * 2, [(-Uw / 2, 0.0, 0.0), (Uw / 2, 0.0, 0.0)], [(0.0, 0.0, 0.0)] * 2])
    parts = [dict(shape="disk", rho_s=1.0, a=8.0, x=(40.0, 20.3, 0.0))]
    _run_pair(cfg, parts, "f64", 50, 3)


@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
def test_slabs_3d(storage):
    """D3Q19 split along z (in FP32 the unsplit step stages rows through LDS;
    the slab kernel is one node per lane: same arithmetic, same bits)."""
    banner(f"slabs 3d {storage}")
    cfg = dict(lattice="D3Q19", n=(32, 20, 24), periodic=(0, 1, 0), tau=0.65, g=(0.0, 0.0, -5e-4))
    parts = [dict(shape="sphere", rho_s=1.6, a=4.0, x=(10.0, 9.5, 12.0)),
             dict(shape="sphere", rho_s=1.3, a=4.5, x=(20.2, 10.0, 13.4))]
    f0 = random_state((24, 20, 32), 19, 1e-3, seed=4).astype(np.float32).astype(np.float64)
    _run_pair(cfg, parts, storage, 20, 2, f0=f0)


@pytest.mark.parametrize("lattice", ["D2Q9", "D3Q19"])
def test_slabs_fractional_indicator(lattice):
    """The fractional indicator (weights from the global node coordinates in
    every slab kernel, sums in the separate kernel): bit for bit."""
    banner(f"slabs fractional {lattice}")
    if lattice == "D2Q9":
        cfg = dict(lattice="D2Q9", n=(45, 37, 1), periodic=(1, 0, 0), tau=0.7, g=(0.0, -5e-4, 0.0), fractional=1)
        parts = [dict(shape="disk", rho_s=1.5, a=4.0, x=(10.2, 14.7, 0.0)),
                 dict(shape="disk", rho_s=1.2, a=5.0, x=(19.6, 17.1, 0.0)),
                 dict(shape="disk", rho_s=1.4, a=4.5, x=(43.2, 6.3, 0.0))]
        f0 = random_state((1, 37, 45), 9, 1e-3, seed=3)
        _run_pair(cfg, parts, "f64", 30, 3, f0=f0, fused=False)
    else:
        cfg = dict(lattice="D3Q19", n=(17, 15, 19), periodic=(0, 1, 0), tau=0.65, g=(0.0, 0.0, -5e-4), fractional=1)
        parts = [dict(shape="sphere", rho_s=1.6, a=3.0, x=(7.0, 7.5, 9.0)),
                 dict(shape="sphere", rho_s=1.3, a=3.5, x=(12.2, 8.0, 12.4))]
        _run_pair(cfg, parts, "f32", 20, 2, fused=False)


def test_slabs_fluid_only_and_rejections():
    banner("slabs fluid + rejections")
    cfg = dict(lattice="D2Q9", n=(70, 33, 1), periodic=(0, 1, 0), tau=0.7, fluid_accel=(1e-5, 0.0, 0.0))
    f0 = random_state((1, 33, 70), 9, 1e-3, seed=8)
    _run_pair(cfg, [], "f32", 25, 4, f0=f0)
    sim = lbm.Simulation(cfg, [], storage="f32")
    for bad in (0, 34, 65):
        with pytest.raises(lbm.LbmError) as e:
            sim.step_slabs(1, bad)
        assert e.value.code == lbm.LBM_EINVAL
    forcing = lbm.Simulation(dict(cfg, rigid_beta=0.5), [], storage="f32")
    with pytest.raises(lbm.LbmError):
        forcing.step_slabs(1, 2)
