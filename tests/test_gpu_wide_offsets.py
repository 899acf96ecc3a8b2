"""Lattices with Q N >= 2^31: the lattice kernel with 64-bit population offsets.

Node indices stay 32-bit (d N < 2^31); the population offsets q N + node of
the pull and of the stores are 64-bit once Q N reaches 2^31.  Two checks:

* the 64-bit kernel on small lattices (selected with LBM_WIDE_OFFSETS=1 in the
  environment when the context is created): the same bits as the 32-bit
  kernels over runs with bodies in contact, walls and periodic axes, in every
  storage type, D2Q9 and D3Q19, and in FP64 within 1e-12 of the oracle;
* lattices past the 32-bit range (D2Q9 16384 x 16384, Q N = 2.42e9; D3Q19
  512^3, Q N = 2.55e9; at the top of the range D2Q9 24576 x 24576 in FP64,
  whose store byte offsets pass 2^32, and D3Q19 1022 x 1024 x 682 with d N
  just below 2^31): uniform flow along a periodic x between walls stays
  independent of the periodic coordinates, so after three steps every sampled
  column equals that of a lattice four nodes wide (one deep) with the same
  wall-normal rows -- against the oracle within 1e-12 in FP64, bit for bit
  against the small GPU run in FP32 (in D3Q19 the LDS-staged kernel) and FP16.
"""
import os

import numpy as np
import pytest

from gpu_common import banner, rel
from oracle import oracle as O
from paper_2511_01629_amd import lbm

pytestmark = pytest.mark.gpu


def _run(cfg, parts, storage, steps, wide):
    if wide:
        os.environ["LBM_WIDE_OFFSETS"] = "1"
    try:
        sim = lbm.Simulation(cfg, parts, storage=storage)
    finally:
        os.environ.pop("LBM_WIDE_OFFSETS", None)
    rec = sim.step_record(steps)
    f = sim.populations()
    u, p, own = sim.fields()
    sim.close()
    return rec, f, u, p, own


SMALL = {
    # nx = 30 in D3Q19: not a multiple of four, so FP32 takes the one-node-per-lane kernel too
    "D2Q9": (dict(lattice="D2Q9", n=(50, 44, 1), periodic=(1, 0, 0), tau=0.7, g=(0.0, -1e-4, 0.0)),
             [dict(shape="disk", rho_s=1.5, a=6.0, x=(17.0, 20.0, 0.0)),
              dict(shape="ellipse", rho_s=1.3, a=7.0, b=3.5, x=(31.0, 22.5, 0.0), theta=0.4)]),
    "D3Q19": (dict(lattice="D3Q19", n=(30, 26, 28), periodic=(0, 1, 0), tau=0.7, g=(0.0, 0.0, -1e-4)),
              [dict(shape="sphere", rho_s=1.5, a=5.0, x=(10.0, 12.0, 14.0)),
               dict(shape="sphere", rho_s=1.2, a=5.5, x=(21.5, 13.0, 14.5))]),
}


@pytest.mark.parametrize("storage", ["f64", "f32", "f16", "bf16"])
@pytest.mark.parametrize("kind", ["D2Q9", "D3Q19"])
def test_wide_offsets_same_bits_on_small_lattices(kind, storage):
    cfg, parts = SMALL[kind]
    steps = 25
    banner(f"64-bit offsets vs 32-bit {kind} {storage} {steps} steps")
    rn, fn, un, pn, on = _run(cfg, parts, storage, steps, wide=False)
    rw, fw, uw, pw, ow = _run(cfg, parts, storage, steps, wide=True)
    assert np.array_equal(rn, rw)
    assert np.array_equal(fn, fw) and np.array_equal(un, uw) and np.array_equal(pn, pw)
    assert np.array_equal(on, ow)
    if storage == "f64":
        ora = O.Oracle(cfg, parts)
        ro = ora.step(steps, record=True)
        uo, _, own_o = ora.fields()
        assert np.array_equal(ow, own_o)
        assert rel(uw, uo) < 1e-12
        assert np.abs(rw[:, :, 0:3] - ro[:, :, 0:3]).max() < 1e-10


WIDE = {
    # name: (lattice, n, periodic, the small lattice with the same rows, sampled (x, y))
    "D2Q9": ("D2Q9", (16384, 16384, 1), (1, 0, 0), (4, 16384, 1),
             [(0, 0), (1, 0), (3, 16383), (4097, 8191), (16383, 16383), (9000, 12000)]),
    "D3Q19": ("D3Q19", (512, 512, 512), (1, 1, 0), (4, 1, 512), [(0, 0), (3, 511), (257, 130), (511, 0), (511, 511)]),
    # the top of the range: byte offsets of the FP64 stores past 2^32 (604 M nodes), and
    # d N just below 2^31 in D3Q19 (714 M nodes, Q N = 1.36e10)
    "D2Q9-top": ("D2Q9", (24576, 24576, 1), (1, 0, 0), (4, 24576, 1),
                 [(0, 0), (5, 24575), (12288, 12288), (24575, 24575), (20000, 23000)]),
    "D3Q19-top": ("D3Q19", (1022, 1024, 682), (1, 1, 0), (4, 1, 682),
                  [(0, 0), (3, 1023), (511, 700), (1021, 0), (1021, 1023)]),
}


@pytest.mark.parametrize("case,storage", [("D2Q9", "f32"), ("D2Q9", "f16"), ("D3Q19", "f64"), ("D3Q19", "f32"),
                                          ("D3Q19", "f16"), ("D2Q9-top", "f64"), ("D3Q19-top", "f16")])
def test_lattice_past_32bit_population_offsets(case, storage):
    import torch

    kind, n, per, n_small, pts = WIDE[case]
    Q = 9 if kind == "D2Q9" else 19
    d = 2 if kind == "D2Q9" else 3
    N = n[0] * n[1] * n[2]
    assert Q * N >= 2 ** 31 and d * N < 2 ** 31
    banner(f"lattice past 2^31 population offsets {kind} {n} {storage}")
    cfg = dict(lattice=kind, n=n, periodic=per, tau=0.8, u0=(0.02, 0.0, 0.0))
    small_cfg = dict(cfg, n=n_small)
    big = lbm.Simulation(cfg, [], storage=storage)
    big.step(3)
    u, p, _ = big.fields()
    big.close()
    del big
    torch.cuda.empty_cache()
    # (nz, ny, nx) fields: in 2D the sampled (x, y) is a column of x; in 3D a z-column at (x, y)
    if d == 2:
        ub = np.stack([u[0, y, x] for x, y in pts])
        pb = np.stack([p[0, y, x] for x, y in pts])
    else:
        ub = np.stack([u[:, y, x] for x, y in pts])
        pb = np.stack([p[:, y, x] for x, y in pts])
    del u, p
    if storage == "f64":
        ora = O.Oracle(small_cfg, [])
        ora.step(3)
        us, ps, _ = ora.fields()
    else:
        small = lbm.Simulation(small_cfg, [], storage=storage)
        small.step(3)
        us, ps, _ = small.fields()
        small.close()
    if d == 2:
        uo = np.stack([us[0, y, x % 4] for x, y in pts])
        po = np.stack([ps[0, y, x % 4] for x, y in pts])
    else:
        uo = np.stack([us[:, y % n_small[1], x % 4] for x, y in pts])
        po = np.stack([ps[:, y % n_small[1], x % 4] for x, y in pts])
    if storage == "f64":
        assert np.abs(ub - uo).max() / np.abs(uo).max() < 1e-12
        assert np.abs(pb - po).max() / max(np.abs(po).max(), 1e-30) < 1e-11
    else:
        assert np.array_equal(ub, uo) and np.array_equal(pb, po)


def test_past_32bit_offsets_differentiated_run_refused_slabs_split():
    """The lattice adjoint keeps 32-bit population offsets: on a lattice with
    Q N >= 2^31 the differentiated run is refused with EINVAL.  The slab step
    keeps them within each slab buffer: one slab of 16384 x 16386 rows is
    refused, two slabs run and give the unsplit step's bits."""
    import ctypes as C

    import torch

    cfg = dict(lattice="D2Q9", n=(16384, 16384, 1), periodic=(1, 0, 0), tau=0.8, g=(0.0, -1e-5, 0.0))
    parts = [dict(shape="disk", rho_s=1.5, a=8.0, x=(100.0, 200.0, 0.0)),
             dict(shape="disk", rho_s=1.3, a=8.0, x=(8000.0, 8191.5, 0.0))]  # across the slab cut
    banner("Q N >= 2^31: differentiated run refused, slab step split in two")
    ref = lbm.Simulation(cfg, parts, storage="f16")
    ref.step(2)
    u0, p0, o0 = ref.fields()
    P0 = ref.particles()
    ref.close()
    del ref
    torch.cuda.empty_cache()
    sim = lbm.Simulation(cfg, parts, storage="f16")
    fb, bb = C.c_size_t(), C.c_size_t()
    assert sim.lib.lbm_grad_workspace_size(sim.ctx, 10, 5, C.byref(fb), C.byref(bb)) == lbm.LBM_EINVAL
    assert sim.lib.lbm_forward_checkpointed(sim.ctx, 10, 5) == lbm.LBM_EINVAL
    assert sim.lib.lbm_step_slabs(sim.ctx, 1, 1) == lbm.LBM_EINVAL
    sim.step_slabs(2, 2)
    u1, p1, o1 = sim.fields()
    P1 = sim.particles()
    sim.close()
    assert np.array_equal(o0, o1) and np.array_equal(u0, u1) and np.array_equal(p0, p1)
    for k in ("X", "theta", "U", "omega"):
        assert np.array_equal(P0[k], P1[k]), k
