"""Parity at the full workload sizes, in the launch configuration bench.py
times (the library picks the same kernels; only the step count is short).

The oracle runs the same steps; the indicator is compared on every node, the
particle state in full, the populations on a seeded sample of nodes plus every
solid node.  FP64 storage: within 1e-12 relative; FP32 storage: within the
bound of a few steps of FP32 rounding.
"""
import numpy as np
import pytest

from gpu_common import banner, check_owner, pair, rel
from oracle import oracle as O
from paper_2511_01629_amd import lbm
from paper_2511_01629_amd.workloads import workload

pytestmark = pytest.mark.gpu


def _compare(name, storage, steps, tol, nsample=200_000, u_atol=0.0, f_atol=0.0, fractional=False):
    cfg, parts, _, _ = workload(name)
    if fractional:  # the same workload with the fractional indicator
        cfg = dict(cfg, fractional=1)
    banner(f"full size {name} {storage} {steps} steps" + (" fractional" if fractional else ""))
    sim, ora = pair(cfg, parts, storage=storage)
    rg = sim.step_record(steps)
    ro = ora.step(steps, record=True)
    # particle records of every step
    if fractional:  # sums of the FP64 weights, in another order
        assert np.abs(rg[:, :, 13] - ro[:, :, 13]).max() <= 1e-13 * ro[:, :, 13].max()
    else:
        assert np.array_equal(rg[:, :, 13], ro[:, :, 13])  # node counts
    assert np.abs(rg[:, :, 0:3] - ro[:, :, 0:3]).max() <= tol * np.abs(ro[:, :, 0:3]).max()
    Usc = np.abs(ro[:, :, 4:7]).max()
    if Usc > 0:
        assert np.abs(rg[:, :, 4:7] - ro[:, :, 4:7]).max() <= max(10 * tol * Usc, u_atol)
    # indicator on every node (boundary ties allowed)
    _, _, og = sim.fields()
    uo, po, oo = ora.fields()
    Po = ora.particles()
    if fractional:
        assert np.array_equal(og, oo)  # the band, node for node
    else:
        check_owner(og, oo, parts, Po, cfg.get("periodic", (0, 0, 0)))
    # populations on a sample of nodes and on all solid nodes
    fg, fo = sim.populations(), ora.f()
    flat_g = fg.reshape(-1, fg.shape[-1])
    flat_o = fo.reshape(-1, fo.shape[-1])
    rng = np.random.default_rng(2024)
    idx = np.unique(np.concatenate([rng.integers(0, flat_o.shape[0], nsample), np.flatnonzero(oo.reshape(-1) >= 0)]))
    e = rel(flat_g[idx], flat_o[idx])
    ea = float(np.abs(flat_g[idx] - flat_o[idx]).max())
    print(f"[measured] {name} {storage}: population max rel err {e:.3e}, abs {ea:.3e} on {idx.size} nodes",
          flush=True)
    assert e < tol or ea <= f_atol
    return sim, ora


def test_fullsize_sedimentation_f64():
    _compare("sedimentation_2048x4096", "f64", 3, 1e-12)


def test_fullsize_sedimentation_f32():
    _compare("sedimentation_2048x4096", "f32", 3, 2e-6)


def test_fullsize_sedimentation_f16():
    """FP16 storage right after the start: the bodies move at ~1e-6 and the
    populations they set in motion (~1e-7) sit among FP16 subnormals (spacing
    6e-8), so populations and velocities are compared with absolute bounds of a
    few FP16 quanta."""
    _compare("sedimentation_2048x4096", "f16", 2, 2e-3, u_atol=4e-7, f_atol=2.4e-7)


def test_fullsize_spheres_f32():
    _compare("spheres_256x256x512", "f32", 2, 2e-6, nsample=100_000)


def test_fullsize_adjoint_workload_f64():
    _compare("adjoint_512x1024", "f64", 100, 1e-12)


def test_fullsize_fractional_spheres_f32():
    """The fractional indicator at full size: the 64 spheres of 256x256x512
    (the bench's fractional mode), FP32 storage."""
    _compare("spheres_256x256x512", "f32", 2, 2e-6, nsample=100_000, fractional=True)


def test_fullsize_fractional_adjoint_workload_f64():
    _compare("adjoint_512x1024", "f64", 100, 1e-12, fractional=True)


def test_fullsize_disk_settling_f64():
    _compare("disk_settling_400x1600", "f64", 100, 1e-12)


LARGEST = {
    # lattice: (n, periodic, the small lattice with the same rows, sampled (x, y))
    "D2Q9": ((16384, 14563, 1), (1, 0, 0), (4, 14563, 1), [(0, 0), (1, 0), (3, 0), (4097, 0), (16383, 0)]),
    "D3Q19": ((512, 512, 431), (1, 1, 0), (4, 1, 431), [(0, 0), (3, 511), (257, 130), (511, 0), (511, 511)]),
}


@pytest.mark.parametrize("kind,storage", [("D2Q9", "f64"), ("D2Q9", "f16"), ("D3Q19", "f64"), ("D3Q19", "f32"),
                                          ("D3Q19", "f16")])
def test_largest_lattice_index_range(kind, storage):
    """The largest lattices with 32-bit population offsets (Q N just below 2^31: D2Q9
    16384 x 14563, D3Q19 512 x 512 x 431): every population offset q N + node
    sits at the top of the 32-bit index range.  Uniform flow along a periodic
    x between walls (in y, or in z with y periodic) stays independent of the
    periodic coordinates, so after three steps every sampled column equals the
    column of a lattice four nodes wide (one deep) with the same wall-normal
    rows: to the oracle within 1e-12 in FP64, and bit for bit to the small GPU
    run in FP32 (the LDS-staged D3Q19 kernel) and FP16 storage (the same node
    arithmetic)."""
    import torch

    n, per, n_small, pts = LARGEST[kind]
    Q = 9 if kind == "D2Q9" else 19
    assert Q * n[0] * n[1] * n[2] < 2 ** 31
    banner(f"largest lattice {kind} {n} {storage}")
    cfg = dict(lattice=kind, n=n, periodic=per, tau=0.8, u0=(0.02, 0.0, 0.0))
    small_cfg = dict(cfg, n=n_small)
    big = lbm.Simulation(cfg, [], storage=storage)
    big.step(3)
    u, p, _ = big.fields()
    big.close()
    del big
    torch.cuda.empty_cache()
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
    uo = np.stack([us[:, y % n_small[1], x % 4] for x, y in pts])
    po = np.stack([ps[:, y % n_small[1], x % 4] for x, y in pts])
    if storage == "f64":
        assert np.abs(ub - uo).max() / np.abs(uo).max() < 1e-12
        assert np.abs(pb - po).max() / max(np.abs(po).max(), 1e-30) < 1e-11
    else:
        assert np.array_equal(ub, uo) and np.array_equal(pb, po)
