"""Fractional indicator (an extension beyond the paper's binary indicator, for
gradients in the positions): a node of the band |x - X_i| < R_i + 1/2
belongs to particle i with the weight chi = min(1, R_i + 1/2 - |x - X_i|),
which multiplies its acceleration and penalization strength and weights the
momentum sums and the mass of Algorithm 1.

* GPU against the FP64 oracle: FP64 storage within 1e-12 (disks in contact
  with one across a periodic axis, K = 1 and K = 2; spheres in D3Q19), the
  band identical node for node, the weight sums N_i = sum chi to round-off;
  FP32 and FP16 storage within the bounds of the other reduced-storage tests.
* The weights matter: the same run with the binary indicator ends elsewhere.
* What the library rejects: ellipses and the rigid-velocity forcing (the
  differentiated run is covered by test_gpu_adjoint_positions.py).
"""
import numpy as np
import pytest

from gpu_common import banner, pair, rel
from oracle import oracle as O
from paper_2511_01629_amd import lbm
from paper_2511_01629_amd.workloads import random_state

pytestmark = pytest.mark.gpu


def _disks(K=1):
    cfg = dict(lattice="D2Q9", n=(45, 37, 1), periodic=(1, 0, 0), tau=0.7, g=(0.0, -5e-4, 0.0), eps_p=2.0,
               eps_w=1.0, delta=1.0, K=K, fractional=1)
    parts = [dict(shape="disk", rho_s=1.5, a=4.0, x=(10.2, 14.7, 0.0)),
             dict(shape="disk", rho_s=1.2, a=5.0, x=(19.6, 17.1, 0.0)),
             dict(shape="disk", rho_s=1.4, a=4.5, x=(43.2, 6.3, 0.0))]  # across the periodic x axis
    return cfg, parts


def _compare(cfg, parts, steps, f0=None, storage="f64", tol=1e-12, xtol=1e-12):
    sim, ora = pair(cfg, parts, storage=storage, f0=f0)
    rg = sim.step_record(steps)
    ro = ora.step(steps, record=True)
    # records: X theta U omega A N (N = sum chi)
    scaleX = max(np.abs(ro[:, :, 0:3]).max(), 1.0)
    eX = np.abs(rg[:, :, 0:3] - ro[:, :, 0:3]).max() / scaleX
    eU = rel(rg[:, :, 4:7], ro[:, :, 4:7])
    eN = np.abs(rg[:, :, 13] - ro[:, :, 13]).max() / np.abs(ro[:, :, 13]).max()
    fg, fo = sim.populations(), ora.f()
    ug, _, og = sim.fields()
    uo, _, oo = ora.fields()
    ef, eu = rel(fg, fo), rel(ug, uo)
    print(f"[measured] fractional {storage}: X {eX:.2e}, U {eU:.2e}, N {eN:.2e}, f {ef:.2e}, u {eu:.2e}", flush=True)
    assert np.array_equal(og, oo)  # the band, node for node
    assert ro[:, :, 13].min() > 0 and np.any(ro[:, :, 13] != np.round(ro[:, :, 13]))  # weight sums, not counts
    assert eX < xtol and eU < tol * 10 and eN < max(tol, 1e-14) and ef < tol and eu < tol
    return sim, ora, rg, ro


@pytest.mark.parametrize("K", [1, 2])
def test_fractional_parity_2d(K):
    banner(f"fractional parity 2d K={K}")
    cfg, parts = _disks(K)
    f0 = random_state((1, 37, 45), 9, 1e-3, seed=5)
    _, _, rg, _ = _compare(cfg, parts, 30, f0=f0)
    assert np.abs(rg[:, :, 10:12]).max() > 1e-6  # contact forces acted


def test_fractional_parity_3d():
    banner("fractional parity 3d")
    cfg = dict(lattice="D3Q19", n=(17, 15, 19), periodic=(0, 1, 0), tau=0.65, g=(0.0, 0.0, -5e-4), fractional=1)
    parts = [dict(shape="sphere", rho_s=1.6, a=3.0, x=(7.0, 7.5, 9.0)),
             dict(shape="sphere", rho_s=1.3, a=3.5, x=(12.2, 8.0, 12.4))]
    _compare(cfg, parts, 25)


@pytest.mark.parametrize("storage,tol,xtol", [("f32", 5e-5, 1e-6), ("f16", 5e-3, 1e-4)])
def test_fractional_reduced_storage(storage, tol, xtol):
    banner(f"fractional {storage}")
    cfg, parts = _disks()
    sim, ora = pair(cfg, parts, storage=storage)
    rg = sim.step_record(200)
    ro = ora.step(200, record=True)
    eX = np.abs(rg[:, :, 0:2] - ro[:, :, 0:2]).max()
    u_g, _, _ = sim.fields()
    u_o, _, _ = ora.fields()
    eu = np.abs(u_g - u_o).max() / np.abs(u_o).max()
    print(f"[measured] fractional {storage}: |X err| {eX:.2e} l.u., u err {eu:.2e} rel", flush=True)
    assert eX < xtol and eu < tol


def test_fractional_differs_from_binary():
    banner("fractional vs binary")
    cfg, parts = _disks()
    a = lbm.Simulation(cfg, parts, storage="f64")
    b = lbm.Simulation(dict(cfg, fractional=0), parts, storage="f64")
    ra, rb = a.step_record(50), b.step_record(50)
    assert np.abs(ra[:, :, 0:2] - rb[:, :, 0:2]).max() > 1e-8
    assert np.any(ra[-1, :, 13] != rb[-1, :, 13])


def test_fractional_rejections():
    banner("fractional rejections")
    cfg, parts = _disks()
    with pytest.raises(lbm.LbmError) as e:
        lbm.Simulation(cfg, parts + [dict(shape="ellipse", rho_s=1.3, a=5.0, b=2.5, x=(30.0, 25.0, 0.0), theta=0.4)],
                       storage="f64")
    assert e.value.code == lbm.LBM_EINVAL
    with pytest.raises(lbm.LbmError) as e:
        lbm.Simulation(dict(cfg, rigid_beta=0.5), parts, storage="f64")
    assert e.value.code == lbm.LBM_EINVAL
