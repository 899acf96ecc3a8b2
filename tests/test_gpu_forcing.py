"""Rigid-velocity forcing (an extension beyond the paper, whose constraint acts
through the stress penalization of eq. 17): on the nodes of particle i the
acceleration gains 2 beta (U_i + omega_i x r - u), with U_i, omega_i the
momentum sums of the same step (eq. 22a-b), so that the velocity entering
the collision is (1 - beta) u + beta (U_i + omega_i x r).

* GPU against the FP64 oracle: FP64 storage within 1e-12 (with and without
  the stress penalty, K = 1 and K = 3, D2Q9 with contacts and a periodic
  axis, D3Q19), FP32 storage within the FP32 bounds of the other parity
  tests, FP16 storage within its own.
* The rigidity table: a neutrally buoyant disk carried and turned by a
  channel flow (the set-up of the penalization-strength study) under the
  paper's stress penalty, the forcing added to it, and the forcing alone;
  the GPU reproduces the oracle's residuals, and the disk's velocity moves by
  under 1 % when the forcing is added to the stress penalty (the forcing
  adds no net momentum over a body whose nodes are centred on X_i).
"""
import numpy as np
import pytest

from gpu_common import banner
from measures import rigidity_residual
from oracle import oracle as O
from paper_2511_01629_amd import lbm
from paper_2511_01629_amd.workloads import place
from test_gpu_parity import _compare_run

pytestmark = pytest.mark.gpu


def _contacts(**kw):
    kinds = [("disk", 5.0, 5.0)] * 5 + [("ellipse", 6.0, 3.0)] * 3
    parts = place((64, 96), kinds, seed=7, rho_range=(1.2, 1.8), upper_axis=1, gap=0.3, margin=0.3)
    cfg = dict(lattice="D2Q9", n=(64, 96, 1), periodic=(0, 0, 0), tau=0.6, g=(0.0, -2e-4, 0.0), **kw)
    return cfg, parts


@pytest.mark.parametrize("beta,nopen,K", [(0.5, 0, 1), (1.0, 1, 1), (0.3, 0, 3), (0.8, 1, 3)])
def test_forcing_parity_2d(beta, nopen, K):
    banner(f"forcing parity 2d beta={beta} no_stress={nopen} K={K}")
    cfg, parts = _contacts(rigid_beta=beta, no_stress_penalty=nopen, K=K)
    _, _, rg, _ = _compare_run(cfg, parts, 150, xtol=1e-11, fused=False)
    assert np.abs(rg[:, :, 10:12]).max() > 0


def test_forcing_parity_periodic_ellipse():
    banner("forcing parity periodic")
    cfg = dict(lattice="D2Q9", n=(80, 60, 1), periodic=(1, 1, 0), tau=0.7, g=(0.0, -3e-4, 0.0), rigid_beta=0.6)
    parts = [dict(shape="ellipse", rho_s=1.5, a=7.0, b=3.5, x=(2.3, 30.2, 0.0), theta=0.7),
             dict(shape="disk", rho_s=1.3, a=6.0, x=(40.4, 1.7, 0.0))]
    _compare_run(cfg, parts, 120, fused=False)


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_forcing_parity_3d(storage):
    banner(f"forcing parity 3d {storage}")
    cfg = dict(lattice="D3Q19", n=(20, 15, 19), periodic=(0, 1, 0), tau=0.65, g=(0.0, 0.0, -5e-4), rigid_beta=0.7)
    parts = [dict(shape="sphere", rho_s=1.6, a=3.0, x=(7.0, 7.5, 9.0)),
             dict(shape="sphere", rho_s=1.3, a=3.5, x=(12.2, 8.0, 12.4))]
    if storage == "f64":
        _compare_run(cfg, parts, 40)
    else:
        _compare_run(cfg, parts, 40, storage="f32", tol=5e-6, xtol=1e-7)


@pytest.mark.parametrize("storage,utol,xtol", [("f32", 1e-4, 1e-6), ("f16", 1e-2, 1e-3)])
def test_forcing_reduced_storage(storage, utol, xtol):
    banner(f"forcing {storage}")
    cfg, parts = _contacts(rigid_beta=0.5)
    sim = lbm.Simulation(cfg, parts, storage=storage)
    ora = O.Oracle(cfg, parts)
    rg = sim.step_record(100)
    ro = ora.step(100, record=True)
    eX = np.abs(rg[:, :, 0:2] - ro[:, :, 0:2]).max()
    u_g, _, _ = sim.fields()
    u_o, _, _ = ora.fields()
    eu = np.abs(u_g - u_o).max() / np.abs(u_o).max()
    print(f"[measured] forcing {storage}: |X err| {eX:.2e} l.u., u err {eu:.2e} rel", flush=True)
    assert eX < xtol and eu < utol


CHANNEL = dict(lattice="D2Q9", n=(64, 48, 1), periodic=(1, 0, 0), tau=0.8, fluid_accel=(2e-6, 0.0, 0.0))
DISK = [dict(shape="disk", rho_s=1.0, a=8.0, x=(32.0, 16.5, 0.0))]
TABLE = [("stress penalty (the paper)", {}), ("stress + forcing 0.25", dict(rigid_beta=0.25)),
         ("stress + forcing 0.5", dict(rigid_beta=0.5)), ("stress + forcing 1", dict(rigid_beta=1.0)),
         ("neither", dict(no_stress_penalty=1)), ("forcing 0.5 alone", dict(no_stress_penalty=1, rigid_beta=0.5)),
         ("forcing 1 alone", dict(no_stress_penalty=1, rigid_beta=1.0))]


def test_forcing_rigidity_table():
    """Residual max |u - (U + omega x r)| over the disk after 3000 steps,
    relative to max |u|: of the velocity u of eq. (15a) with gravity alone
    (what the populations carry before the forcing, as lbm_get_fields reports
    it), and of the velocity that enters the collision,
    (1 - beta)(u - U - omega x r) in the same units."""
    banner("forcing rigidity table")
    rows = []
    for name, extra in TABLE:
        cfg = dict(CHANNEL, **extra)
        sim = lbm.Simulation(cfg, DISK, storage="f64")
        sim.step(3000)
        u, _, own = sim.fields()
        P = sim.particles()
        r, umax = rigidity_residual(u, own, P, cfg["periodic"])
        o = O.Oracle(cfg, DISK)
        o.step(3000)
        uo, _, owno = o.fields()
        ro, umaxo = rigidity_residual(uo, owno, o.particles(), cfg["periodic"])
        beta = extra.get("rigid_beta", 0.0)
        rows.append((name, r / umax, (1 - beta) * r / umax, P["U"][0][0], P["omega"][0][2]))
        print(f"[measured] {name:28s} residual of u {r / umax:.3e}  in the collision {(1 - beta) * r / umax:.3e}  "
              f"U {P['U'][0][0]:.6e}  omega {P['omega'][0][2]:.4e}", flush=True)
        assert abs(r - ro) <= 1e-9 * umaxo
    ref = rows[0]
    for name, _, coll, U, _ in rows[1:4]:  # the forcing added to the stress penalty
        assert abs(U / ref[3] - 1) < 0.01, name
    assert rows[1][2] < ref[2] and rows[2][2] < ref[2]  # beta 0.25, 0.5: closer to rigid where it counts
    assert rows[4][1] > 10 * ref[1]  # with neither, the disk is just fluid
