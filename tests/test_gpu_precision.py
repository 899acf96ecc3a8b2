"""Reduced-precision storage against the FP64 oracle.

FP32 storage (FP32 arithmetic), FP16 and BF16 storage of the populations
(FP32 arithmetic) with FP64 particle sums and Algorithm 1.  Populations are
stored as they are: in the velocity-based model the rest state has f^eq = 0
(eq. 13), so f itself is the deviation from rest.  The bounds are twice the
errors measured on MI355X (velocity max-norm relative to the largest
velocity; particle centre error in lattice units).
"""
import numpy as np
import pytest

from gpu_common import banner, pair
from paper_2511_01629_amd.workloads import place

pytestmark = pytest.mark.gpu

# storage: (u max-norm / max|u|, max |X - X_oracle| in l.u.), twice the
# values measured on MI355X: f32 3.5e-5 / 4.8e-5, f16 1.7e-3 / 3.9e-4,
# bf16 7.9e-2 / 2.1e-2.  FP32 is limited by FP32 arithmetic, not storage:
# rounding only the stored populations of the FP64 oracle to FP32 gives
# 1.1e-7 / 4.7e-9, while FP32 node arithmetic on the CPU gives 2.1e-5 / 2.2e-5.
BOUNDS = {"f32": (7e-5, 1e-4), "f16": (3.4e-3, 8e-4), "bf16": (0.16, 0.042)}


def _settling():
    cfg = dict(lattice="D2Q9", n=(120, 360, 1), periodic=(0, 0, 0), tau=0.6, g=(0.0, -1e-5, 0.0))
    parts = [dict(shape="disk", rho_s=1.5, a=12.0, x=(60.0, 300.0, 0.0))]
    return cfg, parts


@pytest.mark.parametrize("storage", ["f32", "f16", "bf16"])
def test_single_disk_settling_error(storage):
    """A disk of radius 12 settling in a closed 120x360 channel, 3000 steps."""
    banner(f"precision settling {storage}")
    cfg, parts = _settling()
    sim, ora = pair(cfg, parts, storage=storage)
    rg = sim.step_record(3000)
    ro = ora.step(3000, record=True)
    ug, _, _ = sim.fields()
    uo, _, _ = ora.fields()
    eu = float(np.abs(ug - uo).max() / np.abs(uo).max())
    ex = float(np.abs(rg[:, 0, 0:2] - ro[:, 0, 0:2]).max())
    eU = float(np.abs(rg[:, 0, 4:6] - ro[:, 0, 4:6]).max() / np.abs(ro[:, 0, 4:6]).max())
    print(f"[measured] storage={storage} u_rel={eu:.3e} X_abs={ex:.3e} U_rel={eU:.3e} "
          f"U_end={ro[-1, 0, 5]:.4e}", flush=True)
    bu, bx = BOUNDS[storage]
    assert eu < bu and ex < bx
