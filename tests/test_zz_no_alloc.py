"""lbm_step_record_noalloc (the variant of lbm_step_record that allocates
nothing: its per-step records go through the library's static device array)
against lbm_step_record, through the C ABI: two calls in a row on the same
contexts, the second with fewer steps, and then a third on a context with
fewer particles; the records and the final state agree bit for bit (both run
the same kernels in the same order)."""
import numpy as np
import pytest

from gpu_common import banner
from paper_2511_01629_amd import lbm
from paper_2511_01629_amd.workloads import place

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_noalloc_record_matches_record(storage):
    banner(f"no-allocation record {storage}")
    kinds = [("disk", 5.0, 5.0)] * 5 + [("ellipse", 6.0, 3.0)] * 3
    parts = place((64, 96), kinds, seed=7, rho_range=(1.2, 1.8), upper_axis=1, gap=0.3, margin=0.3)
    cfg = dict(lattice="D2Q9", n=(64, 96, 1), periodic=(0, 0, 0), tau=0.6, g=(0.0, -2e-4, 0.0))
    a = lbm.Simulation(cfg, parts, storage=storage)
    b = lbm.Simulation(cfg, parts, storage=storage)
    contact = 0.0
    for n in (120, 35):  # the second call is smaller: stale records of the first must not leak
        ra = a.step_record(n)
        rb = b.step_record_noalloc(n)
        assert ra.shape == rb.shape == (n, len(parts), 14)
        assert np.array_equal(ra, rb)
        contact = max(contact, np.abs(ra[:, :, 10:12]).max())
    assert contact > 0  # the collision forces acted (bodies start inside the collision range)
    assert np.array_equal(a.populations(), b.populations())
    # fewer particles on another context of the same GPU: its own records only
    c = lbm.Simulation(cfg, parts[:3], storage=storage)
    d = lbm.Simulation(cfg, parts[:3], storage=storage)
    assert np.array_equal(c.step_record(10), d.step_record_noalloc(10))
    # beyond the static array: rejected before any step
    lim = (1 << 20) // (len(parts) * 20)
    with pytest.raises(lbm.LbmError) as e:
        b.step_record_noalloc(lim + 1)
    assert e.value.code == lbm.LBM_EINVAL
    assert b.step_index == 155
