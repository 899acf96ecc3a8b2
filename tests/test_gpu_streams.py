"""Contexts on streams of the caller.

Two contexts, each on its own torch stream (default priority), stepped in
turn one step at a time, end bit-for-bit where the same runs end alone on
the current stream: nothing is shared between contexts, and every kernel
and copy of a context goes to its own stream.  The sums run in a fixed
order, so the results are reproducible to the bit.
"""
import numpy as np
import pytest

from gpu_common import banner
from paper_2511_01629_amd import lbm
from paper_2511_01629_amd.workloads import place, random_state

pytestmark = pytest.mark.gpu


def _cases():
    cfg_a = dict(lattice="D2Q9", n=(45, 37, 1), periodic=(1, 0, 0), tau=0.7, g=(0.0, -5e-4, 0.0))
    parts_a = [dict(shape="disk", rho_s=1.5, a=4.0, x=(10.2, 14.7, 0.0)),
               dict(shape="disk", rho_s=1.2, a=5.0, x=(19.0, 17.1, 0.0)),
               dict(shape="ellipse", rho_s=1.4, a=6.0, b=3.0, x=(36.5, 16.3, 0.0), theta=0.9)]
    cfg_b = dict(lattice="D3Q19", n=(20, 18, 26), periodic=(0, 1, 0), tau=0.8, g=(0.0, 0.0, -3e-4))
    parts_b = place((20, 18, 26), [("sphere", 3.5, 3.5)] * 3, seed=33, rho_range=(1.3, 1.7), upper_axis=2, gap=0.4,
                    margin=0.3)
    return (cfg_a, parts_a), (cfg_b, parts_b)


def _start(cfg, parts, storage, stream=None, seed=0):
    sim = lbm.Simulation(cfg, [], storage=storage, max_particles=len(parts), stream=stream)
    n = cfg["n"]
    Q = 9 if cfg["lattice"] == "D2Q9" else 19
    sim.set_populations(random_state((n[2], n[1], n[0]), Q, 1e-3, seed=seed))
    sim.set_particles(parts)
    return sim


def _state(sim):
    P = sim.particles()
    return sim.populations(), P["X"], P["U"], P["omega"]


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_contexts_on_own_streams(storage):
    banner(f"two contexts on own streams {storage}")
    import torch

    (cfg_a, parts_a), (cfg_b, parts_b) = _cases()
    steps = 40
    alone = []
    for k, (cfg, parts) in enumerate(((cfg_a, parts_a), (cfg_b, parts_b))):
        sim = _start(cfg, parts, storage, seed=k)
        sim.step(steps)
        alone.append(_state(sim))
        sim.close()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    a = _start(cfg_a, parts_a, storage, stream=s1, seed=0)
    b = _start(cfg_b, parts_b, storage, stream=s2, seed=1)
    for _ in range(steps):
        a.step(1)
        b.step(1)
    a.sync()
    b.sync()
    for sim, ref in ((a, alone[0]), (b, alone[1])):
        for got, want in zip(_state(sim), ref):
            assert np.array_equal(got, want)
    assert a.step_index == steps and b.step_index == steps
    a.close()
    b.close()
