"""The seeded synthetic workloads (inputs only): every configuration is
accepted by the library's host checks, and the bodies of each placement
respect its stated recipe -- inside the box with the wall margin, centres in
the upper half along gravity, bounding circles or spheres at least the gap
apart, densities in the stated range -- and the same seed gives the same
placement."""
import ctypes as C

import numpy as np
import pytest

from paper_2511_01629_amd import lbm
from paper_2511_01629_amd.workloads import NAMES, workload


@pytest.mark.parametrize("name", NAMES)
def test_workload_accepted_and_placed_by_its_recipe(name):
    cfg, parts, steps, info = workload(name)
    assert steps > 0 and info["desc"]
    lib = lbm.load()
    c = lbm.make_config(cfg, max_particles=max(len(parts), 1))
    size = C.c_size_t()
    assert lib.lbm_workspace_size(C.byref(c), C.byref(size)) == 0
    d = 2 if cfg["lattice"] == "D2Q9" else 3
    n = np.array(cfg["n"][:d], dtype=float)
    X = np.array([p["x"][:d] for p in parts]).reshape(len(parts), d)
    R = np.array([p["a"] for p in parts])
    for k in range(d):
        if not cfg["periodic"][k]:
            assert np.all(X[:, k] - R >= -0.5) and np.all(X[:, k] + R <= n[k] - 0.5)
    if len(parts) > 1:
        gaps = np.linalg.norm(X[:, None, :] - X[None, :, :], axis=-1) - (R[:, None] + R[None, :])
        np.fill_diagonal(gaps, np.inf)
        assert gaps.min() >= 2.0 - 1e-12
    g = np.array(cfg["g"][:d])
    if len(parts) > 1 and np.any(g != 0):
        ax = int(np.argmax(np.abs(g)))
        assert np.all(X[:, ax] >= 0.5 * n[ax] - 1e-9)
    X2 = np.array([p["x"][:d] for p in workload(name)[1]]).reshape(len(parts), d)
    assert np.array_equal(X, X2)


def test_sphere_boxes_share_fluid_and_spheres():
    """The reduced 3D box keeps the full-size sphere workload's fluid, gravity,
    radius and density range; only the box and the sphere count change."""
    big, pb, sb, _ = workload("spheres_256x256x512")
    small, ps, ss, _ = workload("spheres_64x64x128")
    for k in ("lattice", "tau", "g", "periodic", "K", "eps_p", "eps_w", "delta"):
        assert big[k] == small[k], k
    assert sb == ss == 5000
    assert {p["a"] for p in pb} == {p["a"] for p in ps} == {8.0}
    rho = [p["rho_s"] for p in pb + ps]
    assert min(rho) >= 1.2 and max(rho) <= 1.8
