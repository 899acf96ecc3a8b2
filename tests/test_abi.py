"""The C-ABI library loads and exports every symbol include/lbm.h declares,
and rejects invalid configurations on the host (no compute call, no GPU)."""
import ctypes as C
import os
import re

import pytest

from paper_2511_01629_amd import lbm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "lbm.h")).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char \*)\s*(lbm_\w+)\s*\(", txt, re.M)))


def test_header_declares_the_binding_exports():
    assert _declared() == sorted(lbm.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = lbm.load()
    for name in _declared():
        assert hasattr(lib, name), name


def _base():
    return dict(lattice="D2Q9", n=(64, 32, 1), periodic=(1, 0, 0), tau=0.8, storage="f32")


@pytest.mark.parametrize("bad", [
    dict(tau=0.5), dict(tau=0.3), dict(alpha=2.0), dict(n=(0, 32, 1)), dict(lattice="D3Q19", n=(8, 8, -1)),
    dict(K=0), dict(eps_p=0.0), dict(delta=-1.0), dict(n=(40000, 40000, 1)),
])
def test_invalid_configs_rejected_on_host(bad):
    lib = lbm.load()
    cfg = dict(_base(), **bad)
    c = lbm.make_config(cfg, max_particles=4)
    size = C.c_size_t()
    assert lib.lbm_workspace_size(C.byref(c), C.byref(size)) == lbm.LBM_EINVAL
    ctx = C.c_void_p()
    assert lib.lbm_create(C.byref(c), C.byref(ctx)) == lbm.LBM_EINVAL
    assert not ctx.value


@pytest.mark.parametrize("lattice,n,ok", [
    ("D2Q9", (16384, 16384, 1), True),    # Q N = 2.42e9: 64-bit population offsets
    ("D3Q19", (512, 512, 512), True),     # Q N = 2.55e9
    ("D3Q19", (1024, 1024, 682), True),   # d N = 2.1457e9, just below 2^31
    ("D3Q19", (1024, 1024, 683), False),  # d N = 2.1489e9: 32-bit node offsets no longer hold
    ("D2Q9", (32768, 32768, 1), False),   # d N = 2^31
])
def test_lattice_size_limit_is_on_node_offsets(lattice, n, ok):
    """Population offsets q N + node switch to 64 bits when Q N >= 2^31; node
    offsets (and the d N solid-velocity field) stay 32-bit, so d N < 2^31 is
    the limit, checked on the host before any device work."""
    lib = lbm.load()
    c = lbm.make_config(dict(lattice=lattice, n=n, periodic=(1, 0, 0), tau=0.8, storage="f16"), max_particles=4)
    size = C.c_size_t()
    rc = lib.lbm_workspace_size(C.byref(c), C.byref(size))
    if ok:
        Q = 9 if lattice == "D2Q9" else 19
        assert rc == 0 and size.value >= 2 * Q * n[0] * n[1] * n[2] * 2
    else:
        assert rc == lbm.LBM_EINVAL


def _walls(axis, lo, hi):
    w = [[(0.0, 0.0, 0.0), (0.0, 0.0, 0.0)] for _ in range(3)]
    w[axis] = [lo, hi]
    return w


@pytest.mark.parametrize("bad", [
    dict(wall_velocity=_walls(1, (0.0, 0.01, 0.0), (0.0, 0.0, 0.0))),                     # normal motion
    dict(periodic=(0, 1, 0), wall_velocity=_walls(0, (0.0, 0.01, 0.0), (0.0, 0.0, 0.0))),  # x walls
    dict(periodic=(1, 1, 0), wall_velocity=_walls(1, (0.01, 0.0, 0.0), (0.0, 0.0, 0.0))),  # periodic axis
    dict(periodic=(0, 0, 0), wall_velocity=_walls(1, (0.01, 0.0, 0.0), (0.0, 0.0, 0.0))),  # x walls fixed
    dict(wall_velocity=_walls(1, (float("nan"), 0.0, 0.0), (0.0, 0.0, 0.0))),
])
def test_moving_walls_rejected_on_host(bad):
    """Moving walls: one axis (y, or z in 3D), tangential, every other axis
    periodic; anything else is EINVAL before any device work."""
    lib = lbm.load()
    c = lbm.make_config(dict(_base(), **bad), max_particles=4)
    size = C.c_size_t()
    assert lib.lbm_workspace_size(C.byref(c), C.byref(size)) == lbm.LBM_EINVAL
    good = lbm.make_config(dict(_base(), wall_velocity=_walls(1, (-0.01, 0.0, 0.0), (0.01, 0.0, 0.0))))
    assert lib.lbm_workspace_size(C.byref(good), C.byref(size)) == 0


def test_invalid_storage_and_particle_cap():
    lib = lbm.load()
    c = lbm.make_config(_base(), max_particles=70000)
    ctx = C.c_void_p()
    assert lib.lbm_create(C.byref(c), C.byref(ctx)) == lbm.LBM_EINVAL
    c = lbm.make_config(_base(), max_particles=1)
    c.storage = 7
    assert lib.lbm_create(C.byref(c), C.byref(ctx)) == lbm.LBM_EINVAL


def test_workspace_size_scales_with_storage():
    lib = lbm.load()
    sizes = {}
    for s in ("f64", "f32", "f16"):
        c = lbm.make_config(_base(), storage=s, max_particles=8)
        size = C.c_size_t()
        assert lib.lbm_workspace_size(C.byref(c), C.byref(size)) == 0
        sizes[s] = size.value
    N = 64 * 32
    # two population buffers of Q*N elements differ by the element size
    assert sizes["f64"] - sizes["f32"] >= 2 * 9 * N * 4 - 4096
    assert sizes["f32"] - sizes["f16"] >= 2 * 9 * N * 2 - 4096


def test_null_arguments():
    lib = lbm.load()
    assert lib.lbm_create(None, None) == lbm.LBM_EINVAL
    assert lib.lbm_destroy(None) == lbm.LBM_EINVAL
    assert lib.lbm_step(None, 1) == lbm.LBM_EINVAL
    # every call taking a context rejects NULL before any device work
    size = C.c_size_t()
    step = C.c_int64()
    for rc in (lib.lbm_workspace_size(None, C.byref(size)), lib.lbm_set_particles(None, None, 0),
               lib.lbm_step_record(None, 0, None), lib.lbm_sync(None), lib.lbm_get_fields(None, None, None, None),
               lib.lbm_get_populations(None, None), lib.lbm_set_populations(None, None),
               lib.lbm_get_particles(None, None, 0), lib.lbm_forward_checkpointed(None, 1, 1),
               lib.lbm_backward(None, None, None, None, None), lib.lbm_profile(None, 1),
               lib.lbm_profile_read(None, None, None, 0), lib.lbm_get_step(None, C.byref(step)),
               lib.lbm_get_fields_device(None, None, None, None), lib.lbm_set_params(None, None, 0.0, None),
               lib.lbm_state_size(None, C.byref(size)), lib.lbm_save_state(None, None),
               lib.lbm_load_state(None, None), lib.lbm_step_slabs(None, 1, 2),
               lib.lbm_grad_workspace_size(None, 1, 1, None, None), lib.lbm_forward_checkpointed_ws(None, 1, 1, None, 0),
               lib.lbm_backward_ws(None, None, None, None, None, None, 0), lib.lbm_grad_positions(None, None)):
        assert rc == lbm.LBM_EINVAL
    assert lib.lbm_workspace_size(C.byref(lbm.make_config(_base())), None) == lbm.LBM_EINVAL
    # lbm_copy: NULL with bytes > 0, misaligned pointers, sizes that are not whole 16-byte words
    assert lib.lbm_copy(None, None, 16, None) == lbm.LBM_EINVAL
    assert lib.lbm_copy(C.c_void_p(0x1008), C.c_void_p(0x2000), 16, None) == lbm.LBM_EINVAL
    assert lib.lbm_copy(C.c_void_p(0x1000), C.c_void_p(0x2000), 24, None) == lbm.LBM_EINVAL
    assert lib.lbm_copy(None, None, 0, None) == lbm.LBM_OK
    # lbm_copy_arrays: the same, and an array count outside 1..32
    assert lib.lbm_copy_arrays(None, None, 9, 16, None) == lbm.LBM_EINVAL
    assert lib.lbm_copy_arrays(C.c_void_p(0x1000), C.c_void_p(0x2004), 9, 16, None) == lbm.LBM_EINVAL
    assert lib.lbm_copy_arrays(C.c_void_p(0x1000), C.c_void_p(0x2000), 9, 40, None) == lbm.LBM_EINVAL
    assert lib.lbm_copy_arrays(C.c_void_p(0x1000), C.c_void_p(0x2000), 0, 16, None) == lbm.LBM_EINVAL
    assert lib.lbm_copy_arrays(C.c_void_p(0x1000), C.c_void_p(0x2000), 33, 16, None) == lbm.LBM_EINVAL
    assert lib.lbm_copy_arrays(None, None, 9, 0, None) == lbm.LBM_OK
    # a rejected configuration leaves its reason for lbm_last_error(NULL)
    bad = lbm.make_config(_base(), storage="f32", max_particles=8)
    bad.tau = 0.4
    out = C.c_void_p()
    assert lib.lbm_create(C.byref(bad), C.byref(out)) == lbm.LBM_EINVAL and not out.value
    assert b"tau" in lib.lbm_last_error(None)
