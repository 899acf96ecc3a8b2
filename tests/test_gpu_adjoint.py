"""The hand-written adjoint against the oracle's complex-step derivative.

Both differentiate the step map with the indicator sequence frozen; the
complex-step oracle is exact to rounding, so in FP64 storage the adjoint
gradient must agree to near rounding.  Loss: a weighted sum of the final
centres (weights seeded), parameters: each rho_s, tau and |g|.
"""
import numpy as np
import pytest

from gpu_common import banner
from oracle import oracle as O
from paper_2511_01629_amd import lbm
from paper_2511_01629_amd.workloads import place

pytestmark = pytest.mark.gpu


def oracle_gradient(cfg, parts, steps, w):
    """Complex-step derivative of L = sum(w * X_final) for each parameter."""
    npart = len(parts)
    out = []
    for k in range(npart + 2):
        seed = dict(d_rho_s=[0.0] * npart, d_tau=0.0, d_gmag=0.0, h=1e-30)
        if k < npart:
            seed["d_rho_s"][k] = 1.0
        elif k == npart:
            seed["d_tau"] = 1.0
        else:
            seed["d_gmag"] = 1.0
        o = O.Oracle(cfg, parts, complex_step=seed)
        o.step(steps)
        Xi = o.particles(imag=True)["X"]
        out.append(float((w * Xi).sum() / seed["h"]))
    return np.array(out)


def gpu_gradient(cfg, parts, steps, every, w, storage="f64"):
    sim = lbm.Simulation(cfg, parts, storage=storage)
    sim.forward_checkpointed(steps, every)
    X_end = sim.particles()["X"].copy()
    f_end = sim.populations()
    g_rho, g_tau, g_g = sim.backward(w)
    # the final state is restored after the sweep
    assert np.array_equal(sim.populations(), f_end) and np.array_equal(sim.particles()["X"], X_end)
    again = sim.backward(w)
    assert np.array_equal(again[0], g_rho) and again[1] == g_tau and again[2] == g_g  # deterministic
    return np.concatenate([g_rho, [g_tau, g_g]])


def _check(ga, go, tol):
    scale = np.abs(go).max()
    err = np.abs(ga - go) / np.maximum(np.abs(go), 1e-3 * scale)
    print(f"[measured] max rel err {err.max():.3e}", flush=True)
    for a, o in zip(ga, go):
        print(f"   adjoint {a: .10e}  oracle {o: .10e}", flush=True)
    assert err.max() < tol, err


def test_adjoint_2d_contacts_f64():
    banner("adjoint 2d contacts f64")
    kinds = [("disk", 5.0, 5.0)] * 3 + [("ellipse", 6.0, 3.0)]
    parts = place((48, 64), kinds, seed=31, rho_range=(1.3, 1.8), upper_axis=1, gap=0.3, margin=0.3)
    cfg = dict(lattice="D2Q9", n=(48, 64, 1), periodic=(0, 0, 0), tau=0.65, g=(0.0, -3e-4, 0.0))
    w = np.random.default_rng(5).normal(size=(len(parts), 3))
    w[:, 2] = 0.0
    steps = 60
    go = oracle_gradient(cfg, parts, steps, w)
    ga = gpu_gradient(cfg, parts, steps, 16, w)
    _check(ga, go, 1e-8)


@pytest.mark.parametrize("every", [50, 7, 1])
def test_adjoint_2d_periodic_mean_height_f64(every):
    """The mean-height loss of the differentiated workload on a small box, x
    periodic; one segment, uneven segments, and every frame kept (every = 1)."""
    banner(f"adjoint 2d periodic f64 every={every}")
    parts = place((40, 72), [("disk", 6.0, 6.0)] * 3, seed=32, rho_range=(1.2, 1.6), upper_axis=1, gap=0.5,
                  margin=0.3)
    cfg = dict(lattice="D2Q9", n=(40, 72, 1), periodic=(1, 0, 0), tau=0.7, g=(0.0, -2e-4, 0.0))
    w = np.zeros((len(parts), 3))
    w[:, 1] = 1.0 / len(parts)
    go = oracle_gradient(cfg, parts, 50, w)
    ga = gpu_gradient(cfg, parts, 50, every, w)
    _check(ga, go, 1e-8)


def test_adjoint_3d_f64():
    banner("adjoint 3d f64")
    parts = place((20, 18, 26), [("sphere", 3.5, 3.5)] * 3, seed=33, rho_range=(1.3, 1.7), upper_axis=2, gap=0.4,
                  margin=0.3)
    cfg = dict(lattice="D3Q19", n=(20, 18, 26), periodic=(0, 1, 0), tau=0.7, g=(0.0, 0.0, -3e-4))
    w = np.random.default_rng(6).normal(size=(len(parts), 3))
    go = oracle_gradient(cfg, parts, 30, w)
    ga = gpu_gradient(cfg, parts, 30, 7, w)
    _check(ga, go, 1e-8)


def test_adjoint_2d_f32_storage():
    """FP32 storage and arithmetic (FP64 particle adjoint): the gradient of the
    same loss within the stated relative bound."""
    banner("adjoint 2d f32")
    parts = place((40, 72), [("disk", 6.0, 6.0)] * 3, seed=32, rho_range=(1.2, 1.6), upper_axis=1, gap=0.5,
                  margin=0.3)
    cfg = dict(lattice="D2Q9", n=(40, 72, 1), periodic=(1, 0, 0), tau=0.7, g=(0.0, -2e-4, 0.0))
    w = np.zeros((len(parts), 3))
    w[:, 1] = 1.0 / len(parts)
    go = oracle_gradient(cfg, parts, 50, w)
    ga = gpu_gradient(cfg, parts, 50, 10, w, storage="f32")
    _check(ga, go, 1e-3)


# 2-byte storage of the populations (FP32 arithmetic, FP64 particle adjoint):
# relative bounds on the gradient, about twice the errors measured on MI355X
TWO_BYTE_BOUNDS = {"f16": 1e-5, "bf16": 1e-4}  # measured 4.6e-6 and 4.8e-5


@pytest.mark.parametrize("storage", ["f16", "bf16"])
def test_adjoint_2d_two_byte_storage(storage):
    """The FP32-storage case in FP16 and BF16 storage: the gradient of the
    mean final height against the FP64 complex-step oracle, to the rounding
    of the stored populations."""
    banner(f"adjoint 2d {storage}")
    parts = place((40, 72), [("disk", 6.0, 6.0)] * 3, seed=32, rho_range=(1.2, 1.6), upper_axis=1, gap=0.5,
                  margin=0.3)
    cfg = dict(lattice="D2Q9", n=(40, 72, 1), periodic=(1, 0, 0), tau=0.7, g=(0.0, -2e-4, 0.0))
    w = np.zeros((len(parts), 3))
    w[:, 1] = 1.0 / len(parts)
    go = oracle_gradient(cfg, parts, 50, w)
    ga = gpu_gradient(cfg, parts, 50, 10, w, storage=storage)
    _check(ga, go, TWO_BYTE_BOUNDS[storage])


@pytest.mark.parametrize("every", [10, 1])
def test_adjoint_two_byte_odd_lattice(every):
    """FP16 storage on a lattice with Q N odd (45 x 37): Q N 2 bytes per
    population frame is not a multiple of 4, and the indicator frames that
    follow the population frames in the checkpoint buffers must still start
    on the 4-byte boundary the rasterisation's 32-bit compare-and-swap needs
    (frames are laid out on 256-byte strides).  Segments of 10 and every
    frame kept; the gradient against the complex-step oracle."""
    banner(f"adjoint 2d f16 odd lattice every={every}")
    parts = [dict(shape="disk", rho_s=1.5, a=4.0, x=(10.2, 14.7, 0.0)),
             dict(shape="disk", rho_s=1.2, a=5.0, x=(19.6, 17.1, 0.0)),
             dict(shape="disk", rho_s=1.4, a=4.5, x=(43.2, 6.3, 0.0))]
    cfg = dict(lattice="D2Q9", n=(45, 37, 1), periodic=(1, 0, 0), tau=0.7, g=(0.0, -5e-4, 0.0), eps_p=2.0,
               eps_w=1.0, delta=1.0)
    w = np.zeros((len(parts), 3))
    w[:, 1] = 1.0 / len(parts)
    go = oracle_gradient(cfg, parts, 40, w)
    ga = gpu_gradient(cfg, parts, 40, every, w, storage="f16")
    _check(ga, go, TWO_BYTE_BOUNDS["f16"])  # measured 3.1e-6


def test_adjoint_rejects_bad_use():
    banner("adjoint errors")
    parts = [dict(shape="disk", rho_s=1.5, a=5.0, x=(20.0, 30.0, 0.0))]
    cfg = dict(lattice="D2Q9", n=(40, 60, 1), tau=0.7, g=(0.0, -1e-4, 0.0))
    sim = lbm.Simulation(cfg, parts, storage="f32")
    with pytest.raises(lbm.LbmError) as e:
        sim.backward(np.zeros((1, 3)))
    assert e.value.code == lbm.LBM_ESTATE
    sim.step(1)
    with pytest.raises(lbm.LbmError) as e:
        sim.forward_checkpointed(5, 2)
    assert e.value.code == lbm.LBM_ESTATE
    sim2 = lbm.Simulation(dict(cfg, K=2), parts, storage="f32")
    with pytest.raises(lbm.LbmError) as e:
        sim2.forward_checkpointed(5, 2)
    assert e.value.code == lbm.LBM_EINVAL


def test_autograd_wrapper_matches_oracle():
    """torch.autograd over the checkpointed run: loss.backward() gives the
    complex-step oracle gradient of the mean final height."""
    banner("autograd wrapper")
    import torch

    from paper_2511_01629_amd.autograd import Run, mean_height_loss

    parts = place((40, 72), [("disk", 6.0, 6.0)] * 3, seed=32, rho_range=(1.2, 1.6), upper_axis=1, gap=0.5,
                  margin=0.3)
    cfg = dict(lattice="D2Q9", n=(40, 72, 1), periodic=(1, 0, 0), tau=0.7, g=(0.0, -2e-4, 0.0))
    run = Run(cfg=cfg, particles=parts, steps=50, every=8, storage="f64")
    rho = torch.tensor([p["rho_s"] for p in parts], dtype=torch.float64, requires_grad=True)
    tau = torch.tensor(0.7, dtype=torch.float64, requires_grad=True)
    gmag = torch.tensor(2e-4, dtype=torch.float64, requires_grad=True)
    loss = mean_height_loss(rho, tau, gmag, run)
    loss.backward()
    w = np.zeros((3, 3))
    w[:, 1] = 1.0 / 3
    go = oracle_gradient(cfg, parts, 50, w)
    ga = np.concatenate([rho.grad.numpy(), [tau.grad.item(), gmag.grad.item()]])
    _check(ga, go, 1e-8)
    o = O.Oracle(cfg, parts)
    o.step(50)
    assert abs(loss.item() - o.particles()["X"][:, 1].mean()) < 1e-10


def test_autograd_devices_and_plain_numbers():
    """rho_s on the GPU, tau a plain number, |g| a float32 CPU tensor: the
    centres come back on the GPU, each gradient on its input's device and
    dtype (none for the plain number), equal to the complex-step oracle."""
    banner("autograd devices")
    import torch

    from paper_2511_01629_amd.autograd import Run, mean_height_loss

    parts = place((40, 72), [("disk", 6.0, 6.0)] * 3, seed=32, rho_range=(1.2, 1.6), upper_axis=1, gap=0.5,
                  margin=0.3)
    gmag = torch.tensor(2e-4, dtype=torch.float32, requires_grad=True)
    cfg = dict(lattice="D2Q9", n=(40, 72, 1), periodic=(1, 0, 0), tau=0.7, g=(0.0, -gmag.item(), 0.0))
    run = Run(cfg=cfg, particles=parts, steps=50, every=8, storage="f64")
    rho = torch.tensor([p["rho_s"] for p in parts], dtype=torch.float64, device="cuda", requires_grad=True)
    loss = mean_height_loss(rho, 0.7, gmag, run)
    assert loss.device.type == "cuda"
    loss.backward()
    assert rho.grad.device.type == "cuda" and rho.grad.dtype == torch.float64
    assert gmag.grad.device.type == "cpu" and gmag.grad.dtype == torch.float32
    w = np.zeros((3, 3))
    w[:, 1] = 1.0 / 3
    go = oracle_gradient(cfg, parts, 50, w)
    _check(rho.grad.cpu().numpy(), go[:3], 1e-8)
    assert abs(gmag.grad.item() / go[4] - 1) < 1e-6


def test_adjoint_many_bodies_f64():
    """70 bodies: the particle adjoints run one workgroup per particle."""
    banner("adjoint many bodies f64")
    parts = place((96, 128), [("disk", 3.0, 3.0)] * 70, seed=33, rho_range=(1.3, 1.8), upper_axis=1, gap=0.3,
                  margin=0.3)
    cfg = dict(lattice="D2Q9", n=(96, 128, 1), periodic=(0, 0, 0), tau=0.65, g=(0.0, -3e-4, 0.0))
    w = np.random.default_rng(6).normal(size=(len(parts), 3))
    w[:, 2] = 0.0
    steps = 30
    go = oracle_gradient(cfg, parts, steps, w)
    ga = gpu_gradient(cfg, parts, steps, 10, w)
    _check(ga, go, 1e-8)


@pytest.mark.parametrize("every", [1, 8])
def test_adjoint_in_caller_memory(every):
    """lbm_forward_checkpointed_ws / lbm_backward_ws with every buffer in torch
    tensors (sized by lbm_grad_workspace_size) give the library-allocated
    run's gradients bit for bit; a workspace one byte short is rejected with
    ENOMEM, one off a 256-byte boundary with EINVAL."""
    banner(f"adjoint in caller memory every={every}")
    kinds = [("disk", 5.0, 5.0)] * 4 + [("ellipse", 6.0, 3.0)] * 2
    parts = place((64, 96), kinds, seed=7, rho_range=(1.2, 1.8), upper_axis=1, gap=0.3, margin=0.3)
    cfg = dict(lattice="D2Q9", n=(64, 96, 1), periodic=(0, 0, 0), tau=0.6, g=(0.0, -2e-4, 0.0))
    w = np.random.default_rng(3).normal(size=(len(parts), 3))
    out = []
    for torch_memory in (False, True):
        sim = lbm.Simulation(cfg, parts, storage="f32")
        sim.forward_checkpointed(40, every, torch_memory=torch_memory)
        out.append(sim.backward(w))
        if torch_memory:
            fb, bb = sim.grad_workspace_size(40, every)
            assert sim._fwd_ws.numel() == fb and bb > 0
    (r0, t0, g0), (r1, t1, g1) = out
    assert np.array_equal(r0, r1) and t0 == t1 and g0 == g1
    import ctypes as C

    import torch

    sim = lbm.Simulation(cfg, parts, storage="f32")
    fb, bb = sim.grad_workspace_size(40, every)
    small = torch.empty(fb - 1, dtype=torch.uint8, device="cuda")
    rc = sim.lib.lbm_forward_checkpointed_ws(sim.ctx, 40, every, C.c_void_p(small.data_ptr()), fb - 1)
    assert rc == lbm.LBM_ENOMEM
    # a workspace that does not start on a 256-byte boundary is rejected on
    # the host, before anything is carved from it
    big = torch.empty(fb + 512, dtype=torch.uint8, device="cuda")
    rc = sim.lib.lbm_forward_checkpointed_ws(sim.ctx, 40, every, C.c_void_p(big.data_ptr() + 2), fb)
    assert rc == lbm.LBM_EINVAL
    seed = np.ascontiguousarray(w, dtype=np.float64)
    rc = sim.lib.lbm_backward_ws(sim.ctx, seed.ctypes.data_as(C.POINTER(C.c_double)), None, None, None,
                                 C.c_void_p(big.data_ptr() + 2), fb)
    assert rc == lbm.LBM_EINVAL
