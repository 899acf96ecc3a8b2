"""torch.autograd wrapper of a differentiated run.

LbmTrajectory.apply(rho_s, tau, gmag, run[, X0]) runs `run.steps` steps of
the penalized LBM on the GPU with checkpoints every `run.every` steps and
returns the final particle centres (n x 3, float64, on the device of rho_s).
Its backward calls the library's hand-written adjoint (lbm_backward, and
lbm_grad_positions for X0), so gradients of any loss of the final centres
flow to the solid densities, tau, |g| and, if given, the initial centres X0
(n x 3; with the fractional indicator the gradient of the loss itself, with
the binary one the frozen-indicator derivative), each on its input's device
and dtype (a plain number for tau or |g| gets no gradient).  Every step runs in the HIP
library; this module only marshals tensors.

A Run keeps one library context: its first forward creates it and saves, on
the device, the state right after the particles were set; every forward
loads that state back and sets the parameters (lbm_set_params, which also
measures U^0 again with them), so no context is rebuilt per forward; the
checkpoints and the backward's scratch are torch tensors (torch's allocator
owns every buffer of the differentiated run).  The
checkpoints belong to the context, so a Run holds one differentiated run at
a time: backward through an earlier forward of the same Run raises.
"""
from dataclasses import dataclass, field

import numpy as np
import torch

from . import lbm


@dataclass
class Run:
    cfg: dict
    particles: list
    steps: int
    every: int = 100
    storage: str = "f32"
    device: int = 0
    last: dict = field(default_factory=dict)
    sim: object = field(default=None, repr=False)   # the library context
    start: object = field(default=None, repr=False)  # its state right after set_particles (device bytes)
    generation: int = 0                               # forwards run so far


def _context(run):
    if run.sim is None:
        run.sim = lbm.Simulation(run.cfg, run.particles, storage=run.storage, device=run.device)
        run.start = run.sim.save_state(on_device=True)
    return run.sim


def _number(x):
    return float(x.detach()) if torch.is_tensor(x) else float(x)


class LbmTrajectory(torch.autograd.Function):
    @staticmethod
    def forward(ctx, rho_s, tau, gmag, run, X0=None):
        rho = rho_s.detach().cpu().double().numpy()
        g = np.asarray(run.cfg.get("g", (0.0, 0.0, 0.0)), dtype=np.float64)
        g0 = np.linalg.norm(g)
        if g0 == 0.0:
            raise ValueError("the gravity direction is taken from cfg['g'], which is zero")
        sim = _context(run)
        sim.load_state(run.start)
        if X0 is not None:  # the run starts from these centres instead of run.particles' ones
            x0 = X0.detach().cpu().double().numpy().reshape(len(run.particles), 3)
            sim.set_particles([dict(p, x=tuple(float(v) for v in x0[i])) for i, p in enumerate(run.particles)])
        sim.set_params(rho_s=rho, tau=_number(tau), g=g / g0 * _number(gmag))
        sim.forward_checkpointed(run.steps, run.every, torch_memory=True)
        X = sim.particles()["X"]
        run.generation += 1
        ctx.sim = sim
        ctx.run = run
        ctx.generation = run.generation
        # each gradient goes back on its input's device and dtype (inputs may
        # be CUDA tensors or plain numbers)
        ctx.like = [(t.device, t.dtype) if torch.is_tensor(t) else None for t in (rho_s, tau, gmag, X0)]
        run.last["sim"] = sim
        out = torch.from_numpy(np.ascontiguousarray(X)).to(torch.float64)
        return out.to(rho_s.device) if torch.is_tensor(rho_s) else out

    @staticmethod
    def backward(ctx, gX):
        if ctx.generation != ctx.run.generation:
            raise RuntimeError("a later forward of the same Run replaced this run's checkpoints")
        g_rho, g_tau, g_g = ctx.sim.backward(gX.detach().cpu().double().numpy())
        g_X0 = ctx.sim.grad_positions() if ctx.like[3] is not None and ctx.needs_input_grad[4] else None
        out = []
        for k, g in zip((0, 1, 2, 4), (np.ascontiguousarray(g_rho), g_tau, g_g, g_X0)):
            like = ctx.like[min(k, 3)]
            if not ctx.needs_input_grad[k] or like is None:
                out.append(None)
            else:
                out.append(torch.as_tensor(g, dtype=torch.float64).to(device=like[0], dtype=like[1]))
        return out[0], out[1], out[2], None, out[3]


def final_centres(rho_s, tau, gmag, run, X0=None):
    """Differentiable final particle centres of `run` (see LbmTrajectory)."""
    return LbmTrajectory.apply(rho_s, tau, gmag, run, X0)


def mean_height_loss(rho_s, tau, gmag, run, axis=1, X0=None):
    """L = mean over particles of the final centre coordinate `axis`."""
    return final_centres(rho_s, tau, gmag, run, X0)[:, axis].mean()
