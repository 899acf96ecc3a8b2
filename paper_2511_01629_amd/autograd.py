"""torch.autograd wrapper of a differentiated run.

LbmTrajectory.apply(rho_s, tau, gmag, run) runs `run.steps` steps of the
penalized LBM on the GPU with checkpoints every `run.every` steps and returns
the final particle centres (n x 3, float64).  Its backward calls the library's
hand-written adjoint (lbm_backward), so gradients of any loss of the final
centres flow to the solid densities, tau and |g|.  Every step runs in the HIP
library; this module only marshals tensors.
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


class LbmTrajectory(torch.autograd.Function):
    @staticmethod
    def forward(ctx, rho_s, tau, gmag, run):
        rho = rho_s.detach().cpu().double().numpy()
        cfg = dict(run.cfg)
        cfg["tau"] = float(tau)
        g = np.asarray(cfg.get("g", (0.0, 0.0, 0.0)), dtype=np.float64)
        g0 = np.linalg.norm(g)
        if g0 == 0.0:
            raise ValueError("the gravity direction is taken from cfg['g'], which is zero")
        cfg["g"] = tuple(g / g0 * float(gmag))
        parts = [dict(p, rho_s=float(r)) for p, r in zip(run.particles, rho)]
        sim = lbm.Simulation(cfg, parts, storage=run.storage, device=run.device)
        sim.forward_checkpointed(run.steps, run.every)
        X = sim.particles()["X"]
        ctx.sim = sim
        run.last["sim"] = sim
        return torch.from_numpy(np.ascontiguousarray(X)).to(torch.float64)

    @staticmethod
    def backward(ctx, gX):
        g_rho, g_tau, g_g = ctx.sim.backward(gX.detach().cpu().double().numpy())
        return (torch.from_numpy(np.ascontiguousarray(g_rho)), torch.tensor(g_tau, dtype=torch.float64),
                torch.tensor(g_g, dtype=torch.float64), None)


def final_centres(rho_s, tau, gmag, run):
    """Differentiable final particle centres of `run` (see LbmTrajectory)."""
    return LbmTrajectory.apply(rho_s, tau, gmag, run)


def mean_height_loss(rho_s, tau, gmag, run, axis=1):
    """L = mean over particles of the final centre coordinate `axis`."""
    return final_centres(rho_s, tau, gmag, run)[:, axis].mean()
