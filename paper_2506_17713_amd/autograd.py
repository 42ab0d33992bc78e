"""torch.autograd bridge to the hand-written adjoint (lbm_grad).

    S = NonWettingSaturation.apply(wet, T, setup)

wet is the per-node wetting parameter (phi or drho, by the workload's mode)
as a float64 tensor shaped like the lattice, T the absolute EOS temperature
(0-d float64 tensor), and setup an AdjointSetup naming the workload, geometry,
initial density, horizon and checkpoint interval.  The forward pass runs the
solver on the GPU and the adjoint immediately (one reverse sweep gives the
gradient for every voxel and T at once); backward scales the stored gradient
by the incoming one.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import torch

from . import lbm


@dataclass
class AdjointSetup:
    workload: object            # inputs.Workload (one component, F32 or F64)
    solid: np.ndarray
    rho0: np.ndarray
    nsteps: int
    ckpt_every: int
    rho_mid: float
    delta: float
    device: str = "cuda"


class NonWettingSaturation(torch.autograd.Function):
    @staticmethod
    def forward(ctx, wet: torch.Tensor, T: torch.Tensor, setup: AdjointSetup):
        w = setup.workload
        Tv = float(T)
        w = w.with_(eos_T=(Tv, Tv))
        sol = lbm.Solver(w, setup.solid, setup.rho0, wet=wet.detach().cpu().double().numpy().reshape(1, -1),
                         device=setup.device)
        L, dwet, dT = sol.grad(setup.nsteps, setup.ckpt_every, "saturation", setup.rho_mid, setup.delta)
        sol.close()
        ctx.save_for_backward(dwet.reshape(wet.shape).to(wet.device, wet.dtype),
                              torch.tensor(dT, dtype=T.dtype, device=T.device))
        return torch.tensor(L, dtype=torch.float64, device=wet.device)

    @staticmethod
    def backward(ctx, gL):
        dwet, dT = ctx.saved_tensors
        return gL * dwet, gL.to(dT.device) * dT, None
