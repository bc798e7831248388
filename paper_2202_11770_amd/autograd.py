"""torch.autograd wrapper of the hand-written adjoint (hlb_adjoint_run).

``WssObjective.apply(A, phi, sim, n, obj_t0, obj_t1, n_snap)`` runs ``n``
steps of the update from the simulation's current state and returns
J = sum over t in (obj_t0, obj_t1] of the summed wall shear stress, as a
0-d FP64 tensor.  Its gradients with respect to

  * ``A``   [n_velocity_iolets, n]: the amplitude each velocity iolet uses in
            each of the n updates, and
  * ``phi`` [n_sites]: the per-site wall porosity (caller order),

come from the GPU adjoint sweep with binomial checkpointing (``n_snap``
device snapshots).  The adjoint runs in the forward call -- one forward and
one reverse sweep, however many outputs the graph differentiates -- and
``backward`` only scales the stored gradients.  torch is used for the
tensors; every step of the computation runs in libhlb.so.

``fourier_inlet(theta, n, period, base)`` builds A(s) = base + sum_k
a_k cos(2 pi k s / period) + b_k sin(2 pi k s / period) from theta = (a, b)
in torch, so gradients reach the Fourier coefficients through autograd.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import hlb


def fourier_inlet(theta: torch.Tensor, n: int, period: float, base: float = 0.01) -> torch.Tensor:
    m = theta.shape[0] // 2
    s = torch.arange(n, dtype=theta.dtype, device=theta.device)
    k = torch.arange(1, m + 1, dtype=theta.dtype, device=theta.device)
    ang = 2.0 * math.pi * s[:, None] * k[None, :] / period
    return base + torch.cos(ang) @ theta[:m] + torch.sin(ang) @ theta[m:]


class WssObjective(torch.autograd.Function):
    @staticmethod
    def forward(ctx, A, phi, sim, n: int, obj_t0: int, obj_t1: int, n_snap: int):
        info = hlb.hlb_info(sim.ctx)
        t0 = hlb.hlb_time(sim.ctx)
        vel = [k for k in range(info["n_iolets"]) if sim.iolet_kinds[k] == 0]
        A_h = A.detach().to("cpu", torch.float64).numpy().reshape(len(vel), n)
        for row, k in enumerate(vel):
            # the update t0+s -> t0+s+1 reads table[(t0 + s) mod n]
            hlb.hlb_set_iolet_table(sim.ctx, k, np.roll(A_h[row], t0 % n))
        hlb.hlb_set_porosity(sim.ctx, phi.detach().to("cpu", torch.float64).numpy())
        J, dA, dphi, fw = hlb.hlb_adjoint_run(sim.ctx, n, obj_t0, obj_t1, n_snap)
        ctx.save_for_backward(torch.from_numpy(dA[vel]).to(A.device, A.dtype).reshape(A.shape),
                              torch.from_numpy(dphi).to(phi.device, phi.dtype))
        ctx.forward_steps = fw
        return torch.tensor(J, dtype=torch.float64, device=A.device)

    @staticmethod
    def backward(ctx, gJ):
        dA, dphi = ctx.saved_tensors
        return gJ * dA, gJ * dphi, None, None, None, None, None
