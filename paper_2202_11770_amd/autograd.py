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
tensors and the stream; every step of the computation runs in libhlb.so, and
the parameters, the objective and the gradients never leave the GPU.

``IoletFluxObjective`` does the same for the weighted net outflow through
the iolets, with gradients also for the per-step ghost densities of the
pressure iolets.  Windkessel outlets set on the simulation
(hlb_set_windkessel) stay on, and the adjoint runs through their model,
as long as no ghost-density table is passed (R None): a table passed for a
pressure iolet replaces its model.

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


def _adjoint(sim, A, R, phi, n: int, obj_t0: int, obj_t1: int, n_snap: int, kind: int, weights):
    """Set the per-step tables (velocity rows from A, pressure rows from R if
    given) and the porosity from the device tensors, run the adjoint sweep
    with device outputs; returns J and the gradients of A, R (or None) and
    phi as device tensors like the inputs, and the forward steps taken.

    The library's work is put on torch's current stream of the current
    device; the setters read the parameters there (inputs on the host are
    copied there first) and the outputs are written there; gradients are
    returned on the inputs' devices, so GPU inputs never leave the GPU.  The
    simulation keeps the tables and the porosity set here (its state and
    time are left as they were)."""
    info = hlb.hlb_info(sim.ctx)
    t0 = hlb.hlb_time(sim.ctx)
    dev = torch.device("cuda", torch.cuda.current_device())  # the library's device
    hlb.hlb_set_stream(sim.ctx, torch.cuda.current_stream(dev).cuda_stream)
    vel = [k for k in range(info["n_iolets"]) if sim.iolet_kinds[k] == hlb.HLB_IOLET_VELOCITY]
    pres = [k for k in range(info["n_iolets"]) if sim.iolet_kinds[k] == hlb.HLB_IOLET_PRESSURE]
    for rows, T in ((vel, A), (pres, R)):
        if T is None:
            continue
        Td = T.detach().to(dev, torch.float64).reshape(len(rows), n)
        for r, k in enumerate(rows):
            # the update t0+s -> t0+s+1 reads table[(t0 + s) mod n]
            hlb.hlb_set_iolet_table_device(sim.ctx, k, torch.roll(Td[r], t0 % n).contiguous())
    hlb.hlb_set_porosity_device(sim.ctx, phi.detach().to(dev, torch.float64).contiguous())
    hlb.hlb_set_objective(sim.ctx, kind, weights)
    nio = info["n_iolets"]
    J = torch.zeros(1, dtype=torch.float64, device=dev)
    d_tab = torch.zeros(nio, n, dtype=torch.float64, device=dev)
    dphi = torch.zeros(info["n_sites"], dtype=torch.float64, device=dev)
    try:
        fw = hlb.hlb_adjoint_run_device(sim.ctx, n, obj_t0, obj_t1, n_snap, J, d_tab if nio else None, dphi)
    finally:
        hlb.hlb_set_objective(sim.ctx, hlb.HLB_OBJ_WSS)
    # gradients on the inputs' devices (no copy when they live on the GPU)
    dA = d_tab[vel].to(A.device, A.dtype).reshape(A.shape)
    dR = None if R is None else d_tab[pres].to(R.device, R.dtype).reshape(R.shape)
    return J[0].to(A.device), dA, dR, dphi.to(phi.device, phi.dtype), fw


class WssObjective(torch.autograd.Function):
    @staticmethod
    def forward(ctx, A, phi, sim, n: int, obj_t0: int, obj_t1: int, n_snap: int):
        J, dA, _, dphi, fw = _adjoint(sim, A, None, phi, n, obj_t0, obj_t1, n_snap, hlb.HLB_OBJ_WSS, None)
        ctx.save_for_backward(dA, dphi)
        ctx.forward_steps = fw
        return J.clone()

    @staticmethod
    def backward(ctx, gJ):
        dA, dphi = ctx.saved_tensors
        return gJ * dA, gJ * dphi, None, None, None, None, None


class IoletFluxObjective(torch.autograd.Function):
    """``IoletFluxObjective.apply(A, R, phi, sim, n, obj_t0, obj_t1, n_snap,
    weights)``: J = sum over t in (obj_t0, obj_t1] of sum_k weights[k] Q_k(t),
    Q_k(t) the net outflow through iolet k during the update t-1 -> t
    (hlb_set_objective).  Gradients with respect to A [n_velocity_iolets, n]
    (per-step amplitudes), R [n_pressure_iolets, n] (per-step ghost
    densities) and phi [n_sites] (porosity)."""

    @staticmethod
    def forward(ctx, A, R, phi, sim, n: int, obj_t0: int, obj_t1: int, n_snap: int, weights):
        J, dA, dR, dphi, fw = _adjoint(sim, A, R, phi, n, obj_t0, obj_t1, n_snap, hlb.HLB_OBJ_IOLET_FLUX,
                                       np.asarray(weights, dtype=np.float64))
        ctx.save_for_backward(dA, dR, dphi)
        ctx.forward_steps = fw
        return J.clone()

    @staticmethod
    def backward(ctx, gJ):
        dA, dR, dphi = ctx.saved_tensors
        return gJ * dA, (None if dR is None else gJ * dR), gJ * dphi, None, None, None, None, None, None
