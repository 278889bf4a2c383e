"""Gradients of the droplet deformation through the library's hand-written adjoint.

The deformation D of the shell (D_o) and of the core (D_i), the second-moment stand-in
for the deformation index of Eq. 42 taken from the order parameters, after `nsteps`
coupled steps from the compound droplet initial state, is differentiated with respect to

    theta = (H0, alpha, u_ref, sigma12, sigma13, sigma23)

(field strength and angle, Eq. 41 and Sec. 3; peak velocity of the Poiseuille drive; the
pairwise surface tensions of Eq. 27).  The forward keeps a checkpoint every `ckpt_every`
steps on the device; the backward recomputes one segment at a time and runs the adjoint
steps in reverse (all inside the HIP library, which also returns the u_ref component).
"""
from __future__ import annotations

import torch

from fcd_inputs import channel_drive

from . import fcd
from .sim import Batch, Channel

PARAM_NAMES = ("H0", "alpha", "u_ref", "sigma12", "sigma13", "sigma23")


def workload_at(w, theta):
    """The workload `w` with the six differentiated parameters replaced by `theta` (the
    drive is the one whose Poiseuille peak is u_ref)."""
    H0, alpha, u_ref, s12, s13, s23 = (float(v) for v in theta)
    return w.replace(H0=H0, alpha=alpha, u_ref=u_ref, sigma12=s12, sigma13=s13, sigma23=s23,
                     drive_G=channel_drive(u_ref, w.rho[2], w.tau[2], w.ny))


def theta_of(w):
    return [w.H0, w.alpha, w.u_ref, w.sigma12, w.sigma13, w.sigma23]


class AdjointRun:
    """Checkpointed forward + reverse sweep on one channel (device work buffer owned here)."""

    def __init__(self, ch: Channel, nsteps: int, ckpt_every: int):
        if nsteps < 1 or ckpt_every < 1:
            raise ValueError("need nsteps >= 1 and ckpt_every >= 1")
        self.ch, self.nsteps, self.every = ch, nsteps, ckpt_every
        nbytes = fcd.fcd_adjoint_bytes(ch.lat, nsteps, ckpt_every)
        if nbytes == 0:
            raise ValueError("fcd_adjoint_bytes rejected the lattice or sizes")
        # torch's caching allocator returns 512-byte aligned blocks
        self.work = torch.empty(nbytes, dtype=torch.uint8, device=ch.device)
        self.D = None

    def forward(self, theta) -> list:
        """Re-initialise the channel at theta, run nsteps and return [D_o, D_i]."""
        ch = self.ch
        ch.set_workload(workload_at(ch.w, theta))
        ch.init_droplet()
        self.D = fcd.fcd_adjoint_forward(ch.h, self.nsteps, self.every, self.work.data_ptr())
        return list(self.D)

    def backward(self, dJ_dD) -> list:
        """dJ/dtheta for J = dJ_dD[0] D_o + dJ_dD[1] D_i of the last forward."""
        if self.D is None:
            raise RuntimeError("forward has not run")
        return list(fcd.fcd_adjoint_backward(self.ch.h, [float(dJ_dD[0]), float(dJ_dD[1])]))


class DeformationFunction(torch.autograd.Function):
    """theta (6, float64) -> (D_o, D_i) with a hand-written adjoint backward.

    Usage: DeformationFunction.apply(theta, AdjointRun(channel, nsteps, ckpt_every)).
    """

    @staticmethod
    def forward(ctx, theta: torch.Tensor, run: AdjointRun):
        D = run.forward(theta.detach().cpu().tolist())
        ctx.run = run
        return torch.tensor(D, dtype=torch.float64)

    @staticmethod
    def backward(ctx, grad_D: torch.Tensor):
        g = ctx.run.backward(grad_D.detach().cpu().tolist())
        return torch.tensor(g, dtype=torch.float64), None


def deformation(theta: torch.Tensor, run: AdjointRun) -> torch.Tensor:
    return DeformationFunction.apply(theta, run)


class BatchAdjointRun:
    """The checkpointed forward and reverse sweep of every channel of a batch at once."""

    def __init__(self, bt: Batch, nsteps: int, ckpt_every: int):
        if nsteps < 1 or ckpt_every < 1:
            raise ValueError("need nsteps >= 1 and ckpt_every >= 1")
        self.bt, self.nsteps, self.every = bt, nsteps, ckpt_every
        nbytes = fcd.fcd_batch_adjoint_bytes(bt.h, nsteps, ckpt_every)
        if nbytes == 0:
            raise ValueError("fcd_batch_adjoint_bytes rejected the sizes")
        self.work = torch.empty(nbytes, dtype=torch.uint8, device=bt.device)
        self.D = None

    def forward(self) -> list:
        """Run nsteps from the batch's current state; [(D_o, D_i)] per channel."""
        self.D = fcd.fcd_batch_adjoint_forward(self.bt.h, self.bt.n, self.nsteps, self.every, self.work.data_ptr())
        return self.D

    def backward(self, dJ_dD) -> list:
        """Per channel dJ/d(H0, alpha, u_ref, sigma12, sigma13, sigma23)."""
        if self.D is None:
            raise RuntimeError("forward has not run")
        g = fcd.fcd_batch_adjoint_backward(self.bt.h, [(float(a), float(b)) for a, b in dJ_dD])
        return [list(gk) for gk in g]
