"""Autograd binding of the adjoint along prescribed nuclear paths.

``path_loss(theta, paths, ...)`` returns the per-path losses of the
double-well Newns-Anderson model (Sec. III.B) whose parameters are
``theta = [eps_d, Gamma, eps_1 .. eps_M, omega, g, dG]``; its backward pass
runs ``iesh_adjoint_backward`` in libiesh (checkpointed reverse sweep on the
GPU).  The loss and the gradient layout are those of include/iesh.h.  This
module only marshals arguments.
"""
from __future__ import annotations

import numpy as np
import torch

from ._lib import Ensemble, model_desc

__all__ = ["PathLoss", "path_loss", "ensemble_for"]


def ensemble_for(theta, bath_w, mass, n_elec, n_traj, dt):
    """An FP64 ensemble of the harmonic model with parameters theta."""
    theta = np.asarray(theta, dtype=np.float64)
    M = len(bath_w)
    if theta.shape != (M + 5,):
        raise ValueError(f"theta must have M + 5 = {M + 5} entries")
    model = {"kind": "harmonic", "mass": float(mass), "Gamma": float(theta[1]),
             "omega": float(theta[2 + M]), "g": float(theta[3 + M]), "dG": float(theta[4 + M]),
             "eps_d": float(theta[0])}
    d = model_desc(model, theta[2:2 + M].copy(), np.asarray(bath_w, dtype=np.float64), n_elec)
    return Ensemble([d], {"n_traj": int(n_traj), "dt": float(dt), "precision": "fp64"})


class PathLoss(torch.autograd.Function):
    """losses (n_traj,) = L(theta; paths); d/dtheta through the GPU adjoint."""

    @staticmethod
    def forward(ctx, theta, paths, bath_w, mass, n_elec, dt, ckpt_every, terms):
        p = np.ascontiguousarray(paths.detach().cpu().numpy() if torch.is_tensor(paths) else paths,
                                 dtype=np.float64)
        ens = ensemble_for(theta.detach().cpu().numpy(), bath_w, mass, n_elec, p.shape[0], dt)
        loss = ens.adjoint_forward(p, ckpt_every, terms)
        ctx.ens = ens
        ctx.n_par = theta.shape[0]
        ctx.theta_dtype, ctx.theta_device = theta.dtype, theta.device
        return torch.from_numpy(loss).to(dtype=theta.dtype, device=theta.device)

    @staticmethod
    def backward(ctx, gout):
        w = gout.detach().to(torch.float64).cpu().numpy()
        rows = ctx.ens.adjoint_backward(w)
        g = rows[:, :ctx.n_par].sum(axis=0)
        gt = torch.from_numpy(g).to(dtype=ctx.theta_dtype, device=ctx.theta_device)
        return gt, None, None, None, None, None, None, None


def path_loss(theta, paths, bath_w, mass, n_elec, dt, ckpt_every=100, terms=(1.0, 1.0, 0.0, 0.0)):
    """Per-path losses, differentiable in theta (a float64 tensor of M + 5);
    terms = weights of the population, excitation, hop and force terms."""
    return PathLoss.apply(theta, paths, bath_w, mass, n_elec, dt, ckpt_every, tuple(terms))
