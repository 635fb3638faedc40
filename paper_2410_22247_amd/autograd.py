"""torch.autograd.Function around the adjoint-gradient entry point, and the Adam
driver that maximises the expected cut.

The forward pass calls aaq_energy_grad once (energy and the full gradient come out
of the same forward + adjoint sweep) and stores the gradient; the backward pass only
scales it by the incoming gradient.  Parameters live in float64 tensors on any device;
the library receives them as host arrays (2p doubles per call).
"""
from __future__ import annotations

import json
from typing import Optional

import numpy as np
import torch

from . import api


class QAOAEnergy(torch.autograd.Function):
    """E(gamma, beta) = <psi(gamma, beta)| H |psi(gamma, beta)> with the adjoint gradient.

    Usage: ``QAOAEnergy.apply(gamma, beta, estimator)``; gamma and beta are 1-D float64
    tensors of length p, ``estimator`` an ``api.Estimator`` built with grad=True."""

    @staticmethod
    def forward(ctx, gamma: torch.Tensor, beta: torch.Tensor, est: "api.Estimator"):
        g = gamma.detach().cpu().numpy().astype(np.float64)
        b = beta.detach().cpu().numpy().astype(np.float64)
        e, dg, db, _ = est.energy_grad(g, b)
        ctx.save_for_backward(torch.from_numpy(dg).to(gamma), torch.from_numpy(db).to(beta))
        return torch.tensor(e, dtype=torch.float64, device=gamma.device)

    @staticmethod
    def backward(ctx, grad_out):
        dg, db = ctx.saved_tensors
        return grad_out * dg, grad_out * db, None


def qaoa_energy(gamma: torch.Tensor, beta: torch.Tensor, est: "api.Estimator") -> torch.Tensor:
    return QAOAEnergy.apply(gamma, beta, est)


def adam_maximize(est: "api.Estimator", gamma0, beta0, steps: int = 200, lr: float = 0.01,
                  log_every: int = 0, device: str = "cpu"):
    """Maximise <H> (i.e. minimise -<H>) with torch.optim.Adam (default betas/eps).

    Returns (gamma, beta, history) where history[k] is the energy before step k."""
    gamma = torch.tensor(np.asarray(gamma0, dtype=np.float64), device=device, requires_grad=True)
    beta = torch.tensor(np.asarray(beta0, dtype=np.float64), device=device, requires_grad=True)
    opt = torch.optim.Adam([gamma, beta], lr=lr)
    hist = []
    for k in range(steps):
        opt.zero_grad()
        e = qaoa_energy(gamma, beta, est)
        (-e).backward()
        opt.step()
        hist.append(float(e.detach()))
        if log_every and k % log_every == 0:
            print(json.dumps({"step": k, "energy": hist[-1]}), flush=True)
    return gamma.detach().cpu().numpy(), beta.detach().cpu().numpy(), np.asarray(hist)


def adam_maximize_resident(res: "api.Resident", gamma0, beta0, steps: int = 200, lr: float = 0.01):
    """The same Adam loop with everything on the device: the parameters are one float64
    tensor [gamma, beta] on the evaluator's device, each step runs the resident
    evaluation (aaq_resident_execute) into a row of a device history and feeds
    -dE/dtheta to torch.optim.Adam, all in stream order with no host synchronisation.

    Returns (gamma, beta, history) with history[k] = [E, norm, dE/dgamma, dE/dbeta] at
    the parameters before step k (numpy, read once at the end)."""
    p = res.p
    x = torch.tensor(np.concatenate([np.asarray(gamma0, dtype=np.float64), np.asarray(beta0, dtype=np.float64)]),
                     device=res.params.device, requires_grad=True)
    opt = torch.optim.Adam([x], lr=lr)
    hist = torch.zeros(steps, 2 + 2 * p, dtype=torch.float64, device=x.device)
    for k in range(steps):
        res.execute(x.detach(), hist[k])
        x.grad = -hist[k, 2:]
        opt.step()
    xs = x.detach().cpu().numpy()
    return xs[:p], xs[p:], hist.cpu().numpy()
