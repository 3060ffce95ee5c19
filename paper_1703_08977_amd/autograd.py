"""torch.autograd.Function over the pathwise gradient (he_fk_grad).

``log_space_average(theta, cfg)`` runs start ensemble + propagation (with
checkpoints) for trial parameters theta = (alpha, beta) and returns
L[s] = ln((1/N) sum_i w_i(t_s)) as a float64 CPU tensor; its backward calls
he_fk_grad, the reverse sweep over the checkpoints at fixed start positions
and fixed noise.  With ``score=True`` the backward also carries the derivative
through the |psi_theta|^2 law the start positions are drawn from, so that the
gradient is that of the ensemble expectation.
"""
from __future__ import annotations

import torch

from . import _lib, api


class _LogSpaceAverage(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta, cfg, score):
        th = theta.detach().cpu().double().numpy()
        c = dict(cfg)
        full = list(c["theta"]) + [0.0] * (4 - len(c["theta"]))
        full[0], full[1] = float(th[0]), float(th[1])
        c["theta"] = full
        n_steps, se, ce = c["n_steps"], c["sample_every"], c["ckpt_every"]
        ens = api.Ensemble(c).init()
        ckpt = torch.empty((n_steps // ce + 1, 7, ens.n), dtype=torch.float64, device=ens.device)
        samples = ens.propagate(0, n_steps, se, ckpt=ckpt, ckpt_every=ce)
        host = samples.cpu().numpy()
        _, aux, _ = api.he_fk_energy(host, c["dt"] * se, c["e_ref"], "fd")
        ctx.state = (ens, ckpt, samples, c, bool(score))
        return torch.from_numpy(aux[:, 0].copy())

    @staticmethod
    def backward(ctx, gL):
        ens, ckpt, samples, c, score = ctx.state
        n_steps, se, ce = c["n_steps"], c["sample_every"], c["ckpt_every"]
        nb = api.he_fk_grad_scratch_bytes(ens.p, n_steps, se, ce)
        scratch = torch.empty(nb, dtype=torch.uint8, device=ens.device)
        dtheta = torch.empty(2, dtype=torch.float64, device=ens.device)
        api.he_fk_grad(ens.p, ckpt.data_ptr(), samples.data_ptr(), gL.detach().cpu().double().numpy(), n_steps,
                       se, ce, _lib.GRAD_SCORE if score else 0, scratch.data_ptr(), nb, dtheta.data_ptr())
        g = dtheta.cpu()
        ctx.state = None
        return g, None, None


def log_space_average(theta: torch.Tensor, cfg: dict, score: bool = False) -> torch.Tensor:
    """L[s] for trial parameters theta = (alpha, beta); differentiable with respect to theta."""
    return _LogSpaceAverage.apply(theta, cfg, score)


def energy_fd(L: torch.Tensor, cfg: dict) -> torch.Tensor:
    """E(T) = e_ref - (L[-1] - L[-2]) / dt_sample: the finite-difference energy at the last sample."""
    dts = cfg["dt"] * cfg["sample_every"]
    return cfg["e_ref"] - (L[-1] - L[-2]) / dts


def descend(cfg: dict, steps: int | None = None, lr: float | None = None, score: bool = True, log=None):
    """Plain gradient descent of E(T) over (alpha, beta) at a fixed seed; returns the trace."""
    steps = cfg.get("gd_steps", 20) if steps is None else steps
    lr = cfg.get("gd_lr", 0.05) if lr is None else lr
    theta = torch.tensor(list(cfg["theta"][:2]), dtype=torch.float64, requires_grad=True)
    trace = []
    for it in range(steps + 1):
        L = log_space_average(theta, cfg, score)
        E = energy_fd(L, cfg)
        E.backward()
        g = theta.grad.detach().clone()
        row = {"iter": it, "alpha": float(theta[0]), "beta": float(theta[1]), "E": float(E),
               "dE_dalpha": float(g[0]), "dE_dbeta": float(g[1])}
        trace.append(row)
        if log:
            log(row)
        if it == steps:
            break
        with torch.no_grad():
            theta -= lr * g
            theta[1].clamp_(min=0.0)
        theta.grad = None
    return trace


__all__ = ["log_space_average", "energy_fd", "descend"]
