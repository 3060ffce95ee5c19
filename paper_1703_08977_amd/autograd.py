"""torch.autograd.Function over the pathwise gradient (he_fk_grad).

``log_space_moments(theta, cfg)`` runs start ensemble + propagation (with
checkpoints) for trial parameters theta = (alpha, beta) and returns
L[s] = ln((1/N) sum_i w_i(t_s)) and L2[s] = ln((1/N) sum_i w_i(t_s)^2) as
float64 CPU tensors; its backward calls he_fk_grad, the reverse sweep over
the checkpoints at fixed start positions and fixed noise.  With ``score=True``
the backward also carries the derivative through the |psi_theta|^2 law the
start positions are drawn from, so that the gradient is that of the ensemble
expectation.  L2 - 2 L = ln(<w^2> / <w>^2) = -ln(ESS / N) is the log relative
variance of the weights.
"""
from __future__ import annotations

import numpy as np
import torch

from . import _lib, api


class _LogSpaceMoments(torch.autograd.Function):
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
        return torch.from_numpy(aux[:, 0].copy()), torch.from_numpy(aux[:, 2].copy())

    @staticmethod
    def backward(ctx, gL, gL2):
        ens, ckpt, samples, c, score = ctx.state
        n_steps, se, ce = c["n_steps"], c["sample_every"], c["ckpt_every"]
        nb = api.he_fk_grad_scratch_bytes(ens.p, n_steps, se, ce)
        scratch = torch.empty(nb, dtype=torch.uint8, device=ens.device)
        dtheta = torch.empty(2, dtype=torch.float64, device=ens.device)
        g = gL.detach().cpu().double().numpy()
        flags = _lib.GRAD_SCORE if score else 0
        g2 = gL2.detach().cpu().double().numpy() if gL2 is not None else None
        if g2 is not None and np.any(g2 != 0.0):
            g = np.concatenate([g, g2])
            flags |= _lib.GRAD_MOMENT2
        api.he_fk_grad(ens.p, ckpt.data_ptr(), samples.data_ptr(), g, n_steps, se, ce, flags, scratch.data_ptr(),
                       nb, dtheta.data_ptr())
        out = dtheta.cpu()
        ctx.state = None
        return out, None, None


def log_space_moments(theta: torch.Tensor, cfg: dict, score: bool = False):
    """(L[s], L2[s]) for trial parameters theta = (alpha, beta); differentiable with respect to theta."""
    return _LogSpaceMoments.apply(theta, cfg, score)


def log_space_average(theta: torch.Tensor, cfg: dict, score: bool = False) -> torch.Tensor:
    """L[s] for trial parameters theta = (alpha, beta); differentiable with respect to theta."""
    return _LogSpaceMoments.apply(theta, cfg, score)[0]


def energy_fd(L: torch.Tensor, cfg: dict) -> torch.Tensor:
    """E(T) = e_ref - (L[-1] - L[-2]) / dt_sample: the finite-difference energy at the last sample."""
    dts = cfg["dt"] * cfg["sample_every"]
    return cfg["e_ref"] - (L[-1] - L[-2]) / dts


def weight_variance(L: torch.Tensor, L2: torch.Tensor) -> torch.Tensor:
    """ln(<w^2> / <w>^2) at the last sample: the log relative variance of the path weights."""
    return L2[-1] - 2.0 * L[-1]


def descend(cfg: dict, steps: int | None = None, lr: float | None = None, score: bool = True, log=None,
            objective: str = "energy", first_step: float | None = None):
    """Gradient descent over (alpha, beta) at a fixed seed; returns the trace.

    objective "energy": E(T) by finite differences of L at the last two samples;
    "weight_variance": ln(<w^2> / <w>^2) at T, whose decrease raises the ESS at T;
    "el_variance": ln(<w^2> / <w>^2) / dt^2 after one step from the |psi|^2 start, i.e. the
    variance of E_L under |psi|^2 to leading order in dt (the variance criterion by which
    variational Monte Carlo tunes trial functions), on a one-step propagation of the same
    walkers.  With ``first_step`` the learning rate is set so that the first step moves theta
    by that distance (lr = first_step / |g_0|), then held fixed.
    """
    steps = cfg.get("gd_steps", 20) if steps is None else steps
    lr = cfg.get("gd_lr", 0.05) if lr is None else lr
    theta = torch.tensor(list(cfg["theta"][:2]), dtype=torch.float64, requires_grad=True)
    run = dict(cfg, n_steps=1, sample_every=1, ckpt_every=1) if objective == "el_variance" else cfg
    trace = []
    for it in range(steps + 1):
        L, L2 = log_space_moments(theta, run, score)
        V = weight_variance(L, L2)
        if objective == "energy":
            J = energy_fd(L, run)
        elif objective == "weight_variance":
            J = V
        else:
            J = V / (run["dt"] ** 2)
        E = energy_fd(L, run)
        J.backward()
        g = theta.grad.detach().clone()
        if it == 0 and first_step is not None:
            lr = first_step / max(float(g.norm()), 1e-300)
        th = theta.detach()
        row = {"iter": it, "alpha": float(th[0]), "beta": float(th[1]), "E": float(E.detach()),
               "log_rel_weight_var": float(V.detach()), "objective": objective, "J": float(J.detach()), "lr": lr,
               "dJ_dalpha": float(g[0]), "dJ_dbeta": float(g[1])}
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


__all__ = ["log_space_moments", "log_space_average", "energy_fd", "weight_variance", "descend"]
