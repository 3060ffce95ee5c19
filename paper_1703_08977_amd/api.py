"""Python binding of the C ABI: argument marshalling only.

Every step of the method runs in libhefk's kernels; torch supplies device
memory (``tensor.data_ptr()``) and the stream (``torch.cuda.current_stream()``).
The functions ``he_fk_init``, ``he_fk_propagate``, ``he_fk_energy`` and
``he_fk_grad`` carry the C names; ``Ensemble`` bundles the buffers of one
walker ensemble.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import HeFkParams, HeFkWalkers, check, lib


def make_params(cfg: dict, n_walkers: int | None = None, walker_offset: int = 0, **over) -> HeFkParams:
    """he_fk_params from a workload dict (see ``workloads``)."""
    c = dict(cfg)
    c.update(over)
    p = HeFkParams()
    p.trial = _lib.TRIAL[c["trial"]]
    p.sym = int(c.get("sym", 1))
    p.ee = int(c.get("ee", 1))
    p.noise = _lib.NOISE[c.get("noise", "gauss")]
    p.quad = _lib.QUAD[c.get("quad", "trapezoid")]
    p.contract = int(c.get("contract", 1))
    p.precision = _lib.PRECISION[c.get("precision", "fp64")]
    p.n_metropolis = int(c.get("n_metropolis", 500))
    p.flags = (_lib.FLAG_PLAIN if c.get("plain", False) else 0) | (_lib.FLAG_BRIDGE if c.get("bridge", False) else 0)
    p.Z = float(c.get("Z", 2.0))
    th = list(c["theta"]) + [0.0] * (6 - len(c["theta"]))
    for k in range(6):
        p.theta[k] = float(th[k])
    p.dt = float(c["dt"])
    p.e_ref = float(c.get("e_ref", 0.0))
    p.metropolis_sigma = float(c.get("metropolis_sigma", 0.5))
    p.init_sigma = float(c.get("init_sigma", 1.0))
    p.drift_limit = float(c.get("drift_limit", 0.0))
    p.seed = int(c.get("seed", 0)) & ((1 << 64) - 1)
    p.walker_offset = int(walker_offset)
    p.n_walkers = int(n_walkers if n_walkers is not None else c["n_walkers"])
    return p


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def walkers_struct(x: torch.Tensor, lnw: torch.Tensor, el: torch.Tensor) -> HeFkWalkers:
    return HeFkWalkers(x.data_ptr(), lnw.data_ptr(), el.data_ptr())


def he_fk_init(p: HeFkParams, w: HeFkWalkers, stream=None) -> int:
    return check(lib().he_fk_init(ctypes.byref(p), ctypes.byref(w), _stream(stream)), "he_fk_init")


def he_fk_propagate_workspace_bytes(p: HeFkParams, n_steps: int, sample_every: int) -> int:
    return int(lib().he_fk_propagate_workspace_bytes(ctypes.byref(p), int(n_steps), int(sample_every)))


def he_fk_propagate(p, w, step0, n_steps, sample_every, samples, ckpt, ckpt_every, workspace, workspace_bytes,
                    stream=None) -> int:
    rc = lib().he_fk_propagate(ctypes.byref(p), ctypes.byref(w), int(step0), int(n_steps), int(sample_every),
                               ctypes.c_void_p(samples), ctypes.c_void_p(ckpt or 0), int(ckpt_every),
                               ctypes.c_void_p(workspace), ctypes.c_size_t(workspace_bytes), _stream(stream))
    return check(rc, "he_fk_propagate")


def he_fk_propagate_noalloc(p, w, step0, n_steps, sample_every, samples, ckpt, ckpt_every, stream=None) -> int:
    rc = lib().he_fk_propagate_noalloc(ctypes.byref(p), ctypes.byref(w), int(step0), int(n_steps),
                                       int(sample_every), ctypes.c_void_p(samples), ctypes.c_void_p(ckpt or 0),
                                       int(ckpt_every), _stream(stream))
    return check(rc, "he_fk_propagate_noalloc")


def he_fk_energy(samples: np.ndarray, dt_sample: float, e_ref: float, method: str, fit_w=None, raise_on_error=True):
    """Host estimator; returns (E array, aux [n,3] = (L, ESS, L2), status code)."""
    s = np.ascontiguousarray(samples, dtype=np.float64)
    n = s.shape[0]
    m = _lib.E_METHOD[method]
    out = np.zeros({0: max(n - 1, 1), 1: 1, 2: 2, 3: n}[m])
    aux = np.zeros((n, 3))
    dp = ctypes.POINTER(ctypes.c_double)
    fw = None
    if fit_w is not None:
        fw = np.ascontiguousarray(fit_w, dtype=np.float64)
    rc = lib().he_fk_energy(s.ctypes.data_as(dp), n, float(dt_sample), float(e_ref), m,
                            fw.ctypes.data_as(dp) if fw is not None else None, out.ctypes.data_as(dp),
                            aux.ctypes.data_as(dp))
    if raise_on_error:
        check(rc, "he_fk_energy")
    return out, aux, rc


def he_fk_energy_blocks(partials: np.ndarray, dt_sample: float, e_ref: float, method: str, n_groups: int = 32,
                        fit_w=None):
    """(statistic of all blocks, its delete-one-group jackknife standard error) from the per-block
    partial rows [G, n_samples, 8] of one propagate call."""
    rows = np.ascontiguousarray(partials, dtype=np.float64)
    g, ns = rows.shape[0], rows.shape[1]
    out = np.zeros(2)
    dp = ctypes.POINTER(ctypes.c_double)
    fw = None if fit_w is None else np.ascontiguousarray(fit_w, dtype=np.float64)
    rc = lib().he_fk_energy_blocks(rows.ctypes.data_as(dp), g, ns, int(n_groups), float(dt_sample), float(e_ref),
                                   _lib.E_METHOD[method], fw.ctypes.data_as(dp) if fw is not None else None,
                                   out.ctypes.data_as(dp))
    check(rc, "he_fk_energy_blocks")
    return float(out[0]), float(out[1])


def he_fk_grad_scratch_bytes(p, n_steps, sample_every, ckpt_every) -> int:
    return int(lib().he_fk_grad_scratch_bytes(ctypes.byref(p), int(n_steps), int(sample_every), int(ckpt_every)))


def he_fk_grad(p, ckpt, samples, gL, n_steps, sample_every, ckpt_every, flags, scratch, scratch_bytes, dtheta,
               stream=None) -> int:
    g = np.ascontiguousarray(gL, dtype=np.float64)
    rc = lib().he_fk_grad(ctypes.byref(p), ctypes.c_void_p(ckpt), ctypes.c_void_p(samples),
                          g.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), int(n_steps), int(sample_every),
                          int(ckpt_every), int(flags), ctypes.c_void_p(scratch), ctypes.c_size_t(scratch_bytes),
                          ctypes.c_void_p(dtheta), _stream(stream))
    return check(rc, "he_fk_grad")


class Ensemble:
    """Device buffers of one walker ensemble (structure of arrays) plus its parameters."""

    def __init__(self, cfg: dict, n_walkers: int | None = None, walker_offset: int = 0, device="cuda", **over):
        self.cfg = dict(cfg)
        self.cfg.update(over)
        self.p = make_params(self.cfg, n_walkers, walker_offset)
        n = self.p.n_walkers
        real = torch.float32 if self.cfg.get("precision", "fp64") == "mixed" else torch.float64
        self.device = torch.device(device)
        self.x = torch.empty((6, n), dtype=real, device=self.device)
        self.lnw = torch.empty(n, dtype=torch.float64, device=self.device)
        self.el = torch.empty(n, dtype=real, device=self.device)
        self._ws = None

    @property
    def n(self) -> int:
        return int(self.p.n_walkers)

    def walkers(self) -> HeFkWalkers:
        return walkers_struct(self.x, self.lnw, self.el)

    def init(self, stream=None):
        he_fk_init(self.p, self.walkers(), stream)
        return self

    def workspace(self, n_steps, sample_every):
        nb = he_fk_propagate_workspace_bytes(self.p, n_steps, sample_every)
        if nb == 0:
            raise RuntimeError("he_fk_propagate_workspace_bytes returned 0 (invalid arguments or no device)")
        if self._ws is None or self._ws.numel() < nb:
            self._ws = torch.empty(nb, dtype=torch.uint8, device=self.device)
        return self._ws, nb

    def propagate(self, step0, n_steps, sample_every, samples=None, ckpt=None, ckpt_every=0, stream=None):
        """Returns the device tensor of sample rows [n_steps/sample_every + 1, 8]."""
        ns = n_steps // sample_every + 1
        if samples is None:
            samples = torch.empty((ns, 8), dtype=torch.float64, device=self.device)
        ws, nb = self.workspace(n_steps, sample_every)
        he_fk_propagate(self.p, self.walkers(), step0, n_steps, sample_every, samples.data_ptr(),
                        ckpt.data_ptr() if ckpt is not None else 0, ckpt_every, ws.data_ptr(), nb, stream)
        return samples

    def block_rows(self, n_steps, sample_every):
        """Per-block partial rows [G, n_samples, 8] left in the workspace by the last propagate."""
        ns = n_steps // sample_every + 1
        nb = he_fk_propagate_workspace_bytes(self.p, n_steps, sample_every)
        g = nb // (ns * 64)
        return self._ws[:nb].view(torch.float64).view(g, ns, 8)

    def state(self):
        """Host copies: x [N,6] (float64), lnw [N], el [N]."""
        return (self.x.double().t().contiguous().cpu().numpy(), self.lnw.cpu().numpy(),
                self.el.double().cpu().numpy())


def run(cfg: dict, n_walkers: int | None = None, seed: int | None = None) -> dict:
    """One whole pass of the path for a workload dict: start ensemble, propagation over
    cfg["n_steps"] steps sampled every cfg["sample_every"], and the estimators.

    Returns host arrays: the sample rows, L(t_s), the finite-difference energies E_fd, the
    window energy over [T/2, T] with its walker-block jackknife error, the mixed estimator and
    the ESS at every sample time."""
    c = dict(cfg) if seed is None else dict(cfg, seed=seed)
    ens = Ensemble(c, n_walkers=n_walkers).init()
    n_steps, se = c["n_steps"], c["sample_every"]
    rows = ens.propagate(0, n_steps, se).cpu().numpy()
    dts = c["dt"] * se
    e_fd, aux, _ = he_fk_energy(rows, dts, c["e_ref"], "fd")
    e_win = float(he_fk_energy(rows, dts, c["e_ref"], "window")[0][0])
    e_mix = he_fk_energy(rows, dts, c["e_ref"], "mixed")[0]
    _, err = he_fk_energy_blocks(ens.block_rows(n_steps, se).cpu().numpy(), dts, c["e_ref"], "window")
    return {"samples": rows, "t": np.arange(len(rows)) * dts, "L": aux[:, 0], "ess": aux[:, 1], "E_fd": e_fd,
            "E_window": e_win, "E_window_jackknife": float(err), "E_mixed": e_mix}

