"""Shared helpers of the tests: running the HIP path through the C ABI and
comparing with the oracle.  No arithmetic of the method lives here."""
from __future__ import annotations

import os
import subprocess

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1703_08977_amd", "csrc")


def gpu_available() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def gpu_run(cfg, n_walkers=None, n_steps=None, sample_every=None, walker_offset=0, ckpt_every=0):
    """init + propagate on the GPU through the C ABI; returns host arrays."""
    import torch
    from paper_1703_08977_amd import Ensemble
    n_steps = cfg["n_steps"] if n_steps is None else n_steps
    sample_every = cfg["sample_every"] if sample_every is None else sample_every
    ens = Ensemble(cfg, n_walkers=n_walkers, walker_offset=walker_offset)
    ens.init()
    x0, _, el0 = ens.state()
    ckpt = None
    if ckpt_every:
        ckpt = torch.empty((n_steps // ckpt_every + 1, 7, ens.n), dtype=torch.float64, device="cuda")
    s = ens.propagate(0, n_steps, sample_every, ckpt=ckpt, ckpt_every=ckpt_every)
    torch.cuda.synchronize()
    x, lnw, el = ens.state()
    out = {"x0": x0, "el0": el0, "x": x, "lnw": lnw, "el": el, "samples": s.cpu().numpy(), "ens": ens}
    if ckpt is not None:
        out["ckpt"] = ckpt
    return out


def rel_err(a, b):
    """|a - b| / max(1, |b|), elementwise; equal infinities give 0."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    same = (a == b)
    d = np.abs(a - b) / np.maximum(1.0, np.abs(b))
    return np.where(same, 0.0, d)


def log_mean_weight(samples):
    """L = m + ln S0 - ln N per sample row (-inf where every walker is absorbed)."""
    s = np.asarray(samples, dtype=np.float64)
    with np.errstate(divide="ignore"):
        return s[:, 0] + np.log(s[:, 1]) - np.log(s[:, 6])


_HARNESS = None


def host_harness():
    """Build (once) the host build of the kernels' per-walker code."""
    global _HARNESS
    if _HARNESS is None:
        import shutil
        import tempfile
        hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
        exe = os.path.join(tempfile.mkdtemp(prefix="hefk_host_"), "device_code_host_check")
        subprocess.check_call([hipcc, "-O2", "-std=c++17", "--offload-arch=gfx950", "-I", CSRC, "-I",
                               os.path.join(ROOT, "include"), "-o", exe,
                               os.path.join(ROOT, "tests", "device_code_host_check.cpp")],
                              stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
        _HARNESS = exe
    return _HARNESS


def host_run(cfg, ids, n_steps, sample_every, precision=0):
    import oracle
    th = list(cfg["theta"]) + [0.0] * 4
    flags = (oracle.FLAG_PLAIN if cfg.get("plain", False) else 0) | (oracle.FLAG_BRIDGE if cfg.get("bridge", False) else 0)
    line = "%d %d %d %d %d %d %d %d %d %r %r %r %r %r %r %r %r %r %r %r %d %d %d" % (
        oracle.TRIALS[cfg["trial"]], cfg.get("sym", 1), cfg.get("ee", 1),
        1 if cfg.get("noise", "gauss") == "pm1" else 0, cfg.get("contract", 1),
        1 if cfg.get("quad", "trapezoid") == "right" else 0, precision, cfg.get("n_metropolis", 500), flags,
        float(cfg["Z"]), *[float(v) for v in th[:5]], float(cfg["dt"]), float(cfg["e_ref"]),
        float(cfg.get("metropolis_sigma", 0.5)), float(cfg.get("init_sigma", 1.0)),
        float(cfg.get("drift_limit", 0.0)), int(cfg["seed"]), n_steps,
        sample_every)
    inp = line + "\n%d %s\n" % (len(ids), " ".join(str(int(i)) for i in ids))
    out = subprocess.run([host_harness()], input=inp, capture_output=True, text=True, check=True).stdout
    ns = n_steps // sample_every + 1
    arr = np.array([[float(v) for v in ln.split()] for ln in out.strip().split("\n")])
    return {"x0": arr[:, :6], "x": arr[:, 6:12], "lnw": arr[:, 12], "el": arr[:, 13],
            "ell": arr[:, 14:14 + ns], "els": arr[:, 14 + ns:]}


_ADJ = None


def adjoint_harness():
    """Build (once) the host build of the gradient's per-walker reverse sweep."""
    global _ADJ
    if _ADJ is None:
        import shutil
        import tempfile
        hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
        exe = os.path.join(tempfile.mkdtemp(prefix="hefk_adj_"), "adjoint_host_check")
        subprocess.check_call([hipcc, "-O2", "-std=c++17", "--offload-arch=gfx950", "-I", CSRC, "-I",
                               os.path.join(ROOT, "include"), "-o", exe,
                               os.path.join(ROOT, "tests", "adjoint_host_check.cpp")],
                              stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
        _ADJ = exe
    return _ADJ


def adjoint_host_run(cfg, ids, n_steps, sample_every, ckpt_every, samples, g, g2=None):
    """Per-walker (dJ/dalpha, dJ/dbeta, P, Q) from the host build of the reverse sweep."""
    g2 = np.zeros(len(samples)) if g2 is None else g2
    import oracle
    th = [float(v) for v in (list(cfg["theta"]) + [0.0] * 4)[:4]]
    line = "%d %d %d %d %d %r %r %r %r %r %r %r %r %r %d %d %d %d" % (
        oracle.TRIALS[cfg["trial"]], cfg["ee"], 1 if cfg.get("quad") == "right" else 0, cfg.get("contract", 1),
        cfg["n_metropolis"], float(cfg["Z"]), *th, float(cfg["dt"]), float(cfg["e_ref"]),
        float(cfg["metropolis_sigma"]), float(cfg["init_sigma"]), int(cfg["seed"]), n_steps, sample_every,
        ckpt_every)
    l2 = "%d " % len(samples) + " ".join("%r %r %r %r %r" % (float(samples[s, 0]), float(samples[s, 1]),
                                                            float(samples[s, 3]), float(g[s]), float(g2[s]))
                                         for s in range(len(samples)))
    inp = line + "\n" + l2 + "\n%d %s\n" % (len(ids), " ".join(str(int(i)) for i in ids))
    out = subprocess.run([adjoint_harness()], input=inp, capture_output=True, text=True, check=True).stdout
    return np.array([[float(v) for v in ln.split()] for ln in out.strip().split("\n")])
