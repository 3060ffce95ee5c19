"""Plain FP64 CPU oracle for the generalized Feynman-Kac walker propagation.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py``; the product package never imports
it.  The arithmetic lives in ``he_fk_oracle.c`` (Philox, trial functions,
Metropolis start, propagation, log-domain space average, complex-step
pathwise derivatives); ``estimators.py`` holds the energy estimators.  This
module only marshals arguments and builds the C file with gcc.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "he_fk_oracle.c")
_LIB = os.path.join(_HERE, "libhefk_oracle.so")

TRIALS = {"expo": 0, "pade": 1, "triplet": 2, "pz": 3, "triplet_r0": 4, "pz_sum": 5}
NOISE = {"gauss": 0, "pm1": 1}
QUAD = {"trapezoid": 0, "right": 1}
FLAG_PLAIN = 1   # plain Feynman-Kac walk (no drift, integrand V)
FLAG_BRIDGE = 2  # node-touch (Brownian bridge) survival weight per step


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Params(ctypes.Structure):
    _fields_ = [
        ("trial", ctypes.c_int32), ("sym", ctypes.c_int32), ("ee", ctypes.c_int32),
        ("noise", ctypes.c_int32), ("quad", ctypes.c_int32), ("contract", ctypes.c_int32),
        ("n_metropolis", ctypes.c_int32), ("flags", ctypes.c_int32),
        ("Z", ctypes.c_double), ("theta", ctypes.c_double * 6), ("dt", ctypes.c_double),
        ("e_ref", ctypes.c_double), ("metropolis_sigma", ctypes.c_double),
        ("init_sigma", ctypes.c_double), ("drift_limit", ctypes.c_double), ("seed", ctypes.c_uint64),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        P = ctypes.POINTER
        u64p, dp, ip, u32p = P(ctypes.c_uint64), P(ctypes.c_double), P(ctypes.c_int), P(ctypes.c_uint32)
        pp = P(_Params)
        L.ofk_philox4x32_10.argtypes = [u32p, u32p, u32p]
        L.ofk_init.argtypes = [pp, u64p, ctypes.c_int64, dp, dp]
        L.ofk_propagate.argtypes = [pp, u64p, ctypes.c_int64, dp, dp, dp, ctypes.c_int64, ctypes.c_int64,
                                    ctypes.c_int64, dp, dp, dp]
        L.ofk_tuples.argtypes = [dp, dp, ctypes.c_int64, ctypes.c_int64, dp]
        L.ofk_dlnw_dtheta.argtypes = [pp, u64p, ctypes.c_int64, dp, ctypes.c_int64, ctypes.c_int64,
                                      ctypes.c_int, dp, ip]
        L.ofk_dlnpsi_dtheta.argtypes = [pp, dp, ctypes.c_int]
        L.ofk_dlnpsi_dtheta.restype = ctypes.c_double
        L.ofk_gauss6_c1.argtypes = [pp, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint64, dp, dp]
        L.ofk_gauss6_c2.argtypes = [pp, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint64, dp]
        L.ofk_pm1_6.argtypes = [pp, ctypes.c_uint64, ctypes.c_uint64, dp]
        L.ofk_num_threads.restype = ctypes.c_int
        L.ofk_noise_bulk.argtypes = [pp, ctypes.c_uint64, u64p, ctypes.c_int64, dp]
        _lib = L
    return _lib


def _ptr(a, t=ctypes.c_double):
    return a.ctypes.data_as(ctypes.POINTER(t))


@dataclass
class Eval:
    lnpsi: float
    sign: int
    b: np.ndarray
    el: float
    V: float
    gphi2: float


class _Eval(ctypes.Structure):
    _fields_ = [("lnpsi", ctypes.c_double), ("sign", ctypes.c_int), ("b", ctypes.c_double * 6),
                ("el", ctypes.c_double), ("V", ctypes.c_double), ("gphi2", ctypes.c_double)]


def params(cfg: dict) -> _Params:
    """Oracle parameter block from a workload dict (see paper_1703_08977_amd.workloads)."""
    p = _Params()
    p.trial = TRIALS[cfg["trial"]]
    p.sym = int(cfg.get("sym", 1))
    p.ee = int(cfg.get("ee", 1))
    p.noise = NOISE[cfg.get("noise", "gauss")]
    p.quad = QUAD[cfg.get("quad", "trapezoid")]
    p.contract = int(cfg.get("contract", 1))
    p.n_metropolis = int(cfg.get("n_metropolis", 500))
    p.flags = (FLAG_PLAIN if cfg.get("plain", False) else 0) | (FLAG_BRIDGE if cfg.get("bridge", False) else 0)
    p.Z = float(cfg.get("Z", 2.0))
    th = list(cfg["theta"]) + [0.0] * (6 - len(cfg["theta"]))
    for i in range(6):
        p.theta[i] = float(th[i])
    p.dt = float(cfg["dt"])
    p.e_ref = float(cfg.get("e_ref", 0.0))
    p.metropolis_sigma = float(cfg.get("metropolis_sigma", 0.5))
    p.init_sigma = float(cfg.get("init_sigma", 1.0))
    p.drift_limit = float(cfg.get("drift_limit", 0.0))
    p.seed = int(cfg.get("seed", 0)) & ((1 << 64) - 1)
    return p


def philox(ctr, key):
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    o = np.zeros(4, dtype=np.uint32)
    lib().ofk_philox4x32_10(_ptr(c, ctypes.c_uint32), _ptr(k, ctypes.c_uint32), _ptr(o, ctypes.c_uint32))
    return o


def trial_eval(cfg, y) -> Eval:
    L = lib()
    if not hasattr(L, "_eval_set"):
        L.ofk_trial_eval.argtypes = [ctypes.POINTER(_Params), ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(_Eval)]
        L._eval_set = True
    p = params(cfg)
    y = np.ascontiguousarray(y, dtype=np.float64)
    e = _Eval()
    L.ofk_trial_eval(ctypes.byref(p), _ptr(y), ctypes.byref(e))
    return Eval(e.lnpsi, e.sign, np.array(e.b[:]), e.el, e.V, e.gphi2)


def gauss6(cfg, phase, blk, g, contract=1):
    p = params(cfg)
    xi = np.zeros(6)
    sp = np.zeros(1)
    if contract == 1:
        lib().ofk_gauss6_c1(ctypes.byref(p), phase, blk, g, _ptr(xi), _ptr(sp))
    else:
        lib().ofk_gauss6_c2(ctypes.byref(p), phase, blk, g, _ptr(xi))
    return xi, sp[0]


def pm1_6(cfg, k, g):
    p = params(cfg)
    e = np.zeros(6)
    lib().ofk_pm1_6(ctypes.byref(p), k, g, _ptr(e))
    return e


def noise_bulk(cfg, k, ids):
    """Propagation noise of step k (Gaussian by contract, or +/-1) for the given walkers: [n, 6]."""
    ids = np.ascontiguousarray(np.asarray(ids, dtype=np.uint64))
    out = np.zeros((ids.size, 6))
    lib().ofk_noise_bulk(ctypes.byref(params(cfg)), k, _ptr(ids, ctypes.c_uint64), ids.size, _ptr(out))
    return out


def _ids(ids):
    return np.ascontiguousarray(np.asarray(ids, dtype=np.uint64))


def init(cfg, ids):
    """Metropolis start: x [n,6], el [n] for the given walker ids."""
    ids = _ids(ids)
    n = ids.size
    x = np.zeros((n, 6))
    el = np.zeros(n)
    lib().ofk_init(ctypes.byref(params(cfg)), _ptr(ids, ctypes.c_uint64), n, _ptr(x), _ptr(el))
    return x, el


def propagate(cfg, ids, x, lnw, step0, n_steps, sample_every, record=True, node_dmin=False):
    """Advance walkers (copies); returns (x, lnw, el, ell[n,ns], els[n,ns]), and with
    ``node_dmin`` also the smallest node-distance estimate 1/|grad ln|Phi|| each walker's
    path held while alive ([n], a diagnostic)."""
    ids = _ids(ids)
    n = ids.size
    x = np.ascontiguousarray(x, dtype=np.float64).copy()
    lnw = np.ascontiguousarray(lnw, dtype=np.float64).copy()
    el = np.zeros(n)
    ns = n_steps // sample_every + 1
    ell = np.zeros((n, ns)) if record else None
    els = np.zeros((n, ns)) if record else None
    dmin = np.zeros(n) if node_dmin else None
    lib().ofk_propagate(ctypes.byref(params(cfg)), _ptr(ids, ctypes.c_uint64), n, _ptr(x), _ptr(lnw), _ptr(el),
                        step0, n_steps, sample_every, _ptr(ell) if record else None,
                        _ptr(els) if record else None, _ptr(dmin) if node_dmin else None)
    if node_dmin:
        return x, lnw, el, ell, els, dmin
    return x, lnw, el, ell, els


def tuples(ell, els):
    """Per-sample (m, S0, S1, S2, n_alive, n_nonfinite, n_total, 0) rows."""
    ell = np.ascontiguousarray(ell, dtype=np.float64)
    els = np.ascontiguousarray(els, dtype=np.float64)
    n, ns = ell.shape
    out = np.zeros((ns, 8))
    lib().ofk_tuples(_ptr(ell), _ptr(els), n, ns, _ptr(out))
    return out


def run(cfg, ids, n_steps, sample_every):
    """Start + propagate from step 0; returns dict with final state, sample tuples and the
    node-distance diagnostic of each walker's path."""
    x0, el0 = init(cfg, ids)
    lnw0 = np.zeros(len(x0))
    x, lnw, el, ell, els, dmin = propagate(cfg, ids, x0, lnw0, 0, n_steps, sample_every, node_dmin=True)
    return {"x0": x0, "el0": el0, "x": x, "lnw": lnw, "el": el, "ell": ell, "els": els,
            "samples": tuples(ell, els), "n_steps": n_steps, "sample_every": sample_every, "node_dmin": dmin}


def dlnw_dtheta(cfg, ids, y0, n_steps, sample_every, direction):
    """Complex-step d lnw / d theta_direction at every sample time: [n, ns]."""
    ids = _ids(ids)
    n = ids.size
    y0 = np.ascontiguousarray(y0, dtype=np.float64)
    ns = n_steps // sample_every + 1
    out = np.zeros((n, ns))
    st = ctypes.c_int(0)
    lib().ofk_dlnw_dtheta(ctypes.byref(params(cfg)), _ptr(ids, ctypes.c_uint64), n, _ptr(y0), n_steps,
                          sample_every, direction, _ptr(out), ctypes.byref(st))
    if st.value != 0:
        raise ValueError("complex-step derivative supports the nodeless trials only")
    return out


def dlnpsi_dtheta(cfg, y0, direction):
    p = params(cfg)
    y0 = np.ascontiguousarray(y0, dtype=np.float64)
    return np.array([lib().ofk_dlnpsi_dtheta(ctypes.byref(p), _ptr(y0[i]), direction) for i in range(len(y0))])


def grad_objective(cfg, ids, y0, n_steps, sample_every, gL, score=False, gL2=None):
    """d/d(alpha, beta) of J = sum_s gL_s L_s + sum_s gL2_s L2_s at fixed Y0 and noise, with
    L_s = ln( (1/N) sum_i w_is ) and L2_s = ln( (1/N) sum_i w_is^2 ).

    dL_s/dtheta = sum_i p_is d l_is / dtheta, p_is = w_is / sum_i w_is, and
    dL2_s/dtheta = sum_i q_is 2 d l_is / dtheta, q_is = w_is^2 / sum_i w_is^2.  With
    ``score`` the derivative of the |psi|^2 start law is added through the score
    s_i = 2 d ln|psi(Y0_i)|/dtheta: sum_i (p_is - 1/N) s_i for L_s and sum_i (q_is - 1/N) s_i
    for L2_s (each a derivative of a log of an average over the start law).
    """
    ids = _ids(ids)
    x, lnw, el, ell, els = propagate(cfg, ids, y0, np.zeros(len(y0)), 0, n_steps, sample_every)
    m = ell.max(axis=0)
    w = np.exp(ell - m)
    p = w / w.sum(axis=0)
    q = w * w / (w * w).sum(axis=0)
    g = np.zeros(2)
    gL = np.asarray(gL, dtype=np.float64)
    gL2 = np.zeros_like(gL) if gL2 is None else np.asarray(gL2, dtype=np.float64)
    for d in range(2):
        dl = dlnw_dtheta(cfg, ids, y0, n_steps, sample_every, d)
        g[d] = float(np.sum(gL * np.sum(p * dl, axis=0)) + np.sum(gL2 * np.sum(q * 2.0 * dl, axis=0)))
        if score:
            s = 2.0 * dlnpsi_dtheta(cfg, y0, d)
            g[d] += float(np.sum(gL * ((p - 1.0 / len(ids)) * s[:, None]).sum(axis=0)))
            g[d] += float(np.sum(gL2 * ((q - 1.0 / len(ids)) * s[:, None]).sum(axis=0)))
    return g


def num_threads() -> int:
    return int(lib().ofk_num_threads())


def set_num_threads(n: int) -> None:
    """Threads of the oracle's parallel loops from here on."""
    lib().ofk_set_num_threads(int(n))
