"""Algorithmic VALU work of one walker step and the MI355X VALU issue peak.

The step is per-walker scalar arithmetic (transcendental, integer and
floating point; no contraction, no HBM traffic between sampling times), so
its roofline is the vector-ALU issue rate.

Peak: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 39.32e12 lane-operations/s,
one operation per lane per clock (a wave64 instruction occupies a 16-lane
SIMD for 4 clocks).  This is the published 78.6 TFLOP/s binary32 (and
binary64) FMA rate divided by 2 flops; the 157.3 TFLOP/s binary32 figure
needs packed (v_pk_*) instructions, which this build does not use.

Work: every elementary operation of the step's formulas counts one issue
slot -- add, mul, fma, compare, select, convert, 32-bit integer op, 32x32->64
multiply, and each binary32 hardware transcendental (v_sqrt, v_rcp, v_exp,
v_log, v_sin, v_cos).  On gfx950 these all issue at the full rate: the
compiled binary32 step of the P_z trial has 318 VALU instructions and runs at
1024 x 2.4e9 x 16 / 318 = 1.24e11 walker-steps/s, the measured rate.  Binary64
library functions count their polynomial evaluation and range reduction:
sqrt 8, division 10, exp 20, expm1 25, log 25, sincospi 35.
Counts are per term of the formulas (they are not read back from the
compiled code); the tables below list them.
"""
from __future__ import annotations

PEAK_SLOTS_PER_S = 256 * 4 * 16 * 2.4e9  # 39.32e12

# Philox4x32-10 block per step: 10 rounds x (two 32x32->64 multiplies, four xors), less the
# work that depends only on the walker id, the phase and the key (round 1 and the first
# multiply of round 2, computed once per walker); the key schedule runs on the scalar unit.
PHILOX_BLOCK = 9 * (2 + 4) - 1

# "log" is -2 ln x (the Box-Muller radius argument) including its constant factor
F32 = {"sqrt": 1, "rcp": 1, "exp": 2, "expm1": 10, "log": 2, "sincos": 2}
F64 = {"sqrt": 8, "rcp": 10, "exp": 20, "expm1": 25, "log": 26, "sincos": 35}


def noise_slots(precision: str, noise: str, contract: int) -> float:
    f = F32 if precision == "mixed" else F64
    if noise == "pm1":
        return PHILOX_BLOCK / 20.0 + 6 * 2  # one block per 20 steps; bit extract + select per coordinate
    box_muller = 3 * (f["log"] + f["sqrt"] + f["sincos"] + 2)
    if contract == 2:
        return PHILOX_BLOCK + 14 + 6 * 2 + box_muller  # 21-bit field extraction, convert + scale
    per_uniform = 2 if precision == "mixed" else 2  # funnel shift + add (binary32); convert + scale (binary64)
    return 2 * PHILOX_BLOCK + 6 * per_uniform + box_muller


def trial_slots(precision: str, trial: str) -> float:
    f = F32 if precision == "mixed" else F64
    geometry = 3 + 3 * (3 + f["sqrt"]) + 3 * f["rcp"] + 9  # differences, norms, inverses, unit vectors
    jastrow = 1 + f["rcp"] + 1 + 1 + 2 + 4
    swap = 9 + 12  # half-space test, electrons in, drift out
    if trial == "expo":
        return geometry + 6 + 3
    if trial == "pade":
        return geometry + jastrow + 12 + 6 + 7
    if trial == "triplet":
        return geometry + jastrow + swap + 2 + f["expm1"] + 1 + f["rcp"] + 4 + 8 + 6 + 12 + 10 + 2
    return geometry + jastrow + swap + 2 + f["exp"] + 1 + 1 + f["rcp"] + 6 + 15 + 14 + 6 + 6 + 8 + 4  # pz


def slots_per_walker_step(cfg: dict) -> float:
    """Issue slots of one walker step: noise, Euler step, trial evaluation, limiting,
    node test and state commit, ln w update."""
    prec = cfg.get("precision", "fp64")
    f = F32 if prec == "mixed" else F64
    n = noise_slots(prec, cfg.get("noise", "gauss"), int(cfg.get("contract", 1)))
    t = trial_slots(prec, cfg["trial"])
    euler = 12
    limit = (6 + 1 + 1 + f["sqrt"] + 1 + f["rcp"] + 1 + 6 + 1) if cfg.get("drift_limit", 0.0) > 0 else 0
    node = 6
    lnw = 6
    return float(n + t + euler + limit + node + lnw)


def fp32_flops_per_walker_step(cfg: dict) -> float:
    """binary32 floating-point operations of one mixed step (fma = 2, transcendental = 1)."""
    if cfg.get("precision", "fp64") != "mixed":
        return 0.0
    base = {"expo": 50, "pade": 85, "triplet": 125, "pz": 140}[cfg["trial"]]
    noise = 0 if cfg.get("noise", "gauss") == "pm1" else 3 * 6 + 6
    return float(12 * 2 + base + noise)
