"""Algorithmic VALU work of one walker step and the MI355X VALU issue peak.

The step is scalar transcendental and integer work per walker (no
contraction, no HBM traffic between sampling times), so its roofline is the
vector ALU issue rate.  Peak: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz =
39.32e12 lane-operations per second at one full-rate operation per lane per
clock (wave64 issues over 4 clocks on a 16-lane SIMD).  Operations count in
issue slots:
  full rate (1 slot):     binary32 add / mul / fma / compare / select / convert,
                          binary64 add / mul / fma (full rate on MI355X:
                          78.6 TFLOP/s binary64 = 39.3e12 fma/s), 32-bit integer
                          add / xor / shift / and;
  quarter rate (4 slots): binary32 transcendentals (v_sqrt, v_rcp, v_exp, v_log,
                          v_sin, v_cos), binary64 reciprocal / rsqrt seeds,
                          32x32 -> 64-bit integer multiply (v_mad_u64_u32).
Binary64 library functions are counted at the operation counts of their
usual polynomial evaluations (log 28, exp 22, expm1 26, sincospi 36,
correctly rounded sqrt 11 incl. a quarter-rate seed, division 12 incl. seed).
The counts follow the formulas of the step (they are not read back from the
compiled code); the design doc lists them term by term.
"""
from __future__ import annotations

PEAK_SLOTS_PER_S = 256 * 4 * 16 * 2.4e9  # 39.32e12

# Philox4x32-10 block: 10 rounds x (2 wide multiplies (4 slots) + 2 three-input xors)
PHILOX_BLOCK = 10 * (2 * 4 + 2)

_F32 = {"sqrt": 4, "rcp": 4, "exp": 4 + 1, "log": 4 + 1, "sincos": 8, "expm1": 14}
_F64 = {"sqrt": 11, "rcp": 12, "exp": 22, "log": 28, "sincos": 36, "expm1": 26}


def _noise(precision, noise, contract):
    f = _F32 if precision == "mixed" else _F64
    if noise == "pm1":
        # one block per 20 steps; 6 bit extracts + selects
        return PHILOX_BLOCK / 20.0 + 6 * 2
    blocks = 2 if contract == 1 else 1
    unif = 6 * 3  # field extract, convert, scale
    bm = 3 * (f["log"] + 1 + f["sqrt"] + f["sincos"] + 2)
    return blocks * PHILOX_BLOCK + unif + bm


def _trial(precision, trial):
    f = _F32 if precision == "mixed" else _F64
    geo = 3 * 3 + 3 + 3 * f["sqrt"] + 3 * f["rcp"] + 9  # squared norms, differences, roots, inverses, unit vectors
    if trial == "expo":
        return geo + 6 + 4
    jas = f["rcp"] + 1 + 1 + 1 + 2 + 5
    if trial == "pade":
        return geo + jas + 12 + 6 + 8
    swap = 6 + 3 + 12  # squared radii compare, electron swap in and drift swap out
    if trial == "triplet":
        return geo + jas + swap + f["expm1"] + 2 + f["rcp"] + 6 + 12 + 12 + 6 + 10 + 2
    # pz
    return geo + jas + swap + f["exp"] + 2 + 2 + f["rcp"] + 4 + 14 + 16 + 12 + 6 + 10 + 3


def slots_per_walker_step(cfg: dict) -> float:
    """Issue slots of one walker step (noise, Euler step, trial evaluation, node test, ln w)."""
    prec = cfg.get("precision", "fp64")
    n = _noise(prec, cfg.get("noise", "gauss"), int(cfg.get("contract", 1)))
    t = _trial(prec, cfg["trial"])
    euler = 12
    lnw = 8 if prec == "mixed" else 5  # two conversions in the mixed path, the quadrature, NaN guard
    state = 14  # absorbed-walker freeze (selects on the state)
    return float(n + t + euler + lnw + state)


def fp32_flops_per_walker_step(cfg: dict) -> float:
    """Binary32 floating-point operations of one mixed-precision step (fma = 2, transcendental = 1)."""
    if cfg.get("precision", "fp64") != "mixed":
        return 0.0
    # Euler (6 fma), geometry and trial arithmetic, Box-Muller: counted from the formulas
    base = {"expo": 60, "pade": 95, "triplet": 135, "pz": 150}[cfg["trial"]]
    noise = 0 if cfg.get("noise", "gauss") == "pm1" else 3 * (1 + 1 + 2 + 2) + 6 * 2
    return float(12 + base + noise)
