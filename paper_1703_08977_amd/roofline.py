"""Algorithmic VALU work of one walker step and the MI355X VALU issue peak.

The step is per-walker scalar arithmetic (transcendental, integer and
floating point; no contraction, no HBM traffic between sampling times), so
its roofline is the vector-ALU issue rate.

Peak: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 39.32e12 lane-operations/s,
one main-pipe VALU instruction slot per lane per clock (a wave64 instruction
occupies a 16-lane SIMD for 4 clocks).  This is the published 78.6 TFLOP/s
binary32 (and binary64) FMA rate divided by 2 flops; the 157.3 TFLOP/s
binary32 figure needs packed (v_pk_*) instructions, which this library does
not use.

Work: every elementary operation of the step's formulas counts one main-pipe
slot -- add, mul, fma, compare, select, convert, 32-bit integer op,
32x32->64 multiply, three-input xor.  The binary32 hardware transcendentals
(v_sqrt, v_rsq, v_rcp, v_exp, v_log, v_sin, v_cos) are counted apart: they
issue beside the main pipe.  The counters show it: the mixed P_z step's 205
VALU instructions per wave-step (20 of them transcendental) issue at 0.262
wave-instructions per SIMD-cycle at 2.38 GHz, above the 0.25 that one 4-cycle
slot per instruction would allow, so the roofline is the main pipe's.
Binary64 functions count their polynomial and range-reduction operations (the
table F64 below), a binary64 select as two 32-bit selects.  Counts follow the
formulas term by term (they are not read back from the compiled code).
"""
from __future__ import annotations

PEAK_SLOTS_PER_S = 256 * 4 * 16 * 2.4e9  # 39.32e12

NODE_TRIALS = ("triplet", "triplet_r0", "pz", "pz_sum")

# Philox4x32-10 block per step: 10 rounds x (two 32x32->64 multiplies, two three-input
# xors), less the work fixed per walker or uniform over the wave: round 1 multiplies the
# block index (the step, a scalar) and the walker id (fixed), so it needs only the xor
# that joins them; round 2's product of the fixed word is fixed too.  The key schedule
# runs on the scalar unit.
PHILOX_BLOCK = 10 * (2 + 2) - 3 - 1

# (elementary operations, hardware transcendental instructions) per function
# "dist": r and 1/r from a squared distance q -- binary32 one reciprocal square root and the
# product q (1/r); binary64 a square root and a reciprocal.  "expm1" (arguments <= 0):
# binary32 the series to x^7 beside e^x - 1 and a select, binary64 the reduced series.
F32 = {"sqrt": (0, 1), "rcp": (0, 1), "dist": (1, 1), "exp": (1, 1), "expm1": (11, 1), "log": (1, 1),
       "sincos": (0, 2)}
# binary64 (hefk_f64math.hpp, counted from the code, a binary64 select as two 32-bit selects):
# sqrt  = seed, coupled iteration, correction (8); rcp = seed + two Newton steps (5);
# dist  = seed, the coupled iteration of sqrt, one Newton step on 1/r (11);
# exp   = reduction (4), the degree-11 polynomial (11), 2^k and the underflow guard (5): 20;
# expm1 = reduction (4), the degree-10 polynomial Q (10), r + r^2 Q (2), 2^k, 2^k - 1, guard and
#         fused sum (7): 23;
# log   = exponent and mantissa fields (3), halving above sqrt 2 (5), s = (m - 1)/(m + 1) (8), z (1),
#         the degree-6 polynomial R (6), 2 s (1 + z R) (3), the exponent's two-part ln 2 (3),
#         times -2 dt (1): 31;
# sincos = quadrant reduction (4), y^2 (1), sin(pi y) = y S(y^2) (7), cos(pi y) = C(y^2) (7), the
#         quadrant's exchange (5) and its sign bits (7): 31
F64 = {"sqrt": (8, 0), "rcp": (5, 0), "dist": (11, 0), "exp": (20, 0), "expm1": (23, 0), "log": (31, 0),
       "sincos": (31, 0)}


class _Count:
    def __init__(self):
        self.main = 0.0
        self.trans = 0.0

    def ops(self, n):
        self.main += n

    def fn(self, table, name, times=1):
        m, t = table[name]
        self.main += m * times
        self.trans += t * times


def _noise(c: _Count, f, noise: str, contract: int):
    if noise == "pm1":
        c.ops(PHILOX_BLOCK / 20.0 + 6 * 2)  # one block per 20 steps; bit extract + select per coordinate
        return
    # Box-Muller per pair: the radius sqrt(dt) sqrt(-2 ln u1) as the square root of a scaled
    # logarithm, sin and cos of 2 pi u2; the radius-times-cosine products are the
    # multiplies of the Euler step's fused multiply-adds
    for _ in range(3):
        c.fn(f, "log")
        c.fn(f, "sqrt")
        c.fn(f, "sincos")
    if contract == 2:
        # one block; the six 21-bit fields: four masks, and a shift, a shift and a
        # shift-and-or for each of the two joined fields; convert + scale each
        c.ops(PHILOX_BLOCK + 4 + 2 * 3 + 6 * 2)
    else:
        c.ops(2 * PHILOX_BLOCK + 6 * 2)  # two blocks; funnel shift + add (binary32), convert + scale (binary64)


def _trial(c: _Count, f, trial: str):
    # geometry: D = R1 - R2 (3), three squared norms (3 x 3), the distance and its reciprocal
    # from each, the projections R1.D and R2.D (2 x 3)
    c.ops(3 + 3 * 3 + 2 * 3)
    c.fn(f, "dist", 3)
    drift = 3 * 3  # b1 = a1 R1 + w D, b2 = a2 R2 - w D: w D once per component, a fused multiply-add per coordinate
    if trial == "expo":
        # a_i = -A / r_i (2), b = a_i R_i (6), E_L = -A^2 + (A - Z)(1/r1 + 1/r2) + ee/r12 (3)
        c.ops(2 + 6 + 3)
        return
    # Jastrow: s = 1 + beta r12 and its reciprocal, 1/s^2, u', and the radial part of the local
    # energy's Jastrow terms [2 c beta (1/s + 2 + beta r12) - c^2 / s^2] / s^2 (5) plus the cusp
    # remainder (ee - 2c)/r12 (product, select, sum: 3)
    c.ops(1 + 1 + 1 + 5 + 3)
    c.fn(f, "rcp")
    if trial == "pade":
        # a_i (2), w = u'/r12 (1), drift, cosine difference (3),
        # E_L = -A^2 + (A - Z)(1/r1 + 1/r2) + A u' cos + the Jastrow radial part (5)
        c.ops(2 + 1 + drift + 3 + 5)
        return
    # d = (A - a)(r1 - r2) (2), its sign (1), the pair (t1, t2) (2 selects); the argument -|d| is
    # an operand modifier in binary32 and a select in binary64, where a select takes two slots
    c.ops(2 + 1 + 2 if f is F32 else 2 + 1 + 4 + 2)
    if trial == "triplet":
        c.fn(f, "expm1")
        c.fn(f, "rcp")
        # e = 1 + em, D (2), g1, g2 (2 x 3), the sum of the two Laplacian ratios (two brackets of
        # two fused multiply-adds, t1 and t2 times them, 1/D: 7), g_i / r_i (2), w (1), drift,
        # cross term (5), E_L (5)
        c.ops(1 + 2 + 6 + 7 + 2 + 1 + drift + 5 + 5)
        return
    c.fn(f, "exp")
    c.fn(f, "rcp")
    if trial == "triplet_r0":
        # q_i = r0 - r_i, u_i = 1 + A q_i (4), D (2), g1, g2 (2 x 4), the sum of the two Laplacian
        # ratios (two brackets of five operations, t1 and t2 times them, 1/D: 13), g_i / r_i (2),
        # w (1), drift, cross term (5), E_L (5)
        c.ops(4 + 2 + 8 + 13 + 2 + 1 + drift + 5 + 5)
        return
    if trial == "pz_sum":
        c.fn(f, "rcp")  # 1 / (z1 + z2)
        # t1 + t2 (1), z1 + z2 (1), g1, g2 (2 x 3), a_i (2), w (1), drift, z terms (2), the sum of
        # the two Laplacian ratios (brackets 4, t1 and t2 times them 2, 1/S 1, the node-gradient
        # term 2 iZ (a1 z1 + a2 z2) 4: 11), cross term (3), E_L (5)
        c.ops(1 + 1 + 6 + 2 + 1 + drift + 2 + 11 + 3 + 5)
        return
    # P_z: sym t2 (1), P (2), k1, k2 (2 x 4), a1, a2 (2 x 2), s1, s2 (2), w (1), drift, z terms (2),
    # the sum of the two Laplacian ratios (two brackets of two fused multiply-adds, the products
    # z2 t1 and t2 z1 and their combination with the brackets, 1/P: 9), cross term (5), E_L (5)
    c.ops(1 + 2 + 8 + 4 + 2 + 1 + drift + 2 + 9 + 5 + 5)


def count(cfg: dict) -> _Count:
    prec = cfg.get("precision", "fp64")
    f = F32 if prec == "mixed" else F64
    c = _Count()
    _noise(c, f, cfg.get("noise", "gauss"), int(cfg.get("contract", 1)))
    _trial(c, f, cfg["trial"])
    c.ops(12)  # Euler step: Y + (dt f) b, then + r u, one fused multiply-add each per coordinate
    if cfg.get("drift_limit", 0.0) > 0:
        # |b|^2, 2 a dt |b|^2, 1 + ., 1 + sqrt, 2 / ., the drift's step factor dt f (the
        # limited drift f b enters the next Euler step as (dt f) b), scale e (conversion + product)
        c.ops(6 + 1 + 1 + 1 + 1 + 1 + 2)
        c.fn(f, "sqrt")
        c.fn(f, "rcp")
    c.ops(1)  # the absorbed-walker test
    if cfg["trial"] in NODE_TRIALS:
        # product of the orbital factor with the old sign and its test, the new sign
        # (copysign), ln w = -inf on a crossing (two 32-bit selects)
        c.ops(2 + 1 + 2)
    c.ops(5)  # ln w update in binary64: conversion, shift by e_ref, quadrature (2), NaN guard
    return c


def slots_per_walker_step(cfg: dict) -> float:
    """Main-pipe VALU issue slots of one walker step (the elementary operations; the hardware
    transcendentals issue beside them and are counted by transcendentals_per_walker_step)."""
    return float(count(cfg).main)


def instructions_per_walker_step(cfg: dict) -> float:
    """VALU instructions of one walker step, transcendentals included (what SQ_INSTS_VALU counts)."""
    c = count(cfg)
    return float(c.main + c.trans)


def transcendentals_per_walker_step(cfg: dict) -> float:
    """binary32 hardware transcendental instructions of one walker step (included in the slots)."""
    return float(count(cfg).trans)


# binary32 floating-point operations of the step, term by term from the formulas the step
# evaluates (the kernels' per-walker code).  Convention: add, sub, mul, div 1; fused
# multiply-add 2; each hardware transcendental (sqrt, rsq, rcp, exp2, log2, sin, cos) 1;
# negation, absolute value, copysign, compares, selects and conversions 0; products of
# trial parameters alone are uniform over the launch and do not count, nor does a parameter
# times the member of the pair (t1, t2) = (1, e^{-|d|}) or (e^{-|d|}, 1) that is exactly 1
# (counted at a point with r1 < r2).  Binary64 work (ln w) is not included.
FP32_NOISE = {
    # per pair: the two uniforms, log2 u1, its product with the radius scale, sqrt, sin, cos
    "c2": 6 * 2 + 3 * (1 + 1 + 1 + 2),  # 21-bit fields: (f + 1/2) 2^-21 as one fused multiply-add each
    "c1": 6 * 1 + 3 * (1 + 1 + 1 + 2),  # 23-bit fields: the float 1.m minus (1 - 2^-24)
    "pm1": 0,                           # +-1 by selects; sqrt(dt) is a constant
}
FP32_EULER = 6 * 2 * 2  # Y + (dt f) b, then + r u: two fused multiply-adds per coordinate
# D = R1 - R2 (3); per distance the squared norm (3 mul, 2 add), v_rsq and r = q (1/r) (7 each, 21);
# the projections R1.D and R2.D (5 each)
FP32_GEOMETRY = 3 + 3 * 7 + 2 * 5
FP32_LIMITER = 12 + 6 + 1  # |b|^2 (6 mul, 6 add); f = 2 rcp(1 + sqrt(1 + 2 a dt |b|^2)) (6); dt f (1)
FP32_NODE_TEST = 1         # the product of the orbital factor with the carried sign


def _fp32_jastrow(cusp_zero: bool) -> int:
    # 1/s = rcp(1 + beta r12) (3), 1/s^2 (1), u' = c/s^2 (1); the radial part
    # [2 c beta ((1/s + 2) + beta r12) - c^2 / s^2] / s^2 (8: three for the inner sum, its product,
    # c^2 times 1/s^2, the difference, times 1/s^2, and the sum with the cusp term), whose cusp
    # term (ee - 2c)/r12 adds a product when ee != 2c
    return 3 + 1 + 1 + 8 + (0 if cusp_zero else 1)


def _fp32_trial(trial: str) -> int:
    drift = 3 + 6 * 2  # w D once per component (3), then a fused multiply-add per coordinate
    if trial == "expo":
        # a_i = -A / r_i (2), drift with w = 0 (15), E_L = -A^2 + (A - Z)(1/r1 + 1/r2) + ee/r12 (5)
        return 2 + drift + 5
    if trial == "pade":
        # a_i (2), w = u'/r12 (1), drift, (h1 - h2).h12 (4), E_L (7)
        return 2 + 1 + drift + 4 + 7
    # the pair: d = (A - a)(r1 - r2) (2)
    if trial == "triplet":
        # e^{-|d|} - 1 by the series to x^7 beside e^x - 1 (five fused multiply-adds 10, x^2 and the
        # last one 3, e^x - 1 as a product, v_exp and a subtraction 3: 16), e = 1 + em (1), 1/D (1),
        # g1, g2 (3 each), the two Laplacian brackets (4 each) times t1, t2 (1 each), their
        # difference and 1/D (2), g_i/r_i and u'/r12 (3), drift, cross term (6), E_L (7)
        return 2 + 16 + 1 + 1 + 6 + (4 + 1) * 2 + 2 + 3 + drift + 6 + 7
    if trial == "triplet_r0":
        # e^{-|d|} (2), q_i = r0 - r_i (2), D (3), 1/D (1), u_i = 1 + A q_i (4), g1, g2 (5 each), the
        # two Laplacian brackets (10 each) times t1, t2 (1 each), their difference and 1/D (2),
        # g_i/r_i and u'/r12 (3), drift, cross term (6), E_L (7)
        return 2 + 2 + 2 + 3 + 1 + 4 + 10 + (10 + 1) * 2 + 2 + 3 + drift + 6 + 7
    if trial == "pz_sum":
        # e^{-|d|} (2), 1/(t1 + t2) (2), z1 + z2 and its reciprocal (2), g1, g2 (3 each), a_i = g_i/r_i
        # (2), u'/r12 (1), drift, the z terms of the drift (2), the two Laplacian brackets (4 each)
        # times t1, t2 (1 each), their sum and 1/S (2), the node-gradient term 2/Zs (a1 z1 + a2 z2)
        # and its sum (6), cross term (4), E_L (7)
        return 2 + 2 + 2 + 2 + 6 + 2 + 1 + drift + 2 + (4 + 1) * 2 + 2 + 6 + 4 + 7
    # P_z: e^{-|d|} (2), sym t2 (1), P (3), 1/P (1), k1, k2 (5 each), a_i (2 each), s_i = t/P (2),
    # u'/r12 (1), drift, the z terms of the drift (2), the two Laplacian brackets (4 each) times
    # z2 t1 and t2 z1 (2 each), their sum and 1/P (2), cross term (7), E_L (7)
    return 2 + 2 + 1 + 3 + 1 + 10 + 4 + 2 + 1 + drift + 2 + (4 + 2) * 2 + 2 + 7 + 7


def fp32_flops_per_walker_step(cfg: dict) -> float:
    """binary32 floating-point operations of one mixed step (the convention above)."""
    if cfg.get("precision", "fp64") != "mixed":
        return 0.0
    trial = cfg["trial"]
    noise = "pm1" if cfg.get("noise", "gauss") == "pm1" else ("c2" if int(cfg.get("contract", 1)) == 2 else "c1")
    n = FP32_NOISE[noise] + FP32_EULER + FP32_GEOMETRY + _fp32_trial(trial)
    if trial != "expo":
        n += _fp32_jastrow(float(cfg.get("ee", 1)) == 2.0 * float(cfg["theta"][2]))
    if trial in NODE_TRIALS:
        n += FP32_NODE_TEST
    if cfg.get("drift_limit", 0.0) > 0:
        n += FP32_LIMITER
    return float(n)


def _vjp(c: _Count, f, trial: str):
    """One reverse step of the pathwise gradient (binary64): the vector-Jacobian product of
    F = V . b(Y) + A e(Y) through the trial evaluation, and the sweep's own updates."""
    # geometry again: D (3), squared norms (9), distance and reciprocal of each, unit vectors (9)
    c.ops(3 + 9 + 9)
    c.fn(f, "dist", 3)
    if trial == "pade":
        c.ops(1 + 2)  # s = 1 + beta r12, u' = c / s^2
        c.fn(f, "rcp")
    # w = (h1 - h2).h12 (6), V.h (6), (V1 - V2).h12 (6)
    c.ops(6 + 6 + 6)
    # adjoints of the unit vectors: A alpha u' (2), bh1 and bh2 (2 x 3 x 2), bh12 (3 x 4)
    c.ops(2 + 12 + 12)
    # adjoints of 1/r1 = 1/r2 and 1/r12, d/d alpha (9)
    c.ops(2 + 2 + 5)
    if trial == "pade":
        # d/du', d/d(1/s), d/d beta, d/ds, its share of d/dr12 (17)
        c.ops(5 + 5 + 3 + 2 + 2)
    # back through r = |R|, h = R/r: three projections (9), their sums (3), d/dr (6), grad Y (3 x 7)
    c.ops(9 + 3 + 6 + 21)
    # sweep: V = dt lambda (6), lambda += grad (6), theta-bar (2), the step's weight A (2), P += H (1)
    c.ops(6 + 6 + 2 + 2 + 1)


def grad_tape_bytes_per_walker_step(cfg: dict) -> float:
    """HBM traffic of the reverse sweep per walker-step.  Recomputing segments: the recomputed
    position (6 binary64 coordinates) written to the segment tape once and read back once, and
    ln w likewise at the sampling steps.  Over the stored trajectory (a checkpoint at every
    step): the position read once, and ln w at the sampling steps."""
    se = max(1, int(cfg.get("sample_every", 1)))
    if int(cfg.get("ckpt_every", 50)) == 1:
        return 6 * 8 + 8.0 / se
    return 2.0 * 6 * 8 + 2.0 * 8 / se


def grad_slots_per_walker_step(cfg: dict) -> float:
    """VALU issue slots of the gradient kernel per walker-step: the reverse step, and when the
    sweep recomputes segments, the recomputed forward step (plus the segment's start
    evaluation, once per checkpoint interval)."""
    v = _Count()
    _vjp(v, F64, cfg["trial"])
    ce = max(1, int(cfg.get("ckpt_every", 50)))
    if ce == 1:
        return float(v.main + v.trans)
    fwd = count(dict(cfg, precision="fp64"))
    c = _Count()
    _trial(c, F64, cfg["trial"])
    return float(fwd.main + fwd.trans + (c.main + c.trans) / ce + v.main + v.trans)
