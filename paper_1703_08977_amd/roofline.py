"""Algorithmic VALU work of one walker step and the MI355X VALU issue peak.

The step is per-walker scalar arithmetic (transcendental, integer and
floating point; no contraction, no HBM traffic between sampling times), so
its roofline is the vector-ALU issue rate.

Peak: the published binary32 vector rate, 157.3 TFLOP/s = 256 CUs x 4 SIMDs x
32 lanes x 2.4 GHz fused multiply-adds: 78.64e12 issue slots per second, one
slot being one lane of one binary32 add, multiply or fused multiply-add.  On
this GPU that rate needs no packed instructions: a wave64 binary32 or 32-bit
integer instruction with vector operands issues every 2.1-2.2 SIMD-cycles
(`valu_rates`, profiles/valu_class_costs.txt), and this library uses no
packed (v_pk_*) arithmetic.

Work: the step's formulas, counted term by term (not read back from the
compiled code), in classes of instruction; each class costs its issue time
measured by `valu_rates` on the MI355X (SIMD-cycles per wave64 instruction,
the lower of the class alone and beside binary32 multiply-adds), in slots of
2 SIMD-cycles:

  a32    binary32 add, mul, fma, compare, min/max; 32-bit integer add, logic,
         shift, bit-field ops (three-input xor included)      2.0   -> 1
  sel    32-bit select (a binary64 select is two)              2.28  -> 1.14
  cvt    32-bit integer -> binary32 conversion                 2.46  -> 1.23
  cvt64  conversion to or from binary64                        3.55  -> 1.77
  mad    32 x 32 -> 64-bit integer multiply (Philox)           4.12  -> 2.06
  f64    binary64 add, mul, fma, compare, ldexp, rounding      4.17  -> 2.08
  trans  binary32 hardware transcendental (sqrt, rsq, rcp,
         exp2, log2, sin, cos)                                 8.24  -> 4.12
  seed   binary64 reciprocal or reciprocal square root seed   16.07  -> 8.04

(The a32 cost is the published rate's 2 cycles; binary32 add and multiply
measured 2.15-2.17, the 32-bit xor 2.26, the multiply-add 2.16-2.8 by operand
layout.  Select, conversion and 32x32->64 multiply cost 4.1, 5.5 and 5.8
cycles alone and the lower figures above beside multiply-adds.)  A
transcendental does not issue beside the multiply-adds: with one beside each
multiply-add the pair costs the sum of the two.
"""
from __future__ import annotations

from collections import Counter

PEAK_SLOTS_PER_S = 256 * 4 * 32 * 2.4e9  # 78.64e12: the 157.3 TFLOP/s binary32 rate in fused multiply-adds

# slots (2 SIMD-cycles) per wave64 instruction of each class, from the measured issue costs above
CLASS_SLOTS = {"a32": 1.0, "sel": 1.14, "cvt": 1.23, "cvt64": 1.77, "mad": 2.06, "f64": 2.08, "trans": 4.12,
               "seed": 8.04}

NODE_TRIALS = ("triplet", "triplet_r0", "pz", "pz_sum")

# Philox4x32-10 block per step: 10 rounds x (two 32x32->64 multiplies, two three-input
# xors), less the work fixed per walker or uniform over the wave: round 1 multiplies the
# block index (the step, a scalar) and the walker id (fixed), so it needs only the xor
# that joins them; round 2's product of the fixed word is fixed too.  The key schedule
# runs on the scalar unit.
PHILOX_BLOCK = {"mad": 10 * 2 - 2 - 1, "a32": 10 * 2 - 1}  # 17 + 19

# instruction classes per function
# binary32: "dist" (r and 1/r from a squared distance q) is one reciprocal square root and the
# product q (1/r); "expm1" (arguments <= 0) the series to x^7 beside e^x - 1 and a select.
F32 = {"sqrt": {"trans": 1}, "rcp": {"trans": 1}, "dist": {"a32": 1, "trans": 1}, "exp": {"a32": 1, "trans": 1},
       "expm1": {"a32": 10, "sel": 1, "trans": 1}, "log": {"a32": 1, "trans": 1}, "sincos": {"trans": 2}}
# binary64 (hefk_f64math.hpp, counted from the code, a binary64 select as two 32-bit selects):
# sqrt  = seed, coupled iteration and correction (7);
# rcp   = seed, two Newton steps (4);
# dist  = seed, the coupled iteration of sqrt, one Newton step on 1/r (10);
# exp   = reduction (4), the degree-11 polynomial (11), 2^k (a conversion and ldexp) and the
#         underflow guard (a compare, a select: 2 + 2);
# expm1 = reduction (4), the degree-10 polynomial Q (10), r + r^2 Q (2), 2^k (conversion, ldexp),
#         2^k - 1, the guard (compare, select) and the fused sum;
# log   = exponent and mantissa fields (3 integer), halving above sqrt 2 (compare, product, the
#         mantissa's select, the exponent's increment: 5), s = (m - 1)/(m + 1) (two sums, a
#         reciprocal, a product: 8), z (1), the degree-6 polynomial R (6), 2 s (1 + z R) (3), the
#         exponent's conversion and two-part ln 2 (3), times -2 dt (1);
# sincos = quadrant reduction (4), y^2 (1), sin(pi y) = y S(y^2) (7), cos(pi y) = C(y^2) (7), the
#         quadrant index and the exchange of sine and cosine (conversion, two selects: 5) and the
#         sign bits (7)
F64 = {"sqrt": {"seed": 1, "f64": 7}, "rcp": {"seed": 1, "f64": 4}, "dist": {"seed": 1, "f64": 10},
       "exp": {"f64": 4 + 11 + 1 + 1, "cvt64": 1, "sel": 2},
       "expm1": {"f64": 4 + 10 + 2 + 1 + 1 + 1 + 1, "cvt64": 1, "sel": 2},
       "log": {"a32": 3 + 1, "f64": 2 + 2 + 4 + 1 + 1 + 6 + 3 + 2 + 1, "sel": 2, "seed": 1, "cvt64": 1},
       "sincos": {"f64": 4 + 1 + 7 + 7, "cvt64": 1, "sel": 4, "a32": 7}}


class _Count:
    """Instruction counts of one walker step by class; `arith` is the class of the step's own
    floating-point arithmetic (a32 in binary32, f64 in binary64)."""

    def __init__(self, arith: str = "a32"):
        self.n = Counter()
        self.arith = arith

    def add(self, cls: str, k: float):
        self.n[cls] += k

    def ops(self, k: float):
        self.n[self.arith] += k

    def fn(self, table, name, times=1):
        for cls, k in table[name].items():
            self.n[cls] += k * times

    def philox(self, blocks: float):
        for cls, k in PHILOX_BLOCK.items():
            self.n[cls] += k * blocks

    @property
    def instructions(self) -> float:
        return float(sum(self.n.values()))

    @property
    def slots(self) -> float:
        return float(sum(k * CLASS_SLOTS[c] for c, k in self.n.items()))


def _noise(c: _Count, f, noise: str, contract: int):
    if noise == "pm1":
        c.philox(1 / 20.0)  # one block per 20 steps
        c.add("a32", 6)     # the bit of each coordinate
        c.add("sel", 6)     # +-1 by a select
        return
    # Box-Muller per pair: the radius sqrt(dt) sqrt(-2 ln u1) as the square root of a scaled
    # logarithm, sin and cos of 2 pi u2; the radius-times-cosine products are the
    # multiplies of the Euler step's fused multiply-adds
    for _ in range(3):
        c.fn(f, "log")
        c.fn(f, "sqrt")
        c.fn(f, "sincos")
    # each of the six uniforms: convert its integer field, then scale (binary32: one fused
    # multiply-add with the half-unit offset; binary64: a product)
    cvt = "cvt" if f is F32 else "cvt64"
    if contract == 2:
        # one block; the six 21-bit fields: four masks, and a shift, a shift and a
        # shift-and-or for each of the two joined fields
        c.philox(1)
        c.add("a32", 4 + 2 * 3)
        c.add(cvt, 6)
        c.ops(6)
    elif f is F32:
        c.philox(2)        # two blocks; each 23-bit field to [1, 2) by a funnel shift, then the offset
        c.add("a32", 12)
    else:
        c.philox(2)
        c.add(cvt, 6)
        c.ops(6)


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
    # remainder (ee - 2c)/r12 (product, select, sum: 3; a binary64 select is two)
    c.ops(1 + 1 + 1 + 5 + 2)
    c.add("sel", 1 if f is F32 else 2)
    c.fn(f, "rcp")
    if trial == "pade":
        # a_i (2), w = u'/r12 (1), drift, cosine difference (3),
        # E_L = -A^2 + (A - Z)(1/r1 + 1/r2) + A u' cos + the Jastrow radial part (5)
        c.ops(2 + 1 + drift + 3 + 5)
        return
    # d = (A - a)(r1 - r2) (2), its sign (1), the pair (t1, t2) (2 selects); the argument -|d| is
    # an operand modifier in binary32 and a select in binary64, where a select is two
    c.ops(2 + 1)
    c.add("sel", 2 if f is F32 else 4 + 2)
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
    c = _Count("a32" if f is F32 else "f64")
    _noise(c, f, cfg.get("noise", "gauss"), int(cfg.get("contract", 1)))
    _trial(c, f, cfg["trial"])
    c.ops(12)  # Euler step: Y + (dt f) b, then + r u, one fused multiply-add each per coordinate
    if cfg.get("drift_limit", 0.0) > 0:
        # |b|^2, 2 a dt |b|^2, 1 + ., 1 + sqrt, 2 / ., the drift's step factor dt f (the
        # limited drift f b enters the next Euler step as (dt f) b), scale e (conversion to
        # binary64 + binary64 product)
        c.ops(6 + 1 + 1 + 1 + 1 + 1)
        c.add("cvt64" if f is F32 else "f64", 1)
        c.add("f64", 1)
        c.fn(f, "sqrt")
        c.fn(f, "rcp")
    c.add("f64", 1)  # the absorbed-walker test (ln w, binary64)
    if cfg["trial"] in NODE_TRIALS:
        # product of the orbital factor with the old sign and its test, the new sign
        # (copysign, a 32-bit bit-field insert), ln w = -inf on a crossing (two 32-bit selects)
        c.ops(2)
        c.add("a32", 1)
        c.add("sel", 2)
    # ln w update in binary64: conversion of the local energy (a binary64 step's is a binary64
    # operation), shift by e_ref, quadrature (2), NaN guard (select)
    c.add("cvt64" if f is F32 else "f64", 1)
    c.add("f64", 3)
    c.add("sel", 1)
    return c


def slots_per_walker_step(cfg: dict) -> float:
    """Issue slots of one walker step: every class's instructions at its measured cost
    (CLASS_SLOTS), against PEAK_SLOTS_PER_S."""
    return count(cfg).slots


def instructions_per_walker_step(cfg: dict) -> float:
    """VALU instructions of one walker step (what SQ_INSTS_VALU counts per lane)."""
    return count(cfg).instructions


def transcendentals_per_walker_step(cfg: dict) -> float:
    """binary32 hardware transcendental instructions of one walker step (included in the slots)."""
    return float(count(cfg).n["trans"])


def class_counts(cfg: dict) -> dict:
    """Instructions of one walker step by class."""
    return {k: float(v) for k, v in sorted(count(cfg).n.items())}


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
    v = _Count("f64")
    _vjp(v, F64, cfg["trial"])
    ce = max(1, int(cfg.get("ckpt_every", 50)))
    if ce == 1:
        return v.slots
    fwd = count(dict(cfg, precision="fp64"))
    c = _Count("f64")
    _trial(c, F64, cfg["trial"])
    return fwd.slots + c.slots / ce + v.slots


def grad_instructions_per_walker_step(cfg: dict) -> float:
    """VALU instructions of the reverse step per walker-step (the sweep over the stored
    trajectory)."""
    v = _Count("f64")
    _vjp(v, F64, cfg["trial"])
    return v.instructions
