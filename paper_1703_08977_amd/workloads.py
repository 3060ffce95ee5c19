"""Seeded synthetic workloads: parameter values only, no arithmetic of the method.

Each workload is a plain dict read by both the HIP path (through the
binding) and the CPU oracle, so that both draw the same Philox streams.
Keys:
  trial        "expo" | "pade" | "triplet" | "pz" | "triplet_r0" | "pz_sum"
  theta        [orbital exponent, Jastrow beta, Jastrow c, second exponent a, r0]
  sym          +1 / -1 (P_z trial: singlet "+" or triplet "-" combination)
  Z, ee        nuclear charge; 1 if the potential holds +1/r12
  dt, n_steps, sample_every, n_walkers, seed
  e_ref        trial energy lambda0 (the shift of eq. (4)); it cancels in every
               energy estimate and only keeps ln w of order one
  noise        "gauss" (Euler-Maruyama) | "pm1" (the paper's +/-1 walk)
  quad         "trapezoid" | "right" (the paper's right end-point Riemann sum)
  contract     Gaussian stream contract: 1 (two Philox blocks per step,
               32-bit uniforms) or 2 (one block per step, 21-bit uniforms,
               the same in both precisions: the mixed-vs-FP64 workloads use it
               so that both precisions draw identical increments)
  precision    "fp64" | "mixed" (FP32 coordinates, drift and E_L; FP64 ln w)
  n_metropolis, metropolis_sigma, init_sigma  (start ensemble ~ |psi|^2)
  drift_limit  a >= 0: drift / integrand limiting near the singular points of
               an inexact trial function (0: the plain discretisation)
  plain        True: the plain Feynman-Kac walk of eqs. (2)-(3) (no drift,
               integrand V - e_ref) from the same start ensemble
  bridge       True: node trials weight each step by the chance that its path
               did not touch the node (Brownian bridge)

The e_ref values are variational energies of each trial function measured
with 2^16 Metropolis samples; any value works.
"""
from __future__ import annotations

import copy

# 1^1S, exp(-alpha (r1 + r2)), alpha = 27/16: 4096 walkers, dt = 0.01, T = 2.
HE_GROUND_EXPO_4K = dict(
    name="he_1s_expo_4k", trial="expo", theta=[27.0 / 16.0, 0.0, 0.0, 0.0], Z=2.0, ee=1,
    n_walkers=4096, dt=0.01, n_steps=200, sample_every=5, seed=42, e_ref=-2.84765625,
    noise="gauss", quad="trapezoid", contract=1, precision="fp64",
    n_metropolis=500, metropolis_sigma=0.5, init_sigma=1.0)

# 1^1S, Pade-Jastrow exp(-2(r1+r2)) exp(r12 / (2 (1 + beta r12))), beta = 0.25:
# 2^20 walkers, T = 5, dt in {0.002, 0.001, 0.0005}, seeds 0..15.
HE_GROUND_PADE_1M = dict(
    name="he_1s_pade_1m", trial="pade", theta=[2.0, 0.25, 0.5, 0.0], Z=2.0, ee=1,
    n_walkers=1 << 20, dt=0.002, n_steps=2500, sample_every=25, seed=0, e_ref=-2.8754,
    noise="gauss", quad="trapezoid", contract=1, precision="fp64",
    n_metropolis=500, metropolis_sigma=0.5, init_sigma=1.0,
    dts=[0.002, 0.001, 0.0005], T=5.0, seeds=list(range(16)))

# 2^3S, [e^{-2r1-a r2} - e^{-2r2-a r1}] exp(r12 / (4 (1 + beta r12))), a = 0.6,
# beta = 0.3, node r1 = r2: 2^22 walkers, dt = 0.001, T = 4.
HE_TRIPLET_4M = dict(
    name="he_2tripS_4m", trial="triplet", theta=[2.0, 0.3, 0.25, 0.6], Z=2.0, ee=1,
    n_walkers=1 << 22, dt=0.001, n_steps=4000, sample_every=50, seed=0, e_ref=-2.1222,
    noise="gauss", quad="trapezoid", contract=2, precision="mixed",
    n_metropolis=500, metropolis_sigma=0.5, init_sigma=1.0)

# Gradient of E(T = 2) with respect to (alpha, beta) of the Pade-Jastrow trial:
# 2^18 walkers, dt = 0.002, 1000 steps, a checkpoint at every step: the stored
# trajectory (14.7 GB in binary64) is the reverse sweep's tape, and nothing is recomputed.
HE_GRAD_PADE_256K = dict(
    name="he_1s_pade_grad_256k", trial="pade", theta=[2.0, 0.25, 0.5, 0.0], Z=2.0, ee=1,
    n_walkers=1 << 18, dt=0.002, n_steps=1000, sample_every=50, ckpt_every=1, seed=0,
    e_ref=-2.8754, noise="gauss", quad="trapezoid", contract=1, precision="fp64",
    n_metropolis=500, metropolis_sigma=0.5, init_sigma=1.0, gd_steps=20, gd_lr=0.05)

# 2^1P (P_z, "+" combination) z2 e^{-2r1-r2/2} + z1 e^{-2r2-r1/2} with Jastrow
# beta = 0.3 (c = 1/2): 2^24 walkers, dt = 0.0005, T = 6, 16 seeds.
HE_PZ_16M = dict(
    name="he_2P_pz_16m", trial="pz", sym=1, theta=[2.0, 0.3, 0.5, 0.5], Z=2.0, ee=1,
    n_walkers=1 << 24, dt=0.0005, n_steps=12000, sample_every=100, seed=0, e_ref=-2.1194,
    noise="gauss", quad="trapezoid", contract=2, precision="mixed",
    n_metropolis=500, metropolis_sigma=0.5, init_sigma=1.0, drift_limit=1.0, seeds=list(range(16)))

# The paper's own 2^3S runs (Tables 1 and 2): trial functions 3 and 5,
# (r0 - r1) e^{-alpha1 r1 - alpha2 r2} - (1 <-> 2), the +-1 walk with step 1/scale
# at scale 30 (dt = 1/900), right end-point Riemann sum, times t = 8..48, e_ref =
# the printed trial energy lambda0; about a million paths (2^20 walkers).
PAPER_FN3_1M = dict(
    name="he_2tripS_fn3_1m", trial="triplet_r0", theta=[1.0, 0.0, 0.0, 2.0, 1.0, 0.0], Z=2.0, ee=1,
    n_walkers=1 << 20, dt=1.0 / 900.0, n_steps=48 * 900, sample_every=900, seed=0, e_ref=-2.12412661,
    noise="pm1", quad="right", contract=1, precision="mixed",
    n_metropolis=500, metropolis_sigma=0.5, init_sigma=1.0, t_fit=[8, 16, 24, 32, 40, 48])
PAPER_FN5_1M = dict(
    PAPER_FN3_1M, name="he_2tripS_fn5_1m", theta=[0.636748, 0.0, 0.0, 2.002777, 0.73351723, 0.0],
    e_ref=-2.1742305)
# Trial function 4 (r0 = 1, alpha1 = 0.67180691, alpha2 = 2.00411836) has no table; its e_ref
# is the mean local energy of 2^18 |psi|^2 samples, -2.17315(16).
PAPER_FN4_1M = dict(
    PAPER_FN3_1M, name="he_2tripS_fn4_1m", theta=[0.67180691, 0.0, 0.0, 2.00411836, 1.0, 0.0],
    e_ref=-2.17315)

# The paper's P_z run (Table 5): trial function 7, (z1 + z2)[e^{-a1 r1 - a2 r2} + e^{-a2 r1 - a1 r2}],
# whose exponents are not printed.  Reconstruction: a1 = 2 (the He+ 1s exponent), a2 = 0.25, whose
# mean local energy over |psi|^2, -2.0645(8) from 2^17 samples, matches the printed trial energy
# lambda0 = -2.06460746 used as e_ref.  The outer electron reaches r ~ 10, so the start ensemble takes
# 2000 Metropolis steps of box width 1.
PAPER_FN7_1M = dict(
    PAPER_FN3_1M, name="he_2P_fn7_1m", trial="pz_sum", theta=[2.0, 0.0, 0.0, 0.25, 0.0, 0.0],
    e_ref=-2.06460746, n_metropolis=2000, metropolis_sigma=1.0)

WORKLOADS = {w["name"]: w for w in
             (HE_GROUND_EXPO_4K, HE_GROUND_PADE_1M, HE_TRIPLET_4M, HE_GRAD_PADE_256K, HE_PZ_16M,
              PAPER_FN3_1M, PAPER_FN4_1M, PAPER_FN5_1M, PAPER_FN7_1M)}

# Closed-form systems.
# Z = 2 without 1/r12 and the exact product of hydrogenic 1s orbitals: E_L = -4 exactly.
EXACT_NOEE = dict(
    name="exact_noee", trial="expo", theta=[2.0, 0.0, 0.0, 0.0], Z=2.0, ee=0,
    n_walkers=4096, dt=0.01, n_steps=200, sample_every=10, seed=1, e_ref=-4.0,
    noise="gauss", quad="trapezoid", contract=1, precision="fp64",
    n_metropolis=100, metropolis_sigma=0.5, init_sigma=1.0)

# Two independent hydrogen atoms (Z = 1, no 1/r12), alpha = 1: E_L = -1 (-1/2 per electron).
HYDROGEN = dict(EXACT_NOEE, name="hydrogen", theta=[1.0, 0.0, 0.0, 0.0], Z=1.0, e_ref=-1.0)

# Z = 2 without 1/r12, the exact 1s2s triplet 2s(1) 1s(2) - 1s(1) 2s(2) with 2s = (1 - r) e^{-r},
# 1s = e^{-2r}: the (r0 - r) prefactor trial at (A, a, r0) = (1, 2, 1), no Jastrow.
# E_L = -Z^2/2 - Z^2/8 = -5/2 exactly; the node r1 = r2 is exact.
EXACT_TRIPLET_NOEE = dict(
    EXACT_NOEE, name="exact_triplet_noee", trial="triplet_r0", theta=[1.0, 0.0, 0.0, 2.0, 1.0, 0.0],
    e_ref=-2.5, contract=2)

CLOSED_FORM = {w["name"]: w for w in (EXACT_NOEE, HYDROGEN, EXACT_TRIPLET_NOEE)}


def get(name: str, **overrides) -> dict:
    """A deep copy of a named workload with keys overridden."""
    src = WORKLOADS.get(name) or CLOSED_FORM[name]
    w = copy.deepcopy(src)
    w.update(overrides)
    return w
