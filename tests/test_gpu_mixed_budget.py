"""The mixed-precision step (binary32 coordinates, drift and local energy; binary64
ln w and reductions) held to its stated energy tolerance.

The per-walker parity of the binary64 path is 1e-12; binary32 paths are not
per-walker comparable over thousands of steps, so the claim for the mixed step is
one on the energy: the eq. (4) estimators of a mixed run differ from those of the
binary64 oracle on the same walker ids and the same Philox streams (contract 2
gives both precisions the same uniforms, and both start from the same binary64
start ensemble) by at most MIXED_BUDGET Hartree.  Two forms:

* against the oracle: walkers 0..2^16-1 of the P_z workload (all 12000 steps of
  dt = 0.0005, limiter a = 1) and of the triplet workload (4000 steps of
  dt = 0.001), the window energy over [T/2, T] and the slope L(T)/T;
* at full size, against the binary64 GPU path (itself held to the oracle per
  walker at 1e-12): the paired difference of the window energies over several
  seeds, whose mean plus three standard errors lies inside the budget.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import estimators as est
from paper_1703_08977_amd import he_fk_energy
from paper_1703_08977_amd import workloads as W

from hefk_testutil import gpu_available, gpu_run, log_mean_weight

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs an AMD Instinct GPU")]

MIXED_BUDGET = 2e-6  # Ha: one fifth of the 1e-5 Ha error the time-to-accuracy metric asks for


@pytest.mark.parametrize("name", ["he_2P_pz_16m", "he_2tripS_4m"])
def test_mixed_energy_within_budget_of_the_oracle(name):
    cfg = W.get(name)
    assert cfg["precision"] == "mixed" and cfg["contract"] == 2
    n = 1 << 16
    print("mixed vs oracle: %s, walkers 0..%d, %d steps" % (name, n - 1, cfg["n_steps"]), flush=True)
    g = gpu_run(cfg, n_walkers=n)
    r = oracle.run(dict(cfg, precision="fp64"), np.arange(n), cfg["n_steps"], cfg["sample_every"])
    dts = cfg["dt"] * cfg["sample_every"]
    T = cfg["n_steps"] * cfg["dt"]
    e_mixed = he_fk_energy(g["samples"], dts, cfg["e_ref"], "window")[0][0]
    e_oracle = est.e_window(r["samples"], dts, cfg["e_ref"])
    dL = (log_mean_weight(g["samples"])[-1] - log_mean_weight(r["samples"])[-1]) / T
    print("  E_window mixed %.9f, oracle %.9f, difference %.3e Ha; L(T)/T difference %.3e" %
          (e_mixed, e_oracle, e_mixed - e_oracle, dL), flush=True)
    assert abs(e_mixed - e_oracle) <= MIXED_BUDGET
    assert abs(dL) <= MIXED_BUDGET
    # both sides count the same walkers; the absorption decisions of a handful may differ
    assert g["samples"][-1, 6] == r["samples"][-1, 6]
    assert abs(g["samples"][-1, 4] - r["samples"][-1, 4]) <= 1e-3 * n


def _window(cfg, seed):
    from paper_1703_08977_amd import Ensemble
    ens = Ensemble(dict(cfg, seed=seed)).init()
    rows = ens.propagate(0, cfg["n_steps"], cfg["sample_every"]).cpu().numpy()
    dts = cfg["dt"] * cfg["sample_every"]
    return he_fk_energy(rows, dts, cfg["e_ref"], "window")[0][0]


@pytest.mark.parametrize("name,seeds", [("he_2P_pz_16m", 4), ("he_2tripS_4m", 8)])
def test_mixed_minus_fp64_paired_over_seeds_full_size(name, seeds):
    cfg = W.get(name)
    d = []
    for seed in range(seeds):
        print("paired seeds: %s, seed %d (mixed, then binary64)" % (name, seed), flush=True)
        em = _window(cfg, seed)
        e64 = _window(dict(cfg, precision="fp64"), seed)
        d.append(em - e64)
        print("  seed %d: mixed %.9f, FP64 %.9f, difference %.3e Ha" % (seed, em, e64, d[-1]), flush=True)
    d = np.array(d)
    mean, se = d.mean(), d.std(ddof=1) / math.sqrt(len(d))
    print("  paired mixed - FP64: %.3e +- %.3e Ha over %d seeds" % (mean, se, len(d)), flush=True)
    assert abs(mean) + 3.0 * se <= MIXED_BUDGET
