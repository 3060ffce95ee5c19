"""Statistical GPU tests of the whole path against closed forms and exact energies
(5 sigma; sigma from the sample itself or from walker-block jackknife)."""
import math

import numpy as np
import pytest

from paper_1703_08977_amd import workloads as W

from hefk_testutil import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs an AMD Instinct GPU")]

EXACT_1S = -2.9037243770341195


def test_variational_energy_of_start_ensemble():
    # |psi|^2 start for exp(-alpha(r1 + r2)), alpha = 27/16, 2^20 walkers:
    # <E_L> = alpha^2 - 27 alpha / 8, <1/r_i> = alpha, <1/r12> = 5 alpha / 8
    import torch
    from paper_1703_08977_amd import Ensemble
    cfg = W.get("he_1s_expo_4k", n_walkers=1 << 20)
    e = Ensemble(cfg).init()
    x, _, el = e.state()
    a = 27 / 16
    n = len(el)
    assert abs(el.mean() - (a * a - 27 * a / 8)) < 5 * el.std() / math.sqrt(n)
    inv_r = 0.5 * (1 / np.linalg.norm(x[:, :3], axis=1) + 1 / np.linalg.norm(x[:, 3:], axis=1))
    assert abs(inv_r.mean() - a) < 5 * inv_r.std() / math.sqrt(n)
    inv_r12 = 1 / np.linalg.norm(x[:, :3] - x[:, 3:], axis=1)
    assert abs(inv_r12.mean() - 5 * a / 8) < 5 * inv_r12.std() / math.sqrt(n)
    torch.cuda.synchronize()


def test_hydrogen_projection():
    # two hydrogen atoms with alpha = 0.8: E(0) = alpha^2 - 2 alpha = -0.96; E(T) -> -1
    from paper_1703_08977_amd import Ensemble, he_fk_energy
    from paper_1703_08977_amd.stats import jackknife
    cfg = W.get("hydrogen", theta=[0.8], n_walkers=1 << 20, dt=0.001, n_steps=8000, sample_every=100,
                e_ref=-0.96, n_metropolis=500)
    e = Ensemble(cfg).init()
    s = e.propagate(0, cfg["n_steps"], cfg["sample_every"]).cpu().numpy()
    mix0 = s[0, 2] / s[0, 1]
    x, _, el0 = e.state()
    E, err = jackknife(e.block_rows(cfg["n_steps"], cfg["sample_every"]).cpu().numpy(), 0.1, cfg["e_ref"], "window")
    assert abs(E - he_fk_energy(s, 0.1, cfg["e_ref"], "window")[0][0]) < 1e-12
    # E(t) over t in [4, 8]: excited-state contamination of the 1s projection is e^{-(3/8) 4} ~ 0.2 of
    # the variational error at the window start; the time-step bias is O(dt)
    assert -1.0 - 5 * err - 0.002 < E < -1.0 + 0.01, (E, err)
    assert abs(mix0 + 0.96) < 0.01


def test_ground_state_energy_bounds():
    # Pade-Jastrow trial, 2^20 walkers, dt = 0.001, T = 5: within [exact - 5 sigma - dt bias, exact + 2e-3]
    from paper_1703_08977_amd import Ensemble
    from paper_1703_08977_amd.stats import jackknife
    cfg = W.get("he_1s_pade_1m", dt=0.001, n_steps=5000, sample_every=50)
    e = Ensemble(cfg).init()
    e.propagate(0, cfg["n_steps"], cfg["sample_every"])
    E, err = jackknife(e.block_rows(cfg["n_steps"], cfg["sample_every"]).cpu().numpy(), 0.05, cfg["e_ref"], "window")
    assert EXACT_1S - 5 * err - 5e-4 < E < EXACT_1S + 2e-3, (E, err)


def test_fixed_node_pz_energy_lies_above_the_exact_one():
    # Absorbing at the trial's node gives the lowest energy of that nodal pocket; the P_z trial's
    # node is not exact, so its energy lies above the exact 2^1P energy, by the nodal error of this
    # trial (1.7 mHa at T = 6, dt = 0.0005); mixed precision, 2^22 walkers, 5 sigma of the
    # walker-block jackknife
    from paper_1703_08977_amd import Ensemble
    from paper_1703_08977_amd.stats import jackknife
    exact = -2.123843086498093
    cfg = W.get("he_2P_pz_16m", n_walkers=1 << 22)
    e = Ensemble(cfg).init()
    e.propagate(0, cfg["n_steps"], cfg["sample_every"])
    dts = cfg["dt"] * cfg["sample_every"]
    E, err = jackknife(e.block_rows(cfg["n_steps"], cfg["sample_every"]).cpu().numpy(), dts, cfg["e_ref"], "window")
    assert exact - 5 * err < E < exact + 0.003, (E, err)


def test_triplet_energy_extrapolates_to_the_exact_2_3S_energy():
    # The triplet trial's node r1 = r2 is the exact node of 2^3S, so the fixed-node energy is the
    # exact one.  The continuous drifted walk never reaches that node (the drift repels it as
    # 1/distance); every absorption is a discretisation event, at a rate ~ sqrt(dt).  Per dt in
    # {0.004, 0.002, 0.001, 0.0005}: the window energy over [40, 80], where the projection onto the
    # lowest state of the pocket is complete (4 seeds of 2^22 walkers, mixed precision, errors from
    # the walker-block jackknife); then E(dt) = E0 + a sqrt(dt) + b dt by weighted least squares.
    # E0 must meet the exact 2^3S energy (Table 6, "Var" row) within 3 sigma, and the absorbed
    # fraction must shrink by about sqrt(2) per halving of dt.
    from paper_1703_08977_amd import Ensemble, he_fk_energy_blocks
    exact = -2.17522937823679130
    T, seeds = 80.0, 4
    dts = (0.004, 0.002, 0.001, 0.0005)
    E, S, absorbed = [], [], []
    for dt in dts:
        se = int(round(0.5 / dt))
        cfg = W.get("he_2tripS_4m", dt=dt, n_steps=int(round(T / dt)), sample_every=se)
        vals, errs, dead = [], [], []
        for seed in range(seeds):
            print("triplet limit: dt %g seed %d" % (dt, seed), flush=True)
            e = Ensemble(dict(cfg, seed=seed)).init()
            rows = e.propagate(0, cfg["n_steps"], se).cpu().numpy()
            v, err = he_fk_energy_blocks(e.block_rows(cfg["n_steps"], se).cpu().numpy(), dt * se, cfg["e_ref"],
                                         "window")
            vals.append(v)
            errs.append(err)
            dead.append(1.0 - rows[-1, 4] / rows[-1, 6])
            del e
        E.append(np.mean(vals))
        S.append(math.sqrt(np.mean(np.square(errs)) / seeds))
        absorbed.append(np.mean(dead))
        print("  E(dt = %g) = %.7f +- %.7f, absorbed %.4f" % (dt, E[-1], S[-1], absorbed[-1]), flush=True)
    x = np.array(dts)
    A = np.stack([np.ones_like(x), np.sqrt(x), x], axis=1)
    w = 1.0 / np.square(S)
    cov = np.linalg.inv(A.T @ (A * w[:, None]))
    coef = cov @ (A.T @ (w * np.array(E)))
    e0, e0s = coef[0], math.sqrt(cov[0, 0])
    print("  E0 = %.7f +- %.7f (exact %.7f, %.1f sigma)" % (e0, e0s, exact, (e0 - exact) / e0s), flush=True)
    assert abs(e0 - exact) < 3 * e0s, (e0, e0s)
    assert e0s < 2e-4
    ratios = np.array(absorbed[:-1]) / np.array(absorbed[1:])
    assert np.all((ratios > 1.25) & (ratios < 1.6)), ratios


def test_exact_trial_has_zero_variance_energy():
    # Z = 2 without 1/r12 and the exact trial: every estimator gives -4 with zero spread
    from paper_1703_08977_amd import Ensemble, he_fk_energy
    cfg = W.get("exact_noee", n_walkers=1 << 16, e_ref=-3.5)
    e = Ensemble(cfg).init()
    s = e.propagate(0, 400, 20).cpu().numpy()
    E = he_fk_energy(s, 0.2, cfg["e_ref"], "fd")[0]
    assert np.abs(E + 4.0).max() < 1e-10
    assert np.abs(he_fk_energy(s, 0.2, cfg["e_ref"], "mixed")[0] + 4.0).max() < 1e-12
    ess = he_fk_energy(s, 0.2, cfg["e_ref"], "fd")[1][:, 1]
    assert np.abs(ess - (1 << 16)).max() < 1e-6


@pytest.mark.parametrize("name", ["he_2tripS_fn3_1m", "he_2tripS_fn5_1m"])
def test_paper_trial_energy_lambda0_on_gpu(name):
    # the trial energies lambda0 printed in Tables 1 and 2 (trial functions 3 and 5),
    # from the GPU start ensemble of 2^22 walkers in both precisions
    from paper_1703_08977_amd import Ensemble
    for prec in ("fp64", "mixed"):
        cfg = W.get(name, n_walkers=1 << 22, precision=prec)
        e = Ensemble(cfg).init()
        _, _, el = e.state()
        se = el.std() / math.sqrt(len(el))
        assert abs(el.mean() - cfg["e_ref"]) < 5 * se, (name, prec, el.mean(), cfg["e_ref"], se)


@pytest.mark.parametrize("noise", ["gauss", "pm1"])
def test_long_projection_ground_state_extrapolates_to_the_exact_energy(noise):
    # Pade-Jastrow trial, 2^20 walkers, T = 16 (window [8, 16], past the excited-state
    # decay), dt in {0.002, 0.001}, 4 seeds each; E(dt) = E0 + s dt extrapolated to dt = 0
    # must meet the exact non-relativistic 1^1S energy (5 sigma of the extrapolation), for
    # Gaussian increments and for the paper's +-1 walk alike (both are weak order 1)
    from paper_1703_08977_amd import Ensemble, he_fk_energy
    rows = []
    for dt in (0.002, 0.001):
        se = int(round(0.1 / dt))
        cfg = W.get("he_1s_pade_1m", dt=dt, n_steps=int(round(16 / dt)), sample_every=se, noise=noise)
        vals = []
        for seed in range(4):
            e = Ensemble(dict(cfg, seed=seed)).init()
            s = e.propagate(0, cfg["n_steps"], se).cpu().numpy()
            vals.append(he_fk_energy(s, dt * se, cfg["e_ref"], "window")[0][0])
            del e
        rows.append((dt, float(np.mean(vals)), float(np.std(vals, ddof=1) / 2)))
    (d1, e1, s1), (d2, e2, s2) = rows
    e0 = e2 - (e1 - e2) * d2 / (d1 - d2)           # line through the two points, at dt = 0
    s0 = math.hypot(2 * s2, s1)                    # d e0 / d e2 = 2, d e0 / d e1 = -1
    assert abs(e0 - EXACT_1S) < 5 * s0 + 5e-5, (rows, e0, s0)


def test_bridge_weight_removes_the_missed_node_touches_of_the_brownian_walk():
    # Brownian walkers (the plain walk, potential switched off by Z = 1e-9) in a nodal pocket of
    # r1 = r2, T = 0.5, 2^22 walkers x 4 seeds: ln S(T) = L(T) with the end-point test alone
    # misses the touches inside a step, an O(sqrt dt) error; with the bridge weight ln S(T)
    # no longer depends on dt at this resolution
    from paper_1703_08977_amd import Ensemble
    from hefk_testutil import log_mean_weight

    def lnS(dt, bridge):
        cfg = W.get("exact_triplet_noee", n_walkers=1 << 22, Z=1e-9, e_ref=0.0, plain=True, bridge=bridge,
                    dt=dt, n_steps=int(round(0.5 / dt)), sample_every=int(round(0.1 / dt)))
        v = []
        for seed in range(4):
            e = Ensemble(dict(cfg, seed=seed)).init()
            v.append(log_mean_weight(e.propagate(0, cfg["n_steps"], cfg["sample_every"]).cpu().numpy())[-1])
            del e
        return float(np.mean(v)), float(np.std(v, ddof=1) / 2)

    (b1, sb1), (b2, sb2) = lnS(0.002, True), lnS(0.0005, True)
    (e1, se1), (e2, se2) = lnS(0.002, False), lnS(0.0005, False)
    tol = 5 * math.hypot(sb1, sb2) + 1e-4
    assert abs(b1 - b2) < tol, (b1, b2, tol)
    assert e2 - e1 < -5 * tol, (e1, e2, tol)       # end-point survival still falls with dt
    assert b2 < e2                                  # touches between steps lower the survival


def test_bridge_is_exact_for_brownian_walkers_at_a_flat_node():
    # Trial function 7 has the node plane z1 + z2 = 0.  Brownian walkers (potential off): the
    # distance u = |z1 + z2| / sqrt(2) is a one-dimensional Brownian motion of variance t, which
    # survives to T with probability erf(u0 / sqrt(2 T)).  Over the start ensemble that expectation
    # is exact; with the bridge weight the walk reproduces it at any dt (sigma = sqrt(S (1 - S) / N)),
    # the end-point test alone overshoots by O(sqrt dt).
    from scipy.special import erf
    import torch
    from paper_1703_08977_amd import Ensemble
    T, n = 0.5, 1 << 22
    for dt in (0.004, 0.001):
        k = int(round(T / dt))
        cfg = W.get("he_2P_fn7_1m", n_walkers=n, Z=1e-9, ee=0, e_ref=0.0, plain=True, noise="gauss",
                    quad="trapezoid", dt=dt, n_steps=k, sample_every=k, precision="fp64")
        S = {}
        for bridge in (False, True):
            e = Ensemble(dict(cfg, bridge=bridge)).init()
            u0 = ((e.x[2] + e.x[5]).abs() / math.sqrt(2.0)).cpu().numpy()
            exact = float(np.mean(erf(u0 / math.sqrt(2 * T))))
            s = e.propagate(0, k, k).cpu().numpy()
            S[bridge] = math.exp(s[-1, 0]) * s[-1, 1] / s[-1, 6]
            del e
            torch.cuda.empty_cache()
        sig = math.sqrt(exact * (1 - exact) / n)
        assert abs(S[True] - exact) < 5 * sig, (dt, S, exact, sig)
        assert S[False] - exact > 5 * sig, (dt, S, exact, sig)
