"""GPU tests of the pathwise gradient he_fk_grad (through the C ABI):
against the oracle's complex-step derivative (same start, same noise),
against central differences of the GPU forward map with common random
numbers at the full 2^18-walker size, the start-law score term, the
autograd wrapper, and the argument checks."""
import numpy as np
import pytest

import oracle
from paper_1703_08977_amd import workloads as W

from hefk_testutil import gpu_available, log_mean_weight

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs an AMD Instinct GPU")]


def _forward(cfg, n=None, x0=None):
    import torch
    from paper_1703_08977_amd import Ensemble
    e = Ensemble(cfg, n_walkers=n)
    if x0 is None:
        e.init()
    else:
        e.x.copy_(x0)
        e.lnw.zero_()
    x_start = e.x.clone()
    ns, se, ce = cfg["n_steps"], cfg["sample_every"], cfg["ckpt_every"]
    ckpt = torch.empty((ns // ce + 1, 7, e.n), dtype=torch.float64, device="cuda")
    s = e.propagate(0, ns, se, ckpt=ckpt, ckpt_every=ce)
    torch.cuda.synchronize()
    return e, ckpt, s, x_start


def _grad(e, ckpt, s, cfg, gL, flags=0):
    import torch
    from paper_1703_08977_amd import api
    ns, se, ce = cfg["n_steps"], cfg["sample_every"], cfg["ckpt_every"]
    nb = api.he_fk_grad_scratch_bytes(e.p, ns, se, ce)
    scratch = torch.empty(nb, dtype=torch.uint8, device="cuda")
    d = torch.empty(2, dtype=torch.float64, device="cuda")
    api.he_fk_grad(e.p, ckpt.data_ptr(), s.data_ptr(), gL, ns, se, ce, flags, scratch.data_ptr(), nb, d.data_ptr())
    return d.cpu().numpy()


@pytest.mark.parametrize("over,ce", [({}, 50), ({"quad": "right"}, 25), ({"contract": 2}, 100),
                                     ({"noise": "pm1"}, 50), ({"trial": "expo", "theta": [1.8]}, 50), ({}, 1),
                                     ({"quad": "right", "noise": "pm1"}, 1), ({"trial": "expo", "theta": [1.8]}, 1)])
def test_grad_matches_oracle_complex_step(over, ce):
    cfg = W.get("he_1s_pade_grad_256k", n_steps=200, sample_every=50, ckpt_every=ce, **over)
    n = 3001
    e, ckpt, s, x0 = _forward(cfg, n)
    gL = np.array([0.0, 0.3, -0.7, 1.1, -0.5])
    got = _grad(e, ckpt, s, cfg, gL)
    y0 = x0.t().contiguous().cpu().numpy()
    ref = oracle.grad_objective(cfg, np.arange(n), y0, 200, 50, gL)
    assert np.abs(got - ref).max() <= 1e-10 * max(np.abs(ref).max(), 1e-3), (got, ref)


@pytest.mark.parametrize("over", [{}, {"quad": "right"}])
def test_sweep_over_the_stored_trajectory_equals_the_recomputing_sweep(over):
    # a checkpoint at every step makes the reverse sweep read the stored positions instead
    # of recomputing segments: the same bits, with the score and second-moment terms on
    from paper_1703_08977_amd import _lib
    n = 1 << 16
    gL = np.zeros(21)
    gL[-1], gL[-2], gL[7] = -10.0, 10.0, 0.5
    gL2 = np.zeros(21)
    gL2[-1], gL2[3] = 0.7, -0.2
    flags = _lib.GRAD_SCORE | _lib.GRAD_MOMENT2
    got = {}
    for ce in (1, 50, 10):
        cfg = W.get("he_1s_pade_grad_256k", n_walkers=n, ckpt_every=ce, **over)
        e, ckpt, s, x0 = _forward(cfg)
        got[ce] = _grad(e, ckpt, s, cfg, np.concatenate([gL, gL2]), flags=flags)
        del e, ckpt
    print("dtheta", got)
    assert np.array_equal(got[1], got[50]) and np.array_equal(got[1], got[10]), got


@pytest.mark.parametrize("ce", [1, 50])
def test_grad_matches_the_host_build_of_the_same_sweep(ce):
    # the GPU adjoint against the same reverse sweep compiled for the host (one walker at a
    # time, its own start ensemble and noise), on the GPU's sample rows: per walker the same
    # arithmetic, so the sums over walkers agree to 1e-12
    import math
    from hefk_testutil import adjoint_host_run
    from paper_1703_08977_amd import _lib
    cfg = W.get("he_1s_pade_grad_256k", n_steps=200, sample_every=50, ckpt_every=ce)
    n = 2048
    e, ckpt, s, x0 = _forward(cfg, n)
    gL = np.array([0.0, 0.3, -0.7, 1.1, -0.5])
    gL2 = np.array([0.0, 0.5, 0.0, -0.8, 1.2])
    got = _grad(e, ckpt, s, cfg, np.concatenate([gL, gL2]), flags=_lib.GRAD_MOMENT2)
    host = adjoint_host_run(cfg, np.arange(n), 200, 50, ce, s.cpu().numpy(), gL, gL2)
    ref = np.array([math.fsum(host[:, d]) for d in range(2)])
    print("gpu", got, "host", ref, "diff", got - ref)
    assert np.abs(got - ref).max() <= 1e-12 * max(np.abs(ref).max(), 1e-3), (got, ref)


def test_grad_score_term_matches_oracle():
    cfg = W.get("he_1s_pade_grad_256k", n_steps=200, sample_every=50, ckpt_every=50)
    n = 2048
    e, ckpt, s, x0 = _forward(cfg, n)
    gL = np.array([0.2, 0.0, 0.5, -1.0, 1.3])
    from paper_1703_08977_amd import _lib
    got = _grad(e, ckpt, s, cfg, gL, flags=_lib.GRAD_SCORE)
    ref = oracle.grad_objective(cfg, np.arange(n), x0.t().contiguous().cpu().numpy(), 200, 50, gL, score=True)
    assert np.abs(got - ref).max() <= 1e-10 * max(np.abs(ref).max(), 1e-3), (got, ref)


@pytest.mark.parametrize("score", [False, True])
def test_grad_second_moment_matches_oracle(score):
    # J = sum_s gL_s L_s + sum_s gL2_s L2_s, L2 = ln <w^2> (flag HE_FK_GRAD_MOMENT2)
    from paper_1703_08977_amd import _lib
    cfg = W.get("he_1s_pade_grad_256k", n_steps=200, sample_every=50, ckpt_every=50)
    n = 2048
    e, ckpt, s, x0 = _forward(cfg, n)
    gL = np.array([0.0, 0.3, -0.7, 1.1, -0.5])
    gL2 = np.array([0.0, 0.5, 0.0, -0.8, 1.2])
    flags = _lib.GRAD_MOMENT2 | (_lib.GRAD_SCORE if score else 0)
    got = _grad(e, ckpt, s, cfg, np.concatenate([gL, gL2]), flags=flags)
    ref = oracle.grad_objective(cfg, np.arange(n), x0.t().contiguous().cpu().numpy(), 200, 50, gL, score=score,
                                gL2=gL2)
    assert np.abs(got - ref).max() <= 1e-10 * max(np.abs(ref).max(), 1e-3), (got, ref)


def test_weight_variance_gradient_through_autograd_against_central_differences():
    # d ln(<w^2>/<w>^2)(T) / d(alpha, beta) through the autograd wrapper, against central
    # differences of the GPU forward map at the same start positions and noise
    import torch
    from paper_1703_08977_amd.autograd import log_space_moments, weight_variance
    cfg = W.get("he_1s_pade_grad_256k", n_walkers=1 << 16, n_steps=500, sample_every=50, ckpt_every=50)
    theta = torch.tensor([2.0, 0.25], dtype=torch.float64, requires_grad=True)
    L, L2 = log_space_moments(theta, cfg)
    V = weight_variance(L, L2)
    V.backward()
    e, ckpt, s, x0 = _forward(cfg)
    fd = []
    for d in range(2):
        vals = []
        for sgn in (+1, -1):
            th = list(cfg["theta"])
            th[d] += sgn * 1e-5
            _, _, sp, _ = _forward(dict(cfg, theta=th), x0=x0)
            h = sp.cpu().numpy()
            vals.append(float((2 * h[-1, 0] + np.log(h[-1, 3])) - 2 * (h[-1, 0] + np.log(h[-1, 1])) + np.log(h[-1, 6])))
        fd.append((vals[0] - vals[1]) / 2e-5)
    fd = np.array(fd)
    assert np.abs(theta.grad.numpy() - fd).max() <= 1e-6 * max(np.abs(fd).max(), 1e-3), (theta.grad, fd)


def test_grad_full_size_against_central_differences():
    # 2^18 walkers x 1000 steps, a checkpoint at every step (the reverse sweep reads the
    # stored trajectory): d E(T=2) / d(alpha, beta) against central differences of the
    # GPU forward map at the same start positions and noise.
    cfg = W.get("he_1s_pade_grad_256k")
    e, ckpt, s, x0 = _forward(cfg)
    dts = cfg["dt"] * cfg["sample_every"]
    ns = cfg["n_steps"] // cfg["sample_every"] + 1
    gL = np.zeros(ns)
    gL[-1], gL[-2] = -1.0 / dts, 1.0 / dts  # E(T) = e_ref - (L[-1] - L[-2]) / dts
    got = _grad(e, ckpt, s, cfg, gL)
    fd = []
    for d in range(2):
        vals = []
        for sgn in (+1, -1):
            th = list(cfg["theta"])
            th[d] += sgn * 1e-5
            c = dict(cfg, theta=th)
            _, _, sp, _ = _forward(c, x0=x0)
            vals.append(float(np.sum(gL * log_mean_weight(sp.cpu().numpy()))))
        fd.append((vals[0] - vals[1]) / 2e-5)
    fd = np.array(fd)
    assert np.abs(got - fd).max() <= 1e-6 * max(np.abs(fd).max(), 1e-3), (got, fd)


def test_autograd_function_uses_the_adjoint():
    import torch
    from paper_1703_08977_amd.autograd import energy_fd, log_space_average
    cfg = W.get("he_1s_pade_grad_256k", n_walkers=4096, n_steps=200, sample_every=50, ckpt_every=50)
    theta = torch.tensor([2.0, 0.25], dtype=torch.float64, requires_grad=True)
    L = log_space_average(theta, cfg)
    E = energy_fd(L, cfg)
    E.backward()
    e, ckpt, s, x0 = _forward(cfg)
    gL = np.zeros(5)
    dts = cfg["dt"] * cfg["sample_every"]
    gL[-1], gL[-2] = -1.0 / dts, 1.0 / dts
    ref = _grad(e, ckpt, s, cfg, gL)
    assert np.allclose(theta.grad.numpy(), ref, rtol=1e-12, atol=0)
    assert abs(float(E) - (cfg["e_ref"] - (log_mean_weight(s.cpu().numpy())[-1] -
                                           log_mean_weight(s.cpu().numpy())[-2]) / dts)) < 1e-12


def test_grad_vanishes_in_expectation_for_the_exact_trial():
    # Z = 2 without 1/r12 and psi = e^{-alpha (r1 + r2)} at alpha = 2: E_L = -4 everywhere, so
    # w = 1 on every path and dE(T)/d alpha is the mean of 1/r1 + 1/r2 - 4 over the last
    # interval, zero under |psi|^2 (<1/r> = alpha); the beta component is exactly zero
    from paper_1703_08977_amd import _lib
    cfg = W.get("he_1s_pade_grad_256k", trial="expo", theta=[2.0], ee=0, e_ref=-4.0, dt=0.0005,
                n_steps=1000, sample_every=50, ckpt_every=50)
    dts = cfg["dt"] * cfg["sample_every"]
    ns = cfg["n_steps"] // cfg["sample_every"] + 1
    gL = np.zeros(ns)
    gL[-1], gL[-2] = -1.0 / dts, 1.0 / dts
    g = []
    for seed in range(4):
        c = dict(cfg, seed=seed)
        e, ckpt, s, _ = _forward(c)
        assert np.all(log_mean_weight(s.cpu().numpy()) == 0.0)
        g.append(_grad(e, ckpt, s, c, gL, flags=_lib.GRAD_SCORE))
    g = np.array(g)
    assert np.all(g[:, 1] == 0.0)
    # per seed: sigma(1/r1 + 1/r2) / sqrt(N) = sqrt(2 alpha^2 / N) = 0.0055
    assert abs(g[:, 0].mean()) < 5 * 0.0055 / 2, g[:, 0]


def test_grad_rejects_unsupported_cases():
    import torch
    from paper_1703_08977_amd import _lib, api
    cfg = W.get("he_1s_pade_grad_256k", n_walkers=512, n_steps=100, sample_every=50, ckpt_every=50)
    e, ckpt, s, _ = _forward(cfg)
    gL = np.zeros(3)
    for over in ({"trial": "pz", "sym": 1, "theta": [2, 0.3, 0.5, 0.5]}, {"precision": "mixed"},
                 {"drift_limit": 1.0}):
        p = api.make_params(dict(cfg, **over))
        assert api.he_fk_grad_scratch_bytes(p, 100, 50, 50) == 0
    nb = api.he_fk_grad_scratch_bytes(e.p, 100, 50, 50)
    scratch = torch.empty(nb, dtype=torch.uint8, device="cuda")
    d = torch.empty(2, dtype=torch.float64, device="cuda")
    with pytest.raises(_lib.HeFkError) as ei:
        api.he_fk_grad(e.p, ckpt.data_ptr(), s.data_ptr(), gL, 100, 50, 50, 4, scratch.data_ptr(), nb,
                       d.data_ptr())
    assert ei.value.code == _lib.HE_FK_EINVAL
    with pytest.raises(_lib.HeFkError) as ei:
        api.he_fk_grad(e.p, ckpt.data_ptr(), s.data_ptr(), gL, 100, 50, 50, 0, scratch.data_ptr(), nb - 1,
                       d.data_ptr())
    assert ei.value.code == _lib.HE_FK_ESCRATCH
    with pytest.raises(_lib.HeFkError) as ei:
        api.he_fk_grad(e.p, ckpt.data_ptr(), s.data_ptr(), gL, 100, 50, 30, 0, scratch.data_ptr(), nb,
                       d.data_ptr())
    assert ei.value.code == _lib.HE_FK_EINVAL
