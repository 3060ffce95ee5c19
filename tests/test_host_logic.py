"""CPU tests of the product's host logic: the C ABI loads and exports every
declared symbol, argument checks, the host energy estimators against the
oracle's, and a host build of the kernels' per-walker arithmetic against the
oracle (same Philox streams)."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

import oracle
from oracle import estimators as est
from paper_1703_08977_amd import _lib, api
from paper_1703_08977_amd import workloads as W

from hefk_testutil import ROOT, adjoint_host_run, host_run


def test_library_exports_every_declared_symbol():
    hdr = open(os.path.join(ROOT, "include", "he_fk.h")).read()
    names = set(re.findall(r"^\s*(?:int|size_t|const char\*)\s+(he_fk_\w+)\s*\(", hdr, flags=re.M))
    assert names == set(_lib.EXPORTS)
    L = ctypes.CDLL(_lib.LIB_PATH)
    for n in names:
        assert hasattr(L, n), n


def test_strerror():
    for c in (0, -1, -2, -3, -4, -5):
        assert _lib.strerror(c)
    assert _lib.strerror(-99) == "unknown error"


def _bad_params():
    base = W.get("he_1s_expo_4k")
    yield api.make_params(base, dt=-0.1)
    yield api.make_params(base, dt=float("nan"))
    yield api.make_params(base, n_walkers=0)
    yield api.make_params(base, theta=[0.0])
    yield api.make_params(base, Z=0.0)
    yield api.make_params(base, metropolis_sigma=0.0)
    p = api.make_params(base)
    p.trial = 7
    yield p
    p = api.make_params(W.get("he_2P_pz_16m"))
    p.sym = 0
    yield p
    p = api.make_params(base)
    p.contract = 3
    yield p
    p = api.make_params(base)
    p.walker_offset = (1 << 64) - 10
    yield p
    p = api.make_params(base)
    p.flags = 4            # unknown variant bit
    yield p
    p = api.make_params(base)
    p.reserved = 1
    yield p
    yield api.make_params(base, plain=True, drift_limit=0.5)   # the limiter belongs to the drifted walk
    yield api.make_params(base, bridge=True)                   # no node to touch
    yield api.make_params(W.get("he_1s_pade_1m"), bridge=True)


def test_invalid_params_rejected_before_any_launch():
    w = _lib.HeFkWalkers(1, 1, 1)  # never dereferenced: the checks come first
    for p in _bad_params():
        assert _lib.lib().he_fk_init(ctypes.byref(p), ctypes.byref(w), None) == _lib.HE_FK_EINVAL
        assert _lib.lib().he_fk_propagate_workspace_bytes(ctypes.byref(p), 10, 5) == 0
        assert _lib.lib().he_fk_propagate_noalloc(ctypes.byref(p), ctypes.byref(w), 0, 10, 5, ctypes.c_void_p(1),
                                                  None, 0, None) == _lib.HE_FK_EINVAL
    p = api.make_params(W.get("he_1s_expo_4k"))
    assert _lib.lib().he_fk_init(ctypes.byref(p), None, None) == _lib.HE_FK_EINVAL
    z = _lib.HeFkWalkers(0, 0, 0)
    assert _lib.lib().he_fk_init(ctypes.byref(p), ctypes.byref(z), None) == _lib.HE_FK_EINVAL
    # step arguments: n_steps not a multiple of sample_every, negative steps
    for (s0, ns, se) in ((0, 10, 3), (-1, 10, 5), (0, -5, 5), (0, 10, 0), (2**31 - 5, 10, 5)):
        rc = _lib.lib().he_fk_propagate(ctypes.byref(p), ctypes.byref(w), s0, ns, se, ctypes.c_void_p(1),
                                        None, 0, ctypes.c_void_p(1), ctypes.c_size_t(1 << 30), None)
        assert rc == _lib.HE_FK_EINVAL
        rc = _lib.lib().he_fk_propagate_noalloc(ctypes.byref(p), ctypes.byref(w), s0, ns, se, ctypes.c_void_p(1),
                                                None, 0, None)
        assert rc == _lib.HE_FK_EINVAL


def test_variant_flags_accepted_where_defined_and_not_by_the_gradient():
    ok = [api.make_params(W.get("he_1s_pade_1m"), plain=True),
          api.make_params(W.get("he_2tripS_4m"), bridge=True),
          api.make_params(W.get("he_2P_pz_16m", drift_limit=0.0), plain=True, bridge=True)]
    for p in ok:
        assert _lib.lib().he_fk_propagate_workspace_bytes(ctypes.byref(p), 10, 5) > 0 or not _gpu_visible()
    # the adjoint is derived for the generalized walk only
    p = api.make_params(W.get("he_1s_pade_grad_256k"))
    assert _lib.lib().he_fk_grad_scratch_bytes(ctypes.byref(p), 100, 50, 50) > 0
    p = api.make_params(W.get("he_1s_pade_grad_256k"), plain=True)
    assert _lib.lib().he_fk_grad_scratch_bytes(ctypes.byref(p), 100, 50, 50) == 0


def _gpu_visible():
    import torch
    return torch.cuda.is_available()


def _random_rows(rng, n, N=1000, dead_row=None, bad_row=None):
    s = np.zeros((n, 8))
    t = np.arange(n) * 0.05
    s[:, 0] = -0.1 * t + 0.01 * rng.normal(size=n) + 3.0
    s[:, 1] = rng.uniform(50, 100, size=n)
    s[:, 2] = -2.9 * s[:, 1] * (1 + 0.01 * rng.normal(size=n))
    s[:, 3] = s[:, 1] * rng.uniform(1, 5, size=n)
    s[:, 4] = N
    s[:, 6] = N
    if dead_row is not None:
        s[dead_row, 4] = 0
    if bad_row is not None:
        s[bad_row, 5] = 2
    return s


@pytest.mark.parametrize("n", [3, 4, 41, 121, 600])
def test_energy_estimators_match_oracle(n):
    rng = np.random.default_rng(n)
    s = _random_rows(rng, n)
    e_ref, dts = -2.9, 0.05
    out, aux, rc = api.he_fk_energy(s, dts, e_ref, "fd")
    assert rc == 0
    assert np.abs(out - est.e_fd(s, dts, e_ref)).max() < 1e-12
    assert np.abs(aux[:, 0] - est.log_mean_weight(s)).max() < 1e-14
    assert np.abs(aux[:, 1] - est.ess(s)).max() < 1e-9
    assert np.abs(aux[:, 2] - est.log_mean_square_weight(s)).max() < 1e-14
    out, _, _ = api.he_fk_energy(s, dts, e_ref, "window")
    assert abs(out[0] - est.e_window(s, dts, e_ref)) < 1e-10
    out, _, _ = api.he_fk_energy(s, dts, e_ref, "fit")
    Ef, a = est.e_fit(s, dts, e_ref)
    assert abs(out[0] - Ef) < 1e-10 and abs(out[1] - a) < 1e-10
    w = rng.uniform(0.5, 2.0, size=n)
    out, _, _ = api.he_fk_energy(s, dts, e_ref, "fit", fit_w=w)
    Ef, a = est.e_fit(s, dts, e_ref, w=w)
    assert abs(out[0] - Ef) < 1e-10
    out, _, _ = api.he_fk_energy(s, dts, e_ref, "mixed")
    assert np.abs(out - est.e_mixed(s)).max() < 1e-14


@pytest.fixture(scope="module")
def walker_weights():
    # per-walker ln w and E_L at the sample times of an oracle run (4096 walkers of the triplet
    # trial, node absorption included), and the walkers of block 0 absorbed from sample 5 on, so
    # that a whole block has no live walker at the later rows
    cfg = W.get("he_2tripS_4m", precision="fp64", dt=0.01)
    r = oracle.run(cfg, np.arange(4096), 200, 10)
    ell = r["ell"].copy()
    ell[:64, 5:] = -np.inf
    return cfg, ell, r["els"]


@pytest.mark.parametrize("method", ["window", "fit", "fd", "mixed"])
@pytest.mark.parametrize("n_groups", [2, 5, 32, 64])
def test_block_jackknife_matches_a_direct_jackknife(walker_weights, method, n_groups):
    # the library's grouping, merge of partial rows and replicas against a jackknife written
    # here from the walkers themselves: each group's and each replica's rows are recomputed
    # from the walkers they hold (oracle.tuples), with the oracle's estimators
    cfg, ell, els = walker_weights
    block = 64                                  # 64 blocks of 64 walkers
    G = ell.shape[0] // block
    parts = np.stack([oracle.tuples(ell[b * block:(b + 1) * block], els[b * block:(b + 1) * block])
                      for b in range(G)])
    dts, e_ref = 10 * cfg["dt"], cfg["e_ref"]

    def stat(rows):
        if method == "window":
            return est.e_window(rows, dts, e_ref)
        if method == "fit":
            return est.e_fit(rows, dts, e_ref)[0]
        if method == "fd":
            return est.e_fd(rows, dts, e_ref)[-1]
        return est.e_mixed(rows)[-1]

    full, se = api.he_fk_energy_blocks(parts, dts, e_ref, method, n_groups)
    assert abs(full - stat(oracle.tuples(ell, els))) < 1e-11
    sizes = [len(a) for a in np.array_split(np.arange(G), n_groups)]   # larger groups first
    edges = np.concatenate([[0], np.cumsum(sizes)]) * block
    reps = []
    for g in range(n_groups):
        keep = np.ones(ell.shape[0], dtype=bool)
        keep[edges[g]:edges[g + 1]] = False
        reps.append(stat(oracle.tuples(ell[keep], els[keep])))
    reps = np.array(reps)
    se_direct = math.sqrt((n_groups - 1) / n_groups * np.sum((reps - reps.mean()) ** 2))
    assert abs(se - se_direct) < 1e-9 * max(se_direct, 1e-6), (se, se_direct)


def test_block_jackknife_argument_checks():
    parts = np.zeros((1, 4, 8))
    with pytest.raises(_lib.HeFkError):
        api.he_fk_energy_blocks(parts, 0.1, 0.0, "window")
    parts = np.zeros((4, 4, 8))
    with pytest.raises(_lib.HeFkError):
        api.he_fk_energy_blocks(parts, 0.1, 0.0, "window", n_groups=1)


@pytest.mark.parametrize("name,tol,weighted", [("paper_table3.txt", 1e-6, False), ("paper_table4.txt", 1e-6, False),
                                               ("paper_table1.txt", 5e-6, True)])
def test_energy_fit_reproduces_paper_tables(name, tol, weighted):
    rows, lam = [], {}
    for line in open(os.path.join(ROOT, "tests", "golden", name)):
        if line.startswith("# lambda0"):
            parts = line.replace("#", "").split()
            lam = {"l0": float(parts[2]), "l1": float(parts[5])}
        elif line.strip() and not line.startswith("#"):
            rows.append([float(v) for v in line.split()])
    tab = np.array(rows)
    # t * (ls-fit column), or ln z_t with weights 1/sigma^2 (Table 1), at t = 0, 8, ..., 48
    L = np.concatenate([[0.0], tab[:, 2] if weighted else tab[:, 0] * tab[:, 5]])
    w = np.concatenate([[0.0], 1.0 / tab[:, 4] ** 2]) if weighted else None
    N = 150000
    s = np.zeros((len(L), 8))
    s[:, 0] = L + math.log(N)
    s[:, 1] = 1.0
    s[:, 3] = 1.0
    s[:, 4] = N
    s[:, 6] = N
    out, _, rc = api.he_fk_energy(s, 8.0, lam["l0"], "fit", fit_w=w)
    assert rc == 0 and abs(out[0] - lam["l1"]) < tol


def test_energy_error_codes():
    rng = np.random.default_rng(3)
    s = _random_rows(rng, 10, dead_row=4)
    _, aux, rc = api.he_fk_energy(s, 0.05, -2.9, "fd", raise_on_error=False)
    assert rc == _lib.HE_FK_EALLDEAD and np.isfinite(aux[0, 0])
    s = _random_rows(rng, 10, bad_row=7, dead_row=2)
    _, _, rc = api.he_fk_energy(s, 0.05, -2.9, "fd", raise_on_error=False)
    assert rc == _lib.HE_FK_ENONFINITE
    s = _random_rows(rng, 10)
    for args in ((0.0, "fd"), (float("inf"), "fd")):
        _, _, rc = api.he_fk_energy(s, args[0], -2.9, args[1], raise_on_error=False)
        assert rc == _lib.HE_FK_EINVAL
    _, _, rc = api.he_fk_energy(s[:2], 0.05, -2.9, "fit", raise_on_error=False)
    assert rc == _lib.HE_FK_EINVAL
    s[3, 6] = 0
    _, _, rc = api.he_fk_energy(s, 0.05, -2.9, "fd", raise_on_error=False)
    assert rc == _lib.HE_FK_EINVAL


# --------------------------------------------------------------------------
# Host build of the kernels' per-walker code against the oracle (binary64).
# --------------------------------------------------------------------------

HOST_CASES = [
    ("he_1s_expo_4k", {}),
    ("he_1s_pade_1m", {}),
    ("he_1s_pade_1m", {"noise": "pm1"}),
    ("he_1s_pade_1m", {"contract": 2}),
    ("he_1s_pade_1m", {"quad": "right"}),
    ("he_2tripS_4m", {"dt": 0.005}),
    ("he_2P_pz_16m", {"dt": 0.005}),
    ("he_2P_pz_16m", {"dt": 0.005, "sym": -1, "theta": [2.0, 0.3, 0.25, 0.5], "noise": "pm1"}),
    ("hydrogen", {}),
    ("he_2tripS_fn3_1m", {"precision": "fp64"}),
    ("he_2tripS_fn3_1m", {"precision": "fp64", "drift_limit": 1.0}),
    ("he_2tripS_fn5_1m", {"precision": "fp64", "noise": "gauss", "contract": 2, "quad": "trapezoid"}),
    ("he_1s_pade_1m", {"plain": True}),
    ("he_2tripS_4m", {"dt": 0.005, "plain": True}),
    ("he_2tripS_4m", {"dt": 0.005, "bridge": True}),
    ("he_2tripS_4m", {"dt": 0.005, "plain": True, "bridge": True, "noise": "pm1"}),
    ("he_2P_pz_16m", {"dt": 0.005, "bridge": True}),
    ("he_2tripS_fn5_1m", {"precision": "fp64", "bridge": True}),
    ("he_2P_fn7_1m", {"precision": "fp64", "n_metropolis": 300}),
    ("he_2P_fn7_1m", {"precision": "fp64", "n_metropolis": 300, "noise": "gauss", "dt": 0.002, "bridge": True}),
]


@pytest.mark.parametrize("name,over", HOST_CASES, ids=lambda v: str(v))
def test_kernel_arithmetic_host_build_matches_oracle(name, over):
    # 1e-12 per walker; for a trial with a node, the one walker whose path came closest to the
    # node may reach 1e-10: there one Euler step multiplies a rounding difference of the two
    # sides' elementary functions by about dt/d^2 (d the node distance), as on the GPU
    cfg = W.get(name, **over)
    ids = np.arange(48) * 13 + 1
    h = host_run(cfg, ids, 300, 20)
    r = oracle.run(cfg, ids, 300, 20)
    assert np.abs(h["x0"] - r["x0"]).max() < 1e-13
    assert np.array_equal(np.isfinite(h["lnw"]), np.isfinite(r["lnw"]))
    f = np.isfinite(r["ell"])
    assert np.array_equal(f, np.isfinite(h["ell"]))
    alive = np.isfinite(r["lnw"])
    err = np.where(f, np.abs(np.where(f, h["ell"] - r["ell"], 0.0)), 0.0).max(axis=1)
    err = np.maximum(err, np.where(alive, np.abs(h["x"] - r["x"]).max(axis=1), 0.0))
    if cfg["trial"] in ("triplet", "pz", "triplet_r0", "pz_sum"):
        closest = int(np.argmin(r["node_dmin"]))
        assert err[closest] < 1e-10, err[closest]
        err[closest] = 0.0
    assert err.max() < 1e-12, (err.max(), ids[int(np.argmax(err))])


# --------------------------------------------------------------------------
# Host build of the gradient's reverse sweep against the oracle's
# complex-step derivative (two independent methods for the same quantity).
# --------------------------------------------------------------------------

@pytest.mark.parametrize("over,ckpt_every", [({}, 50), ({}, 25), ({}, 1), ({"quad": "right"}, 50),
                                             ({"quad": "right"}, 1), ({"trial": "expo", "theta": [1.8]}, 50),
                                             ({"contract": 2}, 100)])
def test_reverse_sweep_host_build_matches_complex_step(over, ckpt_every):
    cfg = W.get("he_1s_pade_grad_256k", n_steps=200, sample_every=50, **over)
    ids = np.arange(192) * 31 + 5
    r = oracle.run(cfg, ids, 200, 50)
    gL = np.array([0.0, 0.3, -0.7, 1.1, -0.5])
    a = adjoint_host_run(cfg, ids, 200, 50, ckpt_every, r["samples"], gL)
    got = a[:, :2].sum(axis=0)
    ref = oracle.grad_objective(cfg, ids, r["x0"], 200, 50, gL)
    for d in range(2):
        assert abs(got[d] - ref[d]) <= 1e-11 * max(abs(ref[d]), 1e-3)
    # P = sum_s g_s p_is sums to sum_s g_s over walkers
    assert abs(a[:, 2].sum() - gL.sum()) < 1e-12
    # with weights on ln <w^2> as well
    gL2 = np.array([0.0, 0.5, 0.0, -0.8, 1.2])
    a = adjoint_host_run(cfg, ids, 200, 50, ckpt_every, r["samples"], gL, gL2)
    got = a[:, :2].sum(axis=0)
    ref = oracle.grad_objective(cfg, ids, r["x0"], 200, 50, gL, gL2=gL2)
    for d in range(2):
        assert abs(got[d] - ref[d]) <= 1e-11 * max(abs(ref[d]), 1e-3)
    assert abs(a[:, 3].sum() - gL2.sum()) < 1e-12                 # the shares q_is sum to one per row
    assert abs(a[:, 2].sum() - gL.sum() - 2 * gL2.sum()) < 1e-12


@pytest.mark.parametrize("over", [{}, {"quad": "right"}, {"trial": "expo", "theta": [1.8]}])
def test_reverse_sweep_over_the_stored_trajectory_equals_the_recomputing_one(over):
    # with a checkpoint at every step the sweep reads the positions instead of recomputing
    # segments; the recomputed positions are the stored ones, so the two agree bitwise
    cfg = W.get("he_1s_pade_grad_256k", n_steps=200, sample_every=50, **over)
    ids = np.arange(64) * 97 + 3
    r = oracle.run(cfg, ids, 200, 50)
    gL = np.array([0.0, 0.3, -0.7, 1.1, -0.5])
    gL2 = np.array([0.0, 0.5, 0.0, -0.8, 1.2])
    direct = adjoint_host_run(cfg, ids, 200, 50, 1, r["samples"], gL, gL2)
    for ce in (50, 10):
        assert np.array_equal(direct, adjoint_host_run(cfg, ids, 200, 50, ce, r["samples"], gL, gL2)), ce


@pytest.mark.parametrize("over", [{}, {"quad": "right"}, {"trial": "expo", "theta": [1.8]}])
@pytest.mark.parametrize("ckpt_every", [1, 50])
def test_reverse_sweep_per_walker_against_the_tangent(over, ckpt_every):
    # the dot-product test, walker by walker: each walker's adjoint gradient (host build of the
    # reverse sweep) against its tangent, sum_s (g_s p_is + 2 g2_s q_is) d l_is / d theta with
    # the oracle's complex-step d l_is / d theta, to 1e-13 of the largest walker term
    cfg = W.get("he_1s_pade_grad_256k", n_steps=200, sample_every=50, **over)
    ids = np.arange(96) * 37 + 11
    r = oracle.run(cfg, ids, 200, 50)
    gL = np.array([0.0, 0.3, -0.7, 1.1, -0.5])
    gL2 = np.array([0.0, 0.5, 0.0, -0.8, 1.2])
    m, s0, s2 = r["samples"][:, 0], r["samples"][:, 1], r["samples"][:, 3]
    p = np.exp(r["ell"] - m) / s0
    q = np.exp(2.0 * (r["ell"] - m)) / s2
    host = adjoint_host_run(cfg, ids, 200, 50, ckpt_every, r["samples"], gL, gL2)
    for d in range(2):
        dl = oracle.dlnw_dtheta(cfg, ids, r["x0"], 200, 50, d)
        ref = (gL * p * dl).sum(axis=1) + (gL2 * 2.0 * q * dl).sum(axis=1)
        assert np.abs(host[:, d] - ref).max() <= 1e-13 * np.abs(ref).max(), d


def test_binary64_step_functions_against_the_c_library():
    # host build of the binary64 elementary functions of the step (series and Newton
    # forms written for its argument ranges): errors in units of the last place over
    # 2e6 arguments each, and the special values the step relies on
    import shutil
    import subprocess
    import tempfile
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    exe = os.path.join(tempfile.mkdtemp(prefix="hefk_f64_"), "f64math_host_check")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    subprocess.check_call([hipcc, "-O2", "-std=c++17", "--offload-arch=gfx950", "-I",
                           os.path.join(root, "paper_1703_08977_amd", "csrc"), "-o", exe,
                           os.path.join(root, "tests", "f64math_host_check.cpp")],
                          stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
    out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split("\n")
    err = dict(zip(out[0].split()[0::2], map(float, out[0].split()[1::2])))
    assert err["log"] <= 2.5 and err["exp"] <= 1.5 and err["sqrt"] <= 1.0 and err["rcp"] <= 1.0, err
    assert err["sin"] <= 2.0 and err["cos"] <= 2.0, err   # absolute, in units of 2^-53
    assert err["expm1"] <= 2.0 and err["same"] == 1.0, err
    assert err["expm1f"] < 3e-7, err  # binary32: a few units of 2^-24 relative
    assert err["dist"] <= 1.0 and err["idist"] <= 1.5, err
    assert out[1].split()[1:] == ["-inf", "0", "inf", "0", "0", "-1"]


def test_bench_reports_committed_traffic_only_for_the_profiled_configuration():
    import importlib.util
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(root, "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    assert len(bench.source_digest()) == 64
    # another workload, or the same one at another precision, never inherits the profiled bytes
    assert bench.committed_traffic(W.get("he_2P_pz_16m", precision="fp64")) is None
    assert bench.committed_traffic(W.get("he_2tripS_4m")) is None
    t = bench.committed_traffic(W.get("he_2P_pz_16m"))
    assert t is None or 1e9 < t < 1e10


def test_source_digest_ignores_comments_and_layout_only():
    import importlib.util
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    spec = importlib.util.spec_from_file_location("bench_mod2", os.path.join(root, "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    tok = bench._code_tokens
    base = 'int f(int a) {\n  return a * 2; // double it\n}\nconst char* s = "a // b";\n'
    # comments (line and block) and whitespace runs do not count
    assert tok(base) == tok('int f(int a) { /* note */ return a * 2;\n\n}\nconst char* s = "a // b";')
    # a comment marker inside a string or character literal is code
    assert '"a // b"' in tok(base)
    assert tok("char c = '/'; int x;") == "char c = '/'; int x;"
    assert tok('const char* q = "\\"/*\\""; int y;').endswith("int y;")
    # any change to the code does
    assert tok(base) != tok(base.replace("a * 2", "a * 3"))
    assert tok(base) != tok(base.replace('"a // b"', '"a //  b"'))


def test_bench_cases_cover_every_trial_family_and_both_precisions():
    import importlib.util
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    spec = importlib.util.spec_from_file_location("bench_mod3", os.path.join(root, "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    seen = set()
    for label, name, over, n_steps in bench.CASES:
        cfg = W.get(name, n_steps=n_steps, sample_every=100, **over)
        assert cfg["n_walkers"] == 1 << 24 and n_steps % 100 == 0, label
        seen.add((cfg["trial"], cfg["precision"], bool(cfg.get("plain")), bool(cfg.get("bridge"))))
    trials = {t for t, _, _, _ in seen}
    assert {"pz", "triplet", "triplet_r0", "pade", "pz_sum"} <= trials
    assert {p for _, p, _, _ in seen} == {"mixed", "fp64"}
    # the variant kernels (plain walk, node bridge) are timed in both precisions
    assert any(pl or br for _, p, pl, br in seen if p == "mixed")
    assert any(pl or br for _, p, pl, br in seen if p == "fp64")


_FLOPC = None


def _flop_harness():
    global _FLOPC
    if _FLOPC is None:
        import shutil
        import subprocess
        import tempfile
        hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
        exe = os.path.join(tempfile.mkdtemp(prefix="hefk_flops_"), "flop_count_host_check")
        subprocess.check_call([hipcc, "-O1", "-std=c++17", "--offload-arch=gfx950", "-I",
                               os.path.join(ROOT, "paper_1703_08977_amd", "csrc"), "-I", os.path.join(ROOT, "include"),
                               "-o", exe, os.path.join(ROOT, "tests", "flop_count_host_check.cpp")],
                              stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
        _FLOPC = exe
    return _FLOPC


@pytest.mark.parametrize("name,over", [
    ("he_2P_pz_16m", {}),                                         # the benchmark step
    ("he_2P_pz_16m", dict(drift_limit=0.0, sym=-1, theta=[2.0, 0.3, 0.25, 0.5])),
    ("he_2P_pz_16m", dict(noise="pm1")),
    ("he_2tripS_4m", {}), ("he_2tripS_4m", dict(contract=1)),
    ("he_1s_pade_1m", {}), ("he_1s_pade_1m", dict(contract=2)),
    ("he_1s_expo_4k", dict(contract=2)),
    ("he_2tripS_fn5_1m", {}), ("he_2tripS_fn5_1m", dict(noise="gauss", contract=2)),
    ("he_2P_fn7_1m", {}), ("he_2P_fn7_1m", dict(noise="gauss", contract=2, drift_limit=1.0)),
])
def test_fp32_flop_count_of_the_step_matches_the_counted_host_build(name, over):
    # the term-by-term binary32 FLOP count of the roofline module against the same step's code
    # run on the host on a counting binary32 type
    import subprocess
    from paper_1703_08977_amd import roofline
    cfg = W.get(name, **dict(over, precision="mixed"))
    noise = 2 if cfg.get("noise", "gauss") == "pm1" else (1 if cfg.get("contract", 1) == 2 else 0)
    line = "%d %d %d %d %d %r\n" % (oracle.TRIALS[cfg["trial"]], cfg.get("sym", 1), noise, cfg.get("ee", 1),
                                    1 if cfg.get("drift_limit", 0.0) > 0 else 0, float(cfg["theta"][2]))
    out = subprocess.run([_flop_harness()], input=line, capture_output=True, text=True, check=True).stdout.split()
    flops, trans = int(out[0]), int(out[1])
    assert roofline.fp32_flops_per_walker_step(cfg) == flops
    assert roofline.transcendentals_per_walker_step(cfg) == trans


def test_roofline_class_costs_are_the_committed_calibration():
    # every class cost the roofline charges is the one the committed calibration summary
    # derives from its counters (the lower of the class alone and beside binary32 FMAs)
    from paper_1703_08977_amd import roofline
    with open(os.path.join(ROOT, "profiles", "valu_class_costs.txt")) as f:
        text = f.read()
    seen = set()
    for m in re.finditer(r"^(\w+)\s+beside FMAs\s+([\d.]+)\s+alone\s+([\d.]+)\s+->\s+([\d.]+) cycles = ([\d.]+) slots",
                         text, re.M):
        cls, mix, alone, use, slots = m.group(1), *map(float, m.groups()[1:])
        assert abs(use - min(mix, alone)) < 0.006 and abs(slots - use / 2) < 0.006, m.group(0)
        assert abs(roofline.CLASS_SLOTS[cls] - slots) < 0.006, (cls, roofline.CLASS_SLOTS[cls], slots)
        seen.add(cls)
    assert seen == set(roofline.CLASS_SLOTS) - {"a32"}, seen
    assert roofline.CLASS_SLOTS["a32"] == 1.0  # the published rate: 2 SIMD-cycles per wave64 instruction
