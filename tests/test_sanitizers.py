"""Sanitizer builds of the host code (CPU only): the oracle compiled with
AddressSanitizer and UndefinedBehaviorSanitizer into a driver that runs the
4096-walker ground state in full, ragged ensembles of every trial with every
noise, quadrature and variant, and the complex-step gradient; and the host
builds of the kernels' per-walker code (step and reverse sweep) with the same
sanitizers on their host side, run over trial, noise and variant cases in both
precisions; and a replay of the kernels' loop nests whose every array index goes
through the kernels' own layout functions, checked against the host allocation
sizes.  Any report ends the program with a nonzero status."""
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

import oracle
from paper_1703_08977_amd import workloads as W

import hefk_testutil as T

SAN_HOST = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=all"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")


def _hipcc():
    return shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


def test_oracle_under_address_and_undefined_behaviour_sanitizers():
    exe = os.path.join(tempfile.mkdtemp(prefix="hefk_osan_"), "oracle_sanitize")
    subprocess.check_call(["gcc", "-O1", "-g", "-std=c11", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                           "-fno-omit-frame-pointer", "-o", exe, os.path.join(T.ROOT, "tests", "oracle_sanitize_main.c"),
                           "-lm"], stderr=subprocess.DEVNULL)
    r = subprocess.run([exe], capture_output=True, text=True, env=ENV)
    assert r.returncode == 0 and "runtime error" not in r.stderr and "ERROR" not in r.stderr, r.stderr[-3000:]
    assert np.isfinite(float(r.stdout.split()[0]))


@pytest.fixture(scope="module")
def sanitized_step():
    exe = os.path.join(tempfile.mkdtemp(prefix="hefk_dsan_"), "device_code_host_check")
    subprocess.check_call([_hipcc(), "-O1", "-g", "-std=c++17", "--offload-arch=gfx950"] + SAN_HOST +
                          ["-I", T.CSRC, "-I", os.path.join(T.ROOT, "include"), "-o", exe,
                           os.path.join(T.ROOT, "tests", "device_code_host_check.cpp")],
                          stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
    return exe


@pytest.mark.parametrize("name,over", [
    ("he_1s_expo_4k", {}), ("he_1s_pade_1m", {"noise": "pm1", "quad": "right"}),
    ("he_2tripS_4m", {"dt": 0.005, "plain": True, "bridge": True}),
    ("he_2P_pz_16m", {"dt": 0.005, "contract": 2}), ("he_2tripS_fn3_1m", {"drift_limit": 1.0}),
    ("he_2P_fn7_1m", {"n_metropolis": 300, "bridge": True}),
], ids=lambda v: str(v))
@pytest.mark.parametrize("precision", [0, 1])
def test_kernel_step_host_build_under_sanitizers(sanitized_step, name, over, precision):
    # the sanitized host build of the per-walker step gives the same walkers as the plain host build
    cfg = W.get(name, **dict(over, precision="fp64"))
    ids = np.arange(0, 600, 7)
    saved = T._HARNESS
    try:
        T._HARNESS = sanitized_step
        s = T.host_run(cfg, ids, 120, 20, precision=precision)
    finally:
        T._HARNESS = saved
    p = T.host_run(cfg, ids, 120, 20, precision=precision)
    for k in ("x0", "x", "lnw", "ell"):
        assert np.array_equal(s[k], p[k], equal_nan=True), k


def test_reverse_sweep_host_build_under_sanitizers():
    exe = os.path.join(tempfile.mkdtemp(prefix="hefk_asan_"), "adjoint_host_check")
    subprocess.check_call([_hipcc(), "-O1", "-g", "-std=c++17", "--offload-arch=gfx950"] + SAN_HOST +
                          ["-I", T.CSRC, "-I", os.path.join(T.ROOT, "include"), "-o", exe,
                           os.path.join(T.ROOT, "tests", "adjoint_host_check.cpp")],
                          stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
    cfg = W.get("he_1s_pade_grad_256k")
    ids = np.arange(40)
    r = oracle.run(cfg, ids, 200, 50)
    gL = np.zeros(len(r["samples"]))
    gL[-1], gL[-2] = -10.0, 10.0
    for ce in (50, 1):  # the recomputing sweep and the one over the stored trajectory
        saved = T._ADJ
        try:
            T._ADJ = exe
            s = T.adjoint_host_run(cfg, ids, 200, 50, ce, r["samples"], gL)
        finally:
            T._ADJ = saved
        p = T.adjoint_host_run(cfg, ids, 200, 50, ce, r["samples"], gL)
        assert np.array_equal(s, p), ce


def _layout_cases():
    """Configurations of the host replay of the kernels' loop nests: walker counts with
    ragged tails, resident block counts from 1 to more than the chunks, sampling and
    checkpoint spacings, partial rows in LDS (when they fit, as the launcher decides) or in
    the workspace; and the full sizes of the mixed P_z bench step (2^24 walkers, 1536
    resident blocks: the grid of 1525 the profiles show) and of the gradient workload's
    trajectory at a reduced walker count."""
    cases = []
    for n in (1, 255, 256, 257, 3001, 65541):
        for res in (1, 7, 1536, 6100):
            for steps, se, ce in ((300, 100, 0), (200, 50, 1), (200, 50, 25), (300, 1, 0), (1000, 50, 50)):
                ns = steps // se + 1
                cases.append((n, res, steps, se, ce, int(ns * 64 <= 16384)))
    cases.append((1 << 24, 1536, 12000, 100, 0, 1))
    cases.append((4099, 3072, 1000, 50, 1, 1))
    return cases


@pytest.fixture(scope="module")
def layout_check():
    exe = os.path.join(tempfile.mkdtemp(prefix="hefk_layout_"), "layout_host_check")
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                           "-I", T.CSRC, "-o", exe, os.path.join(T.ROOT, "tests", "layout_host_check.cpp")])
    return exe


def test_kernel_index_arithmetic_replayed_under_sanitizers(layout_check):
    # every index of init, propagate, merge and the gradient sweeps through the kernels' own
    # layout functions, checked against the host allocation sizes; each walker's state and
    # each checkpoint entry written exactly once, each chunk visited once
    cases = _layout_cases()
    stdin = "".join("%d %d %d %d %d %d\n" % c for c in cases)
    r = subprocess.run([layout_check], input=stdin, capture_output=True, text=True, env=ENV)
    out = r.stdout.split("\n")
    assert r.returncode == 0 and "runtime error" not in r.stderr and "ERROR" not in r.stderr, (r.stdout[-2000:],
                                                                                                r.stderr[-2000:])
    assert sum(1 for line in out if line.startswith("ok")) == len(cases)
    assert out[len(cases) - 2] == "ok grid=1525"


def test_kernel_index_replay_catches_a_short_array(layout_check):
    # the same replay with the checkpoint array one element short must report the access
    r = subprocess.run([layout_check], input="257 7 200 50 25 1\n", capture_output=True, text=True,
                       env=dict(ENV, HEFK_LAYOUT_SHORT="1"))
    assert r.returncode == 1 and "outside" in r.stdout and "ckpt" in r.stdout, r.stdout
