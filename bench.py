#!/usr/bin/env python3
"""Benchmark: He walker-steps/s on one MI355X, mixed (FP32 step, FP64 ln w and
reductions) against all-FP64, and the time to a 1e-5 Ha statistical error.

A step is one pass of the whole path over one seed of the workload: start
ensemble (Metropolis), propagation over all n_steps with the log-domain space
average at every sampling time, sample rows back to the host, energy
estimators.  value = n_walkers * n_steps / (wall time of one step).

Default workload: the 2^1P (P_z) trial, 2^24 walkers, dt = 0.0005, T = 6
(12000 steps), sampled every 100 steps.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=4)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="he_2P_pz_16m")
    ap.add_argument("--precision", default=None, help="override the workload's precision")
    ap.add_argument("--noise", default=None)
    ap.add_argument("--contract", type=int, default=None)
    ap.add_argument("--fp64-steps", type=int, default=4,
                    help="timed FP64 steps on the first seeds of the mixed leg, for the speedup and the paired "
                         "mixed - FP64 energy difference (0: skip)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-walkers", type=int, default=0,
                    help="walkers of the oracle's timed sample (0: 131072 of the bench workload, about 13 s on 16 "
                         "host threads; grad mode: the whole 2^18-walker gradient workload, about 11 s)")
    ap.add_argument("--grad-walkers", type=int, default=0,
                    help="grad mode: walkers of the gradient workload (0: its own 2^18)")
    ap.add_argument("--oracle-threads", type=int, default=0, help="oracle mode: thread count (0: all)")
    ap.add_argument("--mode", default="bench", choices=["bench", "copy", "oracle", "grad", "cases"],
                    help="copy: a plain 1 GiB device copy, three times after a warm-up (the reference reading of the HBM "
                         "byte counters FETCH_SIZE / WRITE_SIZE), then three sums over 8 GiB (a read-only "
                         "stream), with the rates both reach; oracle: time the CPU oracle alone on the "
                         "4096-walker ground state in full and on walkers 0..65535 of the Pade ground state "
                         "at dt = 0.002; grad: the pathwise gradient of E(T = 2) for the Pade-Jastrow trial, "
                         "2^18 walkers x 1000 steps (forward storing the trajectory, then he_fk_grad reading it back), with the "
                         "oracle's gradient timed beside it; cases: propagate throughput of the other "
                         "trials, noises, precisions and the variant kernels (plain walk, node bridge) "
                         "at 2^24 walkers")
    return ap.parse_args()


def copy_reference():
    """Three plain 1 GiB device copies (the reading of the byte counters), then three sums over
    8 GiB (a read-only stream): the HBM rates these plain kernels reach, timed with events after
    one untimed call of each."""
    import torch
    nbytes = 1 << 30
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)  # warm-up
    copy_rate = []
    for _ in range(3):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        copy_rate.append(2 * nbytes / (e0.elapsed_time(e1) * 1e-3) / 1e12)
    del src, dst
    rbytes = 8 << 30
    big = torch.ones(rbytes // 8, dtype=torch.float64, device="cuda")
    total = big.sum()  # warm-up
    read_rate = []
    for _ in range(3):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        total = big.sum()
        e1.record()
        torch.cuda.synchronize()
        read_rate.append(rbytes / (e0.elapsed_time(e1) * 1e-3) / 1e12)
    assert float(total) == rbytes // 8
    print(json.dumps({"mode": "copy", "bytes_per_copy": nbytes, "copies": 3, "copy_TB_per_s": copy_rate,
                      "read_bytes": rbytes, "read_TB_per_s": read_rate}), flush=True)


def run_leg(cfg, n_steps_timed, n_warmup, seeds):
    """Time full steps; returns per-step wall times, kernel times, energies, block errors."""
    import torch
    from paper_1703_08977_amd import Ensemble, he_fk_energy
    from paper_1703_08977_amd.stats import jackknife

    ens = Ensemble(cfg)
    ns = cfg["n_steps"] // cfg["sample_every"] + 1
    samples = torch.empty((ns, 8), dtype=torch.float64, device="cuda")
    ens.workspace(cfg["n_steps"], cfg["sample_every"])
    dts = cfg["dt"] * cfg["sample_every"]
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def one(seed):
        ens.p.seed = seed
        ens.init()
        ev0.record()
        ens.propagate(0, cfg["n_steps"], cfg["sample_every"], samples=samples)
        ev1.record()
        host = samples.cpu().numpy()  # synchronises the stream
        e_win = he_fk_energy(host, dts, cfg["e_ref"], "window")[0][0]
        return host, e_win

    for i in range(n_warmup):
        one(10_000 + i)
        print("# warmup %d done (%s)" % (i, cfg["precision"]), file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    walls, kern, energies, errs = [], [], [], []
    for i in range(n_steps_timed):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        host, e_win = one(seeds[i])
        torch.cuda.synchronize()
        walls.append(time.perf_counter() - t0)
        kern.append(ev0.elapsed_time(ev1) / 1e3)
        rows = ens.block_rows(cfg["n_steps"], cfg["sample_every"]).cpu().numpy()
        e_jk, s_jk = jackknife(rows, dts, cfg["e_ref"], "window")
        energies.append(e_win)
        errs.append(s_jk)
        print("# step %d (%s): wall %.3f s, propagate %.3f s, E_win %.7f +- %.7f" %
              (i, cfg["precision"], walls[-1], kern[-1], e_win, s_jk), file=sys.stderr, flush=True)
    del ens
    torch.cuda.empty_cache()
    return dict(walls=walls, kern=kern, energies=energies, errs=errs)


KERNEL_SOURCES = ["include/he_fk.h", "paper_1703_08977_amd/csrc/hefk_device.hpp",
                  "paper_1703_08977_amd/csrc/hefk_f64math.hpp", "paper_1703_08977_amd/csrc/hefk_reduce.hpp",
                  "paper_1703_08977_amd/csrc/hefk_kernels.hip", "paper_1703_08977_amd/csrc/build.py"]
COUNTERS = os.path.join(ROOT, "profiles", "propagate_pz_16m_counters.txt")


def _code_tokens(text: str) -> str:
    """C/C++ source with comments removed and each run of whitespace folded to one
    space: edits to comments or layout leave the compiled kernel, and so the digest, as
    they were.  String and character literals are kept verbatim."""
    out, i, n = [], 0, len(text)
    while i < n:
        c = text[i]
        if text.startswith("//", i):
            j = text.find("\n", i)
            i = n if j < 0 else j
            c = " "
        elif text.startswith("/*", i):
            j = text.find("*/", i + 2)
            i = n if j < 0 else j + 2
            c = " "
        elif c in "\"'":
            j = i + 1
            while j < n and text[j] != c:
                j += 2 if text[j] == "\\" else 1
            out.append(text[i:j + 1])
            i = j + 1
            continue
        else:
            i += 1
        if not c.isspace():
            out.append(c)
        elif out and out[-1] != " ":
            out.append(" ")
    return "".join(out).strip()


def source_digest() -> str:
    """sha256 over the code of the propagate kernel's sources (comments and layout
    excluded) and its build script (verbatim: it holds the compiler flags)."""
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), encoding="utf-8") as f:
            text = f.read()
        body = text if rel.endswith(".py") else _code_tokens(text)
        h.update(rel.encode() + b"\0" + body.encode())
    return h.hexdigest()


def config_key(cfg) -> str:
    keys = ("name", "trial", "sym", "n_walkers", "n_steps", "sample_every", "precision", "noise", "contract")
    return " ".join("%s=%s" % (k, cfg.get(k)) for k in keys)


def committed_traffic(cfg):
    """HBM bytes per propagate launch from the committed counter summary (FETCH_SIZE and
    WRITE_SIZE, scaled by a plain copy's reading), if it was taken on these kernel sources
    and this configuration; otherwise None."""
    try:
        with open(COUNTERS) as f:
            kv = dict(ln.split(":", 1) for ln in f.read().splitlines() if ln.startswith("traffic_"))
    except (OSError, ValueError):
        return None
    kv = {k.strip(): v.strip() for k, v in kv.items()}
    if kv.get("traffic_source_digest") != source_digest() or kv.get("traffic_config") != config_key(cfg):
        return None
    return float(kv["traffic_bytes_per_launch"])


def cpu_baseline(cfg, n_walkers):
    """The oracle (FP64, OpenMP) on a bounded sample of the same workload."""
    import numpy as np
    import oracle
    ids = np.arange(n_walkers)
    c = dict(cfg, precision="fp64")
    t0 = time.perf_counter()
    x, _ = oracle.init(c, ids)
    t1 = time.perf_counter()
    oracle.propagate(c, ids, x, np.zeros(n_walkers), 0, cfg["n_steps"], cfg["sample_every"], record=False)
    t2 = time.perf_counter()
    ws = n_walkers * cfg["n_steps"]
    return {"value": ws / (t2 - t0), "unit": "walker-steps/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": "walker ids 0..%d of the workload, all %d steps, start ensemble included "
                      "(start %.2f s, propagation %.2f s, propagation-only %.4g walker-steps/s); host CPU: %s" %
                      (n_walkers - 1, cfg["n_steps"], t1 - t0, t2 - t1, ws / (t2 - t1), cpu_model())}


def oracle_timing(threads=0):
    """Walker-steps/s of the CPU oracle (start ensemble timed apart) on two workloads."""
    import numpy as np
    import oracle
    from paper_1703_08977_amd import workloads as W
    if threads > 0:
        oracle.set_num_threads(threads)
    out = {"mode": "oracle", "threads": oracle.num_threads(), "cpu": cpu_model(), "runs": []}
    for name, n in (("he_1s_expo_4k", 4096), ("he_1s_pade_1m", 1 << 16)):
        cfg = W.get(name, dt=0.002) if name == "he_1s_pade_1m" else W.get(name)
        ids = np.arange(n)
        t0 = time.perf_counter()
        x, _ = oracle.init(cfg, ids)
        t1 = time.perf_counter()
        oracle.propagate(cfg, ids, x, np.zeros(n), 0, cfg["n_steps"], cfg["sample_every"], record=False)
        t2 = time.perf_counter()
        out["runs"].append({"workload": name, "walkers": n, "steps": cfg["n_steps"], "start_s": t1 - t0,
                            "propagate_s": t2 - t1, "walker_steps_per_s": n * cfg["n_steps"] / (t2 - t1)})
    print(json.dumps(out), flush=True)


def grad_bench(n_timed, n_warmup, cpu_walkers, no_cpu, n_walkers=0):
    """Forward propagation storing the trajectory (a checkpoint at every step), then the
    reverse sweep (he_fk_grad) over it, of
    dE(T)/d(alpha, beta), E(T) = e_ref - (L(T) - L(T - ds)) / ds, score term included."""
    import numpy as np
    import torch
    from paper_1703_08977_amd import Ensemble, _lib, api
    from paper_1703_08977_amd import workloads as W
    from paper_1703_08977_amd.roofline import (PEAK_SLOTS_PER_S, grad_slots_per_walker_step,
                                               grad_tape_bytes_per_walker_step)
    cfg = W.get("he_1s_pade_grad_256k", **({"n_walkers": n_walkers} if n_walkers else {}))
    n, K, se, ce = cfg["n_walkers"], cfg["n_steps"], cfg["sample_every"], cfg["ckpt_every"]
    ns = K // se + 1
    dts = cfg["dt"] * se
    ens = Ensemble(cfg)
    samples = torch.empty((ns, 8), dtype=torch.float64, device="cuda")
    ckpt = torch.empty((K // ce + 1, 7, n), dtype=torch.float64, device="cuda")
    ens.workspace(K, se)
    nb = api.he_fk_grad_scratch_bytes(ens.p, K, se, ce)
    scratch = torch.empty(nb, dtype=torch.uint8, device="cuda")
    dtheta = torch.empty(2, dtype=torch.float64, device="cuda")
    g = np.zeros(ns)
    g[-1], g[-2] = -1.0 / dts, 1.0 / dts
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    fwd, bwd, grads = [], [], []
    for i in range(n_warmup + n_timed):
        ens.p.seed = i
        ens.init()
        ev[0].record()
        ens.propagate(0, K, se, samples=samples, ckpt=ckpt, ckpt_every=ce)
        ev[1].record()
        api.he_fk_grad(ens.p, ckpt.data_ptr(), samples.data_ptr(), g, K, se, ce, _lib.GRAD_SCORE,
                       scratch.data_ptr(), nb, dtheta.data_ptr())
        ev[2].record()
        torch.cuda.synchronize()
        if i >= n_warmup:
            fwd.append(ev[0].elapsed_time(ev[1]) / 1e3)
            bwd.append(ev[1].elapsed_time(ev[2]) / 1e3)
            grads.append(dtheta.cpu().tolist())
    tf, tb = sum(fwd) / len(fwd), sum(bwd) / len(bwd)
    slots = grad_slots_per_walker_step(cfg)
    tape = grad_tape_bytes_per_walker_step(cfg)
    ach = slots * n * K / tb / 1e12
    gbs = tape * n * K / tb / 1e9
    # the bound is the resource the kernel's algorithmic work needs longest on at peak rates
    hbm_bound = tape / 8e12 > slots / PEAK_SLOTS_PER_S
    if hbm_bound:
        roof = {"bound": "hbm", "achieved": gbs, "peak": 8000.0, "unit": "GB/s", "frac": gbs / 8000.0,
                "valu_slots_per_walker_step": slots, "valu_Tslot_per_s": ach,
                "valu_frac": ach / (PEAK_SLOTS_PER_S / 1e12)}
    else:
        roof = {"bound": "alu", "achieved": ach, "peak": PEAK_SLOTS_PER_S / 1e12, "unit": "Tslot/s",
                "frac": ach / (PEAK_SLOTS_PER_S / 1e12), "slots_per_walker_step": slots,
                "tape_GB_per_s": gbs, "tape_frac_of_8TB_s": gbs / 8000.0}
    roof["kernel"] = ("he_fk_grad (reverse sweep over the stored trajectory)" if ce == 1 else
                      "he_fk_grad (recompute + reverse sweep)")
    roof["tape_bytes_per_walker_step"] = tape
    out = {"mode": "grad", "workload": cfg["name"], "n_walkers": n, "n_steps": K, "ckpt_every": ce,
           "precision": "fp64", "objective": "E(T = 2) by finite differences of L over the last sample "
                                            "interval, start-law score term included",
           "forward_ms": tf * 1e3, "grad_ms": tb * 1e3,
           "grad_walker_steps_per_s": n * K / tb, "forward_and_grad_walker_steps_per_s": n * K / (tf + tb),
           "dE_dtheta": grads, "roofline": roof}
    if not no_cpu:
        import oracle
        cpu_walkers = cpu_walkers or n
        ids = np.arange(cpu_walkers)
        t0 = time.perf_counter()
        y0, _ = oracle.init(cfg, ids)
        t1 = time.perf_counter()
        oracle.grad_objective(cfg, ids, y0, K, se, g, score=True)
        t2 = time.perf_counter()
        out["cpu_baseline"] = {"value": cpu_walkers * K / (t2 - t1), "unit": "walker-steps/s (gradient)",
                               "cores": oracle.num_threads(), "kind": "oracle",
                               "sample": "walker ids 0..%d, all %d steps: forward pass and the complex-step "
                                         "derivative in each of the two directions (start ensemble %.2f s "
                                         "apart); host CPU: %s" % (cpu_walkers - 1, K, t1 - t0, cpu_model())}
    print(json.dumps(out), flush=True)


# (label, workload, overrides, timed steps): every propagate kernel family at 2^24 walkers
CASES = [
    ("P_z, mixed", "he_2P_pz_16m", {}, 4000),
    ("P_z, FP64", "he_2P_pz_16m", {"precision": "fp64"}, 2000),
    ("P_z, +-1 walk, mixed", "he_2P_pz_16m", {"noise": "pm1"}, 4000),
    ("triplet, mixed", "he_2tripS_4m", {"n_walkers": 1 << 24}, 4000),
    ("triplet, FP64", "he_2tripS_4m", {"n_walkers": 1 << 24, "precision": "fp64"}, 2000),
    ("fn 5 (+-1 walk, right end-point sum), mixed", "he_2tripS_fn5_1m", {"n_walkers": 1 << 24}, 4000),
    ("Pade-Jastrow, FP64", "he_1s_pade_1m", {"n_walkers": 1 << 24, "dt": 0.002}, 2000),
    ("Pade-Jastrow, plain walk, mixed", "he_1s_pade_1m",
     {"n_walkers": 1 << 24, "dt": 0.002, "plain": True, "precision": "mixed", "contract": 2}, 2000),
    ("P_z + bridge, mixed", "he_2P_pz_16m", {"bridge": True}, 2000),
    ("triplet + bridge, mixed", "he_2tripS_4m", {"n_walkers": 1 << 24, "bridge": True}, 2000),
    ("fn 7 + bridge, plain walk, mixed", "he_2P_fn7_1m", {"n_walkers": 1 << 24, "bridge": True, "plain": True},
     2000),
    ("P_z + bridge, FP64", "he_2P_pz_16m", {"bridge": True, "precision": "fp64"}, 1000),
    ("triplet + bridge, FP64", "he_2tripS_4m", {"n_walkers": 1 << 24, "bridge": True, "precision": "fp64"}, 1000),
    ("fn 7 + bridge, plain walk, FP64", "he_2P_fn7_1m",
     {"n_walkers": 1 << 24, "bridge": True, "plain": True, "precision": "fp64"}, 1000),
]


def cases_bench(reps):
    """Propagate throughput per kernel family: start ensemble, 200 untimed steps, then
    `reps` timed propagations of each case's step count (HIP events on the launch
    stream), sampling every 100 steps; the median rate is reported."""
    import torch
    from paper_1703_08977_amd import Ensemble
    from paper_1703_08977_amd import workloads as W
    rows = []
    for label, name, over, n_steps in CASES:
        cfg = W.get(name, n_steps=n_steps, sample_every=100, **over)
        ens = Ensemble(cfg).init()
        ens.propagate(0, 200, 100)
        rates = []
        for _ in range(max(1, reps)):
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
            ev[0].record()
            ens.propagate(0, n_steps, 100)
            ev[1].record()
            torch.cuda.synchronize()
            rates.append(cfg["n_walkers"] * n_steps / (ev[0].elapsed_time(ev[1]) / 1e3))
        rates.sort()
        rows.append({"case": label, "workload": name, "n_walkers": cfg["n_walkers"], "n_steps": n_steps,
                     "precision": cfg["precision"], "walker_steps_per_s": rates[len(rates) // 2]})
        print("%-44s %.3e walker-steps/s" % (label, rows[-1]["walker_steps_per_s"]), file=sys.stderr, flush=True)
        del ens
        torch.cuda.empty_cache()
    print(json.dumps({"mode": "cases", "reps": reps, "cases": rows}), flush=True)


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the walkers of this method share nothing but the per-sample "
              "reduction, and this benchmark measures one MI355X (requested --gpus %d)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.mode == "copy":
        copy_reference()
        return
    if args.mode == "oracle":
        oracle_timing(args.oracle_threads)
        return
    if args.mode == "grad":
        grad_bench(args.steps, args.warmup, args.cpu_walkers, args.no_cpu_baseline, args.grad_walkers)
        return
    if args.mode == "cases":
        cases_bench(args.steps)
        return
    import torch
    from paper_1703_08977_amd import workloads as W
    from paper_1703_08977_amd.roofline import (PEAK_SLOTS_PER_S, class_counts, fp32_flops_per_walker_step,
                                               instructions_per_walker_step, slots_per_walker_step,
                                               transcendentals_per_walker_step)

    over = {}
    if args.precision:
        over["precision"] = args.precision
    if args.noise:
        over["noise"] = args.noise
    if args.contract:
        over["contract"] = args.contract
    cfg = W.get(args.workload, **over)
    n, K = cfg["n_walkers"], cfg["n_steps"]
    seeds = list(range(args.steps))

    main_leg = run_leg(cfg, args.steps, args.warmup, seeds)
    wall = sum(main_leg["walls"]) / len(main_leg["walls"])
    kern = sum(main_leg["kern"]) / len(main_leg["kern"])
    value = n * K / wall

    slots = slots_per_walker_step(cfg)
    achieved = slots * n * K / kern / 1e12
    peak = PEAK_SLOTS_PER_S / 1e12
    roof = {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "Tslot/s", "frac": achieved / peak,
            "frac_is": "VALU issue utilisation: the step's formula-counted instructions, each class at its "
                       "issue cost measured on this GPU (slots of 2 SIMD-cycles per wave64 instruction: "
                       "binary32 and 32-bit integer 1, binary64 2.1, binary32 transcendental 4.1, ...), per "
                       "second, over 256 CU x 4 SIMD x 32 lanes x 2.4 GHz (the 157.3 TFLOP/s binary32 "
                       "rate in fused multiply-adds)",
            "traffic": committed_traffic(cfg), "kernel": "propagate_kernel", "slots_per_walker_step": slots,
            "instructions_by_class": class_counts(cfg),
            "transcendentals_per_walker_step": transcendentals_per_walker_step(cfg),
            "valu_instructions_per_walker_step": instructions_per_walker_step(cfg), "kernel_ms": kern * 1e3}
    fl = fp32_flops_per_walker_step(cfg)
    if fl:
        roof["fp32_flops_per_walker_step"] = fl
        roof["fp32_tflops"] = fl * n * K / kern / 1e12
        roof["fp32_flop_frac_of_157.3"] = roof["fp32_tflops"] / 157.3

    out = {
        "metric": "He walker-steps/s/GPU; mixed FP32 vs FP64 time-to-1e-5 Ha energy error",
        "value": value, "unit": "walker-steps/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": wall * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64" if cfg["precision"] == "mixed" else "f64", "data": "synthetic",
        "config": {"workload": cfg["name"], "trial": cfg["trial"], "sym": cfg.get("sym", 1),
                   "theta": cfg["theta"], "n_walkers": n, "n_steps": K, "dt": cfg["dt"], "T": K * cfg["dt"],
                   "sample_every": cfg["sample_every"], "precision": cfg["precision"],
                   "noise": cfg["noise"], "contract": cfg["contract"], "quad": cfg["quad"],
                   "drift_limit": cfg.get("drift_limit", 0.0), "plain": bool(cfg.get("plain", False)),
                   "bridge": bool(cfg.get("bridge", False)), "n_metropolis": cfg["n_metropolis"],
                   "seeds": seeds},
        "propagate_walker_steps_per_s": n * K / kern,
        "roofline": roof,
        "energy": {"E_window": main_leg["energies"], "jackknife_se": main_leg["errs"]},
    }

    if args.fp64_steps > 0 and cfg["precision"] == "mixed":
        c64 = dict(cfg, precision="fp64")
        n64 = min(args.fp64_steps, args.steps)
        leg = run_leg(c64, n64, 0, seeds[:n64])
        w64 = sum(leg["walls"]) / len(leg["walls"])
        k64 = sum(leg["kern"]) / len(leg["kern"])
        s64 = slots_per_walker_step(c64)
        out["fp64"] = {"value": n * K / w64, "ms_per_step": w64 * 1e3, "propagate_walker_steps_per_s": n * K / k64,
                       "E_window": leg["energies"], "jackknife_se": leg["errs"],
                       "slots_per_walker_step": s64, "instructions_by_class": class_counts(c64),
                       "roofline_frac": s64 * n * K / k64 / PEAK_SLOTS_PER_S}
        out["speedup_mixed_vs_fp64"] = w64 / wall
        # paired mixed - FP64 difference on identical seeds, and the time to a 1e-5 Ha standard error
        m = len(leg["energies"])
        d = [main_leg["energies"][i] - leg["energies"][i] for i in range(m)]
        bias = sum(d) / m
        bias_se = math.sqrt(sum((x - bias) ** 2 for x in d) / (m - 1) / m) if m > 1 else None
        eps = 1e-5
        s_mix = sum(main_leg["errs"]) / len(main_leg["errs"])
        s_64 = sum(leg["errs"]) / m
        # Both precisions draw identical increments from the same start, and their energies differ by
        # the paired bias only (~1e-8 Ha), so they have one sampling error.  The two jackknife
        # estimates differ only through the block grouping (grid sizes differ), so both use the
        # pooled estimate.
        errs = main_leg["errs"] + leg["errs"]
        s_pool = math.sqrt(sum(e * e for e in errs) / len(errs))
        t_mix = wall * s_pool ** 2 / (eps ** 2 - bias ** 2) if abs(bias) < eps else math.inf
        t_64 = w64 * s_pool ** 2 / eps ** 2
        out["time_to_1e-5_Ha"] = {"mixed_s": t_mix, "fp64_s": t_64,
                                  "speedup": (t_64 / t_mix) if math.isfinite(t_mix) else 0.0,
                                  "paired_bias_mixed_minus_fp64": bias, "paired_bias_se": bias_se,
                                  "paired_seeds": m, "sigma_pooled": s_pool,
                                  "sigma_mixed_jackknife": s_mix, "sigma_fp64_jackknife": s_64,
                                  "note": "statistical error only (the time-step bias is common to both "
                                          "precisions); one pooled jackknife error for both, as the paired "
                                          "runs share their increments and start ensemble"}

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg, args.cpu_walkers or 131072)
        print("# cpu baseline done", file=sys.stderr, flush=True)
    print(json.dumps(out), flush=True)
    torch.cuda.synchronize()


if __name__ == "__main__":
    main()
