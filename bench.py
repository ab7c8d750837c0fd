#!/usr/bin/env python3
"""Benchmark of the Cahn-Hilliard ensemble hot path on one MI355X.

A "step" is one time step of the whole path for every member of the batch:
the RHS + x-solve pass, the y-solve pass (and z in 3D), and the F / <C> /
dF/dt reductions on cadence steps.  The metric is lattice-site updates per
second (GLUPS = sites x steps / seconds / 1e9) with the state resident in HBM,
FP32-bulk batched ensembles against plain FP64 single grids.

Prints ONE JSON line.  Default workload: the FP32-bulk batched ensemble of
64 x 512^2 grids; the same line carries the plain FP64 single 1024^2 grid and
the FP64 64 x 512^2 ensemble measured the same way ("compare"), the roofline
figures of the dominant kernel and the oracle timed on the host cores.  The
timed steps are replays of a HIP graph captured and uploaded beforehand, or
direct launches: before the warm-up, one untimed trial of each launch mode
over min(steps, 64) steps picks the faster one for the timed region (graph
replays start after a launch latency of about 0.3 ms; direct launches start
at once, but their classes' streams may share hardware queues).

`--workload model1` measures the droplet-population ensembles instead (Model 1
of the paper): the whole table of Section 3 (100 populations for each N =
128 ... 8192, t in [0, 40]) integrated in one run, as live-droplet stage
evaluations per second, with the ensemble statistics of each N beside the
paper's values.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0  # MI355X HBM3E, published
PEAK_FP64_VECTOR_TFLOPS = 78.6  # MI355X FP64 vector, published
# Algorithmic FP64 operations of one live-droplet stage evaluation of the
# Dormand-Prince pair on dV/dt = 3 (ubar R - 1), the cube root not counted:
# stage value y + h sum_j a_sj k_j (4.3 multiply-adds on average over the six
# new stages), rate 3 (ubar R - 1) (3), mean-field sums (2), error sum (2),
# share of the error norm (~1).
DP_FLOPS_PER_EVAL = 17.0
# Table of the paper's Model 1 statistics (Section 3): N -> (beta0 over
# [20, 40], k of mu_2 = k t over [0, 40]).
MODEL1_PAPER = {512: (0.24, 0.0075), 1024: (0.2613, 0.0036), 2048: (0.2833, 0.0017), 4096: (0.2908, 8.6e-4),
                8192: (0.2995, 4.5e-4)}


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=None, help="timed steps (default: the workload's)")
    p.add_argument("--warmup", type=int, default=100)
    p.add_argument("--workload", default="c3")
    p.add_argument("--compare", default="c2,c3_fp64",
                   help="further workloads reported in the same line, comma-separated ('' = none)")
    p.add_argument("--compare-steps", type=int, default=None)
    p.add_argument("--kernel-steps", type=int, default=200,
                   help="real steps after the timed region whose kernels are timed one by one")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-seconds", type=float, default=15.0)
    p.add_argument("--no-autotune", dest="autotune", action="store_false",
                   help="keep the default tile shapes (autotuning reads the cache first)")
    p.add_argument("--tune-cache", default=os.path.join(ROOT, "paper_1911_03386_amd", "tune_cache.txt"))
    p.add_argument("--graph-steps", type=int, default=64, help="steps per captured HIP graph")
    p.add_argument("--dp-attempts", type=int, default=4096, help="model1: step attempts per launch")
    p.add_argument("--model1-ns", default="", help="model1: only these population sizes (comma-separated)")
    p.add_argument("--dp-cpu-t-end", type=float, default=1.0,
                   help="model1: simulated time of the oracle sample (one N = 2048 population)")
    p.add_argument("--copy-calibration", action="store_true",
                   help="only run a plain device copy of known size (for HBM counter calibration)")
    return p.parse_args()


def kernel_source_sha():
    h = hashlib.sha256()
    for f in ("ch_kernels.hip", "ch_internal.h"):
        with open(os.path.join(ROOT, "paper_1911_03386_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload, kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, if it was taken with the current kernel sources."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_src_sha") != kernel_source_sha():
        return None
    return t.get("workloads", {}).get(workload, {}).get(kernel)


def graph_len(steps, cap):
    """Steps per captured graph: the largest g <= cap that divides the timed
    steps (searched down to cap / 2), so that the timed region is whole graph
    replays; cap itself if none does (the remainder then runs as direct
    launches)."""
    g = max(1, min(cap, steps))
    for d in range(g, max(1, g // 2) - 1, -1):
        if steps % d == 0:
            return d
    return g


def run_gpu(wl, steps, warmup, kernel_steps, graph_steps, autotune, tune_cache):
    import torch

    from paper_1911_03386_amd import Ensemble

    trial = min(steps, 64)
    total = warmup + steps + kernel_steps + 4 * trial + 2
    ens = Ensemble(wl.descs, prec=wl.prec, cadence=wl.cadence, max_samples=total // wl.cadence + 2)
    if autotune:
        ens.autotune(tune_cache)
    ens.init_random()
    # launch mode: one trial of each over `trial` steps (after one untimed
    # pass in that mode); graphs are captured, instantiated and uploaded by
    # set_graph_steps, before anything is timed
    gs = graph_len(steps, graph_steps)
    trials = {}
    for g in (gs, 0):
        ens.set_graph_steps(graph_len(trial, g) if g else 0)
        ens.step(trial)
        torch.cuda.synchronize()
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record(ens.stream)
        ens.step(trial)
        t1.record(ens.stream)
        torch.cuda.synchronize()
        trials["graph" if g else "direct"] = t0.elapsed_time(t1) / trial
    mode = "graph" if trials["graph"] <= trials["direct"] else "direct"
    ens.set_graph_steps(gs if mode == "graph" else 0)
    if warmup:
        ens.step(warmup)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(ens.stream)
    ens.step(steps)
    ev1.record(ens.stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    kms = ens.time_kernels(kernel_steps)  # per-launch ms: [x pass, y pass, z pass]
    F, meanC = ens.energy()
    plan = ens.describe()
    ens.close()
    return dict(wall=wall, gpu_ms=gpu_ms, kernel_ms=[float(x) for x in kms], plan=plan,
                F=[float(x) for x in F[:4]], graph={"launch": mode,
                                                    "trial_ms_per_step": {k: round(v, 5) for k, v in trials.items()},
                                                    "steps_per_graph": gs if mode == "graph" else 0,
                                                    "replays": steps // gs if mode == "graph" else 0,
                                                    "direct_steps": steps % gs if mode == "graph" else steps})


def copy_calibration():
    import torch

    n = 256 * 1024 * 1024  # 1 GiB of float32
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(5):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "launches": 5}))


def cpu_baseline(wl, seconds):
    """The FP64 oracle on a bounded sample: the first member of the workload,
    stepped for about `seconds` of wall time on all host threads, then for
    about a third of that on one thread."""
    import numpy as np

    import oracle

    d = wl.descs[0]
    shape = tuple(d.n[a] for a in range(d.dim))[::-1]
    L = [d.L[a] for a in range(d.dim)]
    sites = int(np.prod(shape))

    def rate(budget):
        C = oracle.init_field(shape, d.c0, d.noise, d.seed)
        C = oracle.step(C, d.gamma, d.dt, 1, L=L)  # warm-up
        t0 = time.perf_counter()
        C = oracle.step(C, d.gamma, d.dt, 3, L=L)
        one = (time.perf_counter() - t0) / 3
        k = max(1, int(budget / max(one, 1e-6)))
        t0 = time.perf_counter()
        C = oracle.step(C, d.gamma, d.dt, k, L=L)
        el = time.perf_counter() - t0
        return sites * k / el / 1e9, k, el

    threads = oracle.num_threads()
    cpu_model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    cpu_model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    v, k, el = rate(seconds)
    prev = oracle.set_num_threads(1)
    v1, k1, el1 = rate(seconds / 3)
    oracle.set_num_threads(prev)
    return {
        "value": v,
        "unit": "GLUPS",
        "cores": threads,
        "cpu_model": cpu_model,
        "kind": "oracle",
        "sample": f"member 0 of {wl.name} ({'x'.join(map(str, shape[::-1]))}), {k} steps, {el:.1f} s",
        "single_thread": {"value": v1, "sample": f"{k1} steps, {el1:.1f} s"},
    }


def bench_model1(args):
    """The Model 1 table of Section 3 on the GPU; see the module docstring."""
    import numpy as np
    import torch

    from paper_1911_03386_amd import workloads as W
    from paper_1911_03386_amd.dp import DropletEnsemble

    ns = tuple(int(v) for v in args.model1_ns.split(",")) if args.model1_ns else W.MODEL1_N
    sizes, radii = W.model1_ensemble(ns=ns)
    warm = 1 if args.warmup > 0 else 0
    for _ in range(warm):
        # the same kernels (16 droplets per thread) on a short run
        e = DropletEnsemble([8192, 128], t_end=1e-3, dt_sample=1e-3)
        e.set_radii([W.model1_radii(8192, 1), W.model1_radii(128, 2)])
        e.run(args.dp_attempts)
        e.close()
    ens = DropletEnsemble(sizes, t_end=W.MODEL1_T_END, dt_sample=0.1)
    ens.set_radii(radii)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    launches, kernel_ms = ens.run(args.dp_attempts)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    infos = [ens.info(m) for m in range(len(sizes))]
    evals = float(sum(i["evals"] for i in infos))
    attempts = int(sum(i["accepted"] + i["rejected"] for i in infos))
    stats = {}
    for n in ns:
        idx = [m for m, v in enumerate(sizes) if v == n]
        b0, _ = ens.ensemble_window(20.0, 40.0, idx)
        _, k = ens.ensemble_window(0.0, 40.0, idx)
        a = [infos[m]["accepted"] + infos[m]["rejected"] for m in idx]
        stats[str(n)] = {"beta0": round(b0, 4), "k": float(f"{k:.3g}"), "paper": MODEL1_PAPER.get(n),
                         "attempts_per_member": int(np.mean(a))}
    ens.close()
    value = evals / wall / 1e9
    achieved = DP_FLOPS_PER_EVAL * evals / (kernel_ms / 1e3) / 1e12
    out = {
        "metric": "live-droplet stage evaluations/s, Model 1 table (7 x 100 populations, t <= 40)",
        "value": round(value, 3),
        "unit": "GEval/s",
        "n_gpus": 1,
        "steps": 1,
        "warmup": warm,
        "ms_per_step": wall * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded U(0,1) initial radii)",
        "config": {"workload": "model1_table" if ns == W.MODEL1_N else "model1_" + "_".join(map(str, ns)),
                   "populations": len(sizes), "sizes": list(ns),
                   "members_per_size": W.MODEL1_M, "t_end": W.MODEL1_T_END, "dt_sample": 0.1,
                   "rtol": 1e-6, "atol": 1e-9, "attempts": attempts, "evals": evals,
                   "time_to_solution_s": round(wall, 3)},
        "roofline": {
            "bound": "alu",
            "kernel": "dp step_kernel",
            "achieved": round(achieved, 3),
            "peak": PEAK_FP64_VECTOR_TFLOPS,
            "unit": "TFLOP/s",
            "frac": round(achieved / PEAK_FP64_VECTOR_TFLOPS, 4),
            "traffic": None,
            "flops_per_eval": DP_FLOPS_PER_EVAL,
            "launches": launches,
            "ms_per_launch": round(kernel_ms / max(1, launches), 3),
        },
        "statistics": stats,
    }
    if not args.no_cpu_baseline:
        R0 = W.model1_ensemble(ns=(2048,), M=1)[1][0]
        out["cpu_baseline"] = cpu_baseline_model1(R0, args.dp_cpu_t_end)
    print(json.dumps(out), flush=True)


def cpu_baseline_model1(R0, t_end):
    """The oracle (numpy, one thread) on one N = 2048 population from t = 0."""
    import numpy as np

    from oracle import droplets as orc

    live = [0]

    def counting_rate(V):
        live[0] += int(np.count_nonzero(V > 0.0))
        return orc.rate(V)

    t0 = time.perf_counter()
    orc.dp45(counting_rate, orc.volumes_from_radii(R0), t_end, 0.1, 1e-6, 1e-9, 1e-4)
    dt = time.perf_counter() - t0
    evals = live[0] * 6.0 / 7.0  # the oracle evaluates all seven stages per attempt
    return {"value": round(evals / dt / 1e9, 6), "unit": "GEval/s", "cores": 1, "kind": "oracle",
            "sample": f"one N=2048 population of the table, t in [0, {t_end}] ({dt:.1f} s)"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); "
              "ensemble members would shard across GPUs without communication", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return
    if args.workload == "model1":
        bench_model1(args)
        return
    from paper_1911_03386_amd import CH_F32_BULK, workloads

    wl = workloads.get(args.workload)
    steps = args.steps if args.steps is not None else wl.steps
    r = run_gpu(wl, steps, args.warmup, args.kernel_steps, args.graph_steps, args.autotune,
                args.tune_cache)
    S = wl.sites
    value = S * steps / (r["gpu_ms"] / 1e3) / 1e9
    word = 4 if wl.prec == CH_F32_BULK else 8
    # Each pass reads the field once and writes it once.  A "launch" of a pass
    # is that pass over the whole batch: one kernel per size class, each timed
    # alone with its own start/end timestamps (the timed steps run the classes
    # concurrently on separate streams; step_frac is the whole-step figure).
    kinds = ["x_pass", "y_pass", "z_pass"]
    kms = r["kernel_ms"]
    dom = max(range(3), key=lambda i: kms[i])
    alg_bytes = 2 * word * S
    achieved = alg_bytes / (kms[dom] / 1e3) / 1e9
    traffic = measured_traffic(wl.name, kinds[dom])
    out = {
        "metric": "lattice-site updates/s (GLUPS) + % HBM roofline, FP32-batched vs FP64-plain",
        "value": round(value, 3),
        "unit": "GLUPS",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": r["gpu_ms"] / steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if wl.prec == CH_F32_BULK else "f64",
        "data": "synthetic (seeded uniform-noise initial conditions)",
        "config": {"workload": wl.name, "members": len(wl.descs), "sites": S,
                   "cadence": wl.cadence, "note": wl.note},
        "roofline": {
            "bound": "hbm",
            "kernel": kinds[dom],
            "achieved": round(achieved, 1),
            "peak": PEAK_HBM_GBS,
            "unit": "GB/s",
            "frac": round(achieved / PEAK_HBM_GBS, 4),
            "traffic": traffic,
            "traffic_source": ("stored rocprofv3 FETCH_SIZE + WRITE_SIZE summary (profiles/traffic.json), "
                               "taken with the current kernel sources") if traffic is not None else None,
            "alg_bytes_per_launch": alg_bytes,
            "ms_per_launch": {k: round(v, 5) for k, v in zip(kinds, kms)},
            "classes": len(r["plan"].strip().splitlines()),
            "step_frac": round(S * 4 * word * (1.5 if wl.descs[0].dim == 3 else 1.0)
                               / (r["gpu_ms"] / steps / 1e3) / 1e9 / PEAK_HBM_GBS, 4),
        },
        "timed_region": r["graph"],
        "plan": r["plan"].strip().splitlines(),
        "kernel_src_sha": kernel_source_sha(),
    }
    compares = []
    for cname in [c for c in args.compare.split(",") if c]:
        wc = workloads.get(cname)
        csteps = args.compare_steps if args.compare_steps is not None else wc.steps
        rc = run_gpu(wc, csteps, args.warmup, args.kernel_steps, args.graph_steps,
                     args.autotune, args.tune_cache)
        wordc = 4 if wc.prec == CH_F32_BULK else 8
        vc = wc.sites * csteps / (rc["gpu_ms"] / 1e3) / 1e9
        compares.append({
            "workload": wc.name,
            "dtype": "f32" if wc.prec == CH_F32_BULK else "f64",
            "value": round(vc, 3),
            "unit": "GLUPS",
            "steps": csteps,
            "ms_per_step": rc["gpu_ms"] / csteps,
            "timed_region": rc["graph"],
            "ms_per_launch": {k: round(v, 5) for k, v in zip(kinds, rc["kernel_ms"])},
            "hbm_frac_of_step": round(wc.sites * 4 * wordc * (1.5 if wc.descs[0].dim == 3 else 1.0)
                                      / (rc["gpu_ms"] / csteps / 1e3) / 1e9 / PEAK_HBM_GBS, 4),
            "headline_over_this": round(value / vc, 2),
        })
    if compares:
        out["compare"] = compares
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
