"""Throughput of the GPU trajectory engine on the 8-qubit all-to-all workload.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--cpu-traj 3072] [--cpu-grid 500] [--no-cpu]

One bench step = one aqt_run: 10^4 trajectories through the whole anneal
(2000 grid points, 1999 trajectory steps each) with the eigenbasis tables
already resident in HBM.  value = trajectory-steps/s of the FP32 MFMA path;
the FP64 and BF16x3 paths are timed the same way and reported beside it, each
with its ground-state-population error against the FP64 master equation.
Prints one JSON line.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "trajectory-steps/s at 1 MI355X (mixed vs FP64) at stated error vs FP64 AME"
PEAK = {"fp32": 157.3e12, "fp64": 78.6e12, "bf16": 2.5e15}
FLOP_PER_TRAJ_STEP = lambda n: 4 * n * n + 10 * n   # overlap GEMM (real n x n by n x 2) + diagonal/norm


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n-traj", type=int, default=10_000)
    ap.add_argument("--cpu-traj", type=int, default=3072)
    ap.add_argument("--cpu-grid", type=int, default=500)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--precisions", default="fp32,fp64,bf16")
    return ap.parse_args()


def load_ame_reference():
    path = os.path.join(ROOT, "tests", "golden", "a2a8_ame_pgs.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        return json.load(f)


def time_precision(eng, torch, K, prec, steps, warmup, seed):
    outs = eng.alloc_outputs(K, 0, per_trajectory=False)
    for w in range(warmup):
        eng.run_into(outs, K, prec, seed=seed + 1000 + w)
    torch.cuda.synchronize()
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    sums = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        for k in ("pgs_sum", "pgs_sumsq", "jump_totals", "net_hist"):
            outs[k].zero_()
        starts[i].record()
        eng.run_into(outs, K, prec, seed=seed + i)
        ends[i].record()
        sums.append((outs["pgs_sum"][-1].clone(), outs["pgs_sumsq"][-1].clone()))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms = [s.elapsed_time(e) for s, e in zip(starts, ends)]
    p = [float(a) / K for a, _ in sums]
    q = [float(b) / K for _, b in sums]
    return {"wall_s": wall, "event_ms": ev_ms, "pgs_final": p, "pgs_sq_final": q}


def cpu_baseline(inst, n_traj, n_steps):
    """The FP64 oracle's trajectory code on the host cores over a bounded sample: the
    first n_steps steps of the same anneal for n_traj trajectories (tables built first,
    untimed, as the GPU precompute is)."""
    import itertools
    from oracle import spectrum, trajectories
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count()
    tabs = list(itertools.islice(spectrum.table_stream(inst), n_steps))
    t0 = time.perf_counter()
    trajectories.run(tabs, inst, n_traj, record=False)
    dt = time.perf_counter() - t0
    steps = n_traj * len(tabs)
    return {"value": steps / dt, "unit": "trajectory-steps/s", "cores": threads, "kind": "oracle",
            "sample": f"{n_traj} trajectories x the first {len(tabs)} of {inst.n_grid - 1} steps of the "
                      f"same 8-qubit anneal (FP64 NumPy oracle, {dt:.1f} s timed; its tables built "
                      f"beforehand, untimed)"}


def measured_traffic(kernel_key):
    """HBM bytes per launch of the timed kernel from the committed rocprofv3 counter
    record, or None when the kernel source changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "k_trajectories_a2a8_n256_K10000_traffic.json")
    src = os.path.join(ROOT, "paper_1710_03431_amd", "csrc", "step.hip")
    try:
        rec = json.load(open(path))
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    except (OSError, ValueError):
        return None
    if rec.get("step_hip_sha256") != sha or rec.get("kernel") != kernel_key:
        return None
    return rec["traffic_bytes"]


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this engine runs on one GPU; multi-GPU runs are not part of this build",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch
    import workloads as W
    from paper_1710_03431_amd.binding import Engine

    inst = W.config_a2a8(args.n_traj)
    K = args.n_traj
    M = inst.n_grid
    n = inst.levels
    eng = Engine(0)
    eng.set_instance(inst)
    t0 = time.perf_counter()
    eng.precompute(M, n)
    precompute_s = time.perf_counter() - t0
    print(f"# precompute {precompute_s:.2f} s (n={n}, M={M})", file=sys.stderr, flush=True)

    ref = load_ame_reference()
    p_ame = ref["pgs"][-1] if ref else None
    results = {}
    for prec in args.precisions.split(","):
        r = time_precision(eng, torch, K, prec, args.steps, args.warmup, seed=inst.seed)
        ms = sum(r["event_ms"]) / len(r["event_ms"])
        mean_p = sum(r["pgs_final"]) / len(r["pgs_final"])
        # standard error of the pooled mean over all timed runs
        R = K * len(r["pgs_final"])
        var = (sum(r["pgs_sq_final"]) * K - R * mean_p * mean_p) / (R - 1)
        se = math.sqrt(max(var, 0.0) / R)
        results[prec] = {"ms": ms, "value": K * (M - 1) / (ms / 1e3), "pgs_final": mean_p, "pgs_se": se,
                         "err_vs_ame": (abs(mean_p - p_ame) if p_ame is not None else None), "wall_s": r["wall_s"]}
        print(f"# {prec}: {ms:.2f} ms/run, {results[prec]['value']:.4g} traj-steps/s, "
              f"P_GS(1)={mean_p:.5f}+-{se:.5f}", file=sys.stderr, flush=True)

    head = results.get("fp32") or next(iter(results.values()))
    head_prec = "fp32" if "fp32" in results else next(iter(results))
    flops = FLOP_PER_TRAJ_STEP(n) * K * (M - 1)
    achieved = flops / (head["ms"] / 1e3)
    roof = {"bound": "mfma", "achieved": achieved / 1e12, "peak": PEAK[head_prec] / 1e12, "unit": "TFLOP/s",
            "frac": achieved / PEAK[head_prec],
            "traffic": measured_traffic("k_trajectories<256, 5, ModeF32>") if head_prec == "fp32" else None,
            "kernel": f"k_trajectories<n=256, {head_prec}>",
            "per_unit": f"{FLOP_PER_TRAJ_STEP(n)} flop per trajectory-step"}
    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(W.config_a2a8(args.cpu_traj), args.cpu_traj, args.cpu_grid)
    line = {
        "metric": METRIC, "value": head["value"], "unit": "trajectory-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": head["ms"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": head_prec, "data": "synthetic",
        "config": {"workload": "8-qubit all-to-all +-1 Ising anneal, full spectrum n=256, 2000 grid points, "
                               "t_f=10us, 10^4 trajectories", "n_traj": K, "n_levels": n, "n_grid": M,
                   "precision": head_prec, "seed": inst.seed},
        "error_vs_fp64_ame": {"P_GS_final_ame": p_ame,
                              **{p: {"P_GS_final": v["pgs_final"], "stderr": v["pgs_se"],
                                     "abs_err": v["err_vs_ame"]} for p, v in results.items()}},
        "paths": {p: {"value": v["value"], "ms_per_step": v["ms"]} for p, v in results.items()},
        "precompute_s": precompute_s,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
