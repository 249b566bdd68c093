"""Throughput of the GPU trajectory engine.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload a2a8|ring4|gadget16|batched|grad|fixed]
                    [--lamb-shift] [--bath-corr RHO] [--bath-terms RHO] [--zx-coupling]
                    [--cpu-traj 3072] [--cpu-grid 500] [--no-cpu]

One bench step = one aqt_run: all trajectories of the workload through the whole
anneal with the eigenbasis tables already resident in HBM (the GPU precompute
runs once, untimed, and is reported as precompute_s).  value = trajectory-steps/s
of the workload's headline precision; the other precisions are timed the same way
and reported beside it, each with its ground-state-population error against the
FP64 master equation where a stored reference exists.  Prints one JSON line.

Workloads:
  a2a8      (default) 8-qubit all-to-all +-1 Ising anneal, full spectrum n = 256,
            2000 grid points, t_f = 10 us, 10^4 trajectories, FP32 headline
  ring4     4-qubit ring, full spectrum n = 16, 1001 grid points, t_f = 1 us,
            10^3 trajectories, FP64 headline (the plain method)
  gadget16  16-qubit two-cluster gadget (N = 65536) truncated to 32 levels by the
            iterative eigensolver, 500 grid points, t_f = 10 us, 10^5 trajectories,
            FP32 headline
  batched   256 instances of 6-10 qubits truncated to 16, 32 or 64 levels, 1000 grid
            points, t_f 1-100 us, 2048 trajectories each, all in one persistent
            graph-captured launch with autotuned tiles; BF16x3 headline
  grad      gradient of the final ground-state population with respect to 16 + 16
            schedule control points and eta (aqt_grad_pgs) on the a2a8 instance,
            10^5 FP32 trajectories; one step = one gradient evaluation (forward run,
            checkpointed replay and adjoint sweep), value = trajectory-steps/s of it
  fixed     the a2a8 anneal with the fixed-step unraveling (aqt_run_fixed_step, 4
            sub-steps per grid step), FP32; value = grid trajectory-steps/s, with the
            waiting-time run timed beside it
--lamb-shift adds the Ohmic Lamb shift to the tables (a2a8, ring4, fixed)
--bath-corr RHO correlates the qubits' baths, C_ab = RHO^|a - b| (a2a8, ring4)
--bath-terms RHO frequency-dependent correlations: local baths correlated as 0.5^|a - b|
            (cutoff 8 pi) plus a bath shared by all qubits with weight RHO and cutoff
            2 pi (one more jump channel) (a2a8, ring4)
--zx-coupling every qubit couples through sz and through sx, each to its own bath
            (2 n_qubits jump channels) (a2a8, ring4)
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
TILE_TQ = {"a2a8": 5}   # column tiles the launch picks for 10^4 trajectories at n = 256 (TT = 40)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="a2a8", choices=("a2a8", "ring4", "gadget16", "batched", "grad", "fixed"))
    ap.add_argument("--lamb-shift", action="store_true")
    ap.add_argument("--bath-corr", type=float, default=None)
    ap.add_argument("--bath-terms", type=float, default=None)
    ap.add_argument("--zx-coupling", action="store_true")
    ap.add_argument("--substeps", type=int, default=4)
    ap.add_argument("--n-traj", type=int, default=0, help="override the workload's trajectory count")
    ap.add_argument("--cpu-traj", type=int, default=3072)
    ap.add_argument("--cpu-grid", type=int, default=0, help="steps of the CPU sample (default per workload)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--precisions", default="")
    return ap.parse_args()


def workload(name, n_traj):
    import workloads as W
    if name == "a2a8":
        inst = W.config_a2a8(n_traj or 10_000)
        return dict(inst=inst, head="fp32", precisions="fp32,fp64,bf16", golden="a2a8_ame_pgs.json", cpu_grid=500,
                    text="8-qubit all-to-all +-1 Ising anneal, full spectrum n=256, 2000 grid points, "
                         f"t_f=10us, {inst.n_traj} trajectories")
    if name == "ring4":
        inst = W.config_small().with_(n_traj=n_traj or 1000)
        return dict(inst=inst, head="fp64", precisions="fp64,fp32", golden="small_ame_pgs.json", cpu_grid=1000,
                    text="4-qubit ring, U[-1,1] couplings, full spectrum n=16, 1001 grid points, t_f=1us, "
                         f"{inst.n_traj} trajectories")
    inst = W.config_gadget(n_traj or 100_000)
    # the oracle's sparse eigensolver takes ~10 s per grid point here: a 4-step CPU sample
    return dict(inst=inst, head="fp32", precisions="fp32,fp64,bf16", golden="gadget16_ame_pgs.json", cpu_grid=4,
                text="16-qubit two-cluster gadget (N=65536) truncated to 32 levels, 500 grid points, "
                     f"t_f=10us, {inst.n_traj} trajectories")


def load_ame_reference(name):
    if not name:
        return None
    path = os.path.join(ROOT, "tests", "golden", name)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        return json.load(f)


def same_grid_as_models(inst):
    """The stored model references are on the workload's own grid."""
    return inst.n_grid == 2000 and inst.t_f == 1.0e4


def converged_error(inst, results):
    """Error of each path's P_GS(1) against the grid-converged AME: the first-order
    Richardson value from the split-step AME on 2x and 4x the steps
    (tests/golden/discretisation.json, written from the oracle), where one is stored for
    this instance and grid."""
    path = os.path.join(ROOT, "tests", "golden", "discretisation.json")
    try:
        cases = json.load(open(path))["cases"]
    except (OSError, ValueError, KeyError):
        return None
    for c in cases:
        if c["instance"] == inst.name and c["n_grid"] == inst.n_grid and c["t_f"] == inst.t_f \
                and not (inst.lamb_shift or inst.bath_corr is not None or inst.bath_terms is not None
                         or inst.coupling is not None):
            conv = c["richardson_from_2M_4M"]
            return {"P_GS_final_converged": conv, "reference": "Richardson from the split-step AME at 2x and 4x steps",
                    "same_grid_ame_minus_converged": c["pgs"][str(inst.n_grid)] - conv,
                    **{p: {"err": v["pgs_final"] - conv, "stderr": v["pgs_se"]} for p, v in results.items()}}
    return None


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
        sums.append((outs["pgs_sum"][-1].clone(), outs["pgs_sumsq"][-1].clone(), outs["jump_totals"].clone()))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms = [s.elapsed_time(e) for s, e in zip(starts, ends)]
    p = [float(a) / K for a, _, _ in sums]
    q = [float(b) / K for _, b, _ in sums]
    jumps = sum(float(j.sum()) for _, _, j in sums) / (K * len(sums))
    return {"wall_s": wall, "event_ms": ev_ms, "pgs_final": p, "pgs_sq_final": q, "jumps_per_traj": jumps}


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
    n_steps = min(n_steps, inst.n_grid - 1)
    tabs = list(itertools.islice(spectrum.table_stream(inst), n_steps))
    t0 = time.perf_counter()
    trajectories.run(tabs, inst, n_traj, record=False)
    dt = time.perf_counter() - t0
    steps = n_traj * len(tabs)
    return {"value": steps / dt, "unit": "trajectory-steps/s", "cores": threads, "kind": "oracle",
            "sample": f"{n_traj} trajectories x the first {len(tabs)} of {inst.n_grid - 1} steps of the "
                      f"same anneal ({inst.name}; FP64 NumPy oracle, {dt:.1f} s timed; its tables built "
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


def bench_batched(args):
    """256 instances in one persistent launch (aqt_batch_*), graph-captured, autotuned."""
    import torch
    import workloads as W
    from paper_1710_03431_amd.binding import Batch, Engine
    insts = W.config_batched(n_traj=args.n_traj or 2048)
    t0 = time.perf_counter()
    engines = []
    for k, inst in enumerate(insts):
        eng = Engine(0)
        eng.set_instance(inst)
        eng.precompute(inst.n_grid, inst.levels)
        engines.append(eng)
        if k % 8 == 7:
            print(f"# precomputed {k + 1}/{len(insts)} instances, {time.perf_counter() - t0:.1f} s",
                  file=sys.stderr, flush=True)
    precompute_s = time.perf_counter() - t0
    print(f"# precompute {precompute_s:.1f} s for {len(insts)} instances", file=sys.stderr, flush=True)
    steps_total = sum(i.n_traj * (i.n_grid - 1) for i in insts)
    flops = sum(FLOP_PER_TRAJ_STEP(i.levels) * i.n_traj * (i.n_grid - 1) for i in insts)
    runs = [dict(n_traj=i.n_traj, seed=i.seed, instance_id=i.instance_id) for i in insts]
    results = {}
    for prec in (args.precisions or "bf16,fp32").split(","):
        t1 = time.perf_counter()
        b = Batch(engines, runs, precision=prec, graph=True, autotune=True)
        setup_s = time.perf_counter() - t1
        for _ in range(args.warmup):
            b.launch()
        torch.cuda.synchronize()
        for o in b.outs:   # jump totals accumulate over launches: count the timed ones only
            o["jump_totals"].zero_()
        torch.cuda.synchronize()
        starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
        ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
        for i in range(args.steps):
            starts[i].record()
            b.launch()
            ends[i].record()
        torch.cuda.synchronize()
        ms = sum(s.elapsed_time(e) for s, e in zip(starts, ends)) / args.steps
        res = b.results()
        jumps = sum(float(r["jump_totals"].sum()) for r in res) / args.steps
        p = [float(r["pgs_sum"][-1]) / i.n_traj for r, i in zip(res, insts)]
        tiles = sorted(set(b.tiles))
        b.close()
        sampled = []
        ref = load_ame_reference("batched_ame_pgs.json")
        for row in (ref["instances"] if ref else []):
            k = row["index"]
            Kk = insts[k].n_traj
            m = float(res[k]["pgs_sum"][-1]) / Kk
            v = (float(res[k]["pgs_sumsq"][-1]) - Kk * m * m) / (Kk - 1)
            sampled.append({"instance": k, "name": insts[k].name, "P_GS_final": m, "P_GS_final_ame": row["pgs"][-1],
                            "abs_err": abs(m - row["pgs"][-1]), "stderr": math.sqrt(max(v, 0.0) / Kk)})
        results[prec] = {"ms": ms, "value": steps_total / (ms / 1e3), "setup_s": setup_s, "tiles": tiles,
                         "mean_pgs_final": sum(p) / len(p), "sampled": sampled,
                         "jumps_per_launch": jumps, "jumps_per_s": jumps / (ms / 1e3)}
        print(f"# {prec}: {ms:.2f} ms/launch, {results[prec]['value']:.4g} traj-steps/s, tiles {tiles}, "
              f"{jumps:.4g} jumps/launch ({jumps / (ms / 1e3):.3g} jumps/s), "
              f"setup (graph capture + autotune) {setup_s:.1f} s", file=sys.stderr, flush=True)
    head_prec = "bf16" if "bf16" in results else next(iter(results))
    head = results[head_prec]
    achieved = flops / (head["ms"] / 1e3)
    cpu = None
    if not args.no_cpu:
        small = insts[0]
        cpu = cpu_baseline(small.with_(n_traj=args.cpu_traj), args.cpu_traj, args.cpu_grid or 200)
    line = {
        "metric": METRIC, "value": head["value"], "unit": "trajectory-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": head["ms"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": head_prec, "data": "synthetic",
        "config": {"workload": f"{len(insts)} instances, 6-10 qubits, n in {{16,32,64}}, 1000 grid points, "
                               f"t_f 1-100 us, {insts[0].n_traj} trajectories each, one graph-captured "
                               "persistent launch", "n_instances": len(insts),
                   "trajectory_steps_per_launch": steps_total, "precision": head_prec},
        # the first eight instances against their stored split-step AME (same grid)
        "error_vs_fp64_ame_same_grid": {p: v["sampled"] for p, v in results.items()},
        # jump-bound (the small-level groups): the handlers' throughput beside the MFMA roofline
        "paths": {p: {"value": v["value"], "ms_per_step": v["ms"], "tiles": v["tiles"],
                      "mean_P_GS_final": v["mean_pgs_final"], "jumps_per_launch": v["jumps_per_launch"],
                      "jumps_per_s": v["jumps_per_s"]} for p, v in results.items()},
        "precompute_s": precompute_s,
        "roofline": {"bound": "mfma", "achieved": achieved / 1e12, "peak": PEAK[head_prec] / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / PEAK[head_prec], "traffic": None,
                     "kernel": f"k_batch<{head_prec}>", "per_unit": "4 n^2 + 10 n flop per trajectory-step"},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line))


def cpu_grad_baseline(inst, n_traj, n_steps):
    """The oracle's per-trajectory gradient estimates (central differences of each path's
    log weight, 2 x (2m + 1) perturbed table streams) on a bounded sample: an anneal of
    n_steps steps of the same step size, n_traj trajectories."""
    from oracle import gradient
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count()
    dt = inst.t_f / (inst.n_grid - 1)
    small = inst.with_(n_grid=n_steps + 1, t_f=dt * n_steps)
    t0 = time.perf_counter()
    gradient.trajectory_gradients(small, n_traj)
    el = time.perf_counter() - t0
    return {"value": n_traj * n_steps / el, "unit": "trajectory-steps/s", "cores": threads, "kind": "oracle",
            "sample": f"{n_traj} trajectories x a {n_steps}-step anneal with the same step size and "
                      f"{2 * len(inst.A_ctrl) + 1} parameters ({inst.name}; FP64 NumPy oracle: trajectories, "
                      f"path replays and the perturbed tables, {el:.1f} s)"}


def bench_grad(args):
    """aqt_grad_pgs on the control-point workload; forward-only aqt_run timed beside it."""
    import torch
    import workloads as W
    from paper_1710_03431_amd.binding import Engine
    inst = W.config_gradient(args.n_traj or 100_000)
    K, M, n = inst.n_traj, inst.n_grid, inst.levels
    m = len(inst.A_ctrl)
    eng = Engine(0)
    eng.set_instance(inst)
    t0 = time.perf_counter()
    eng.precompute(M, n)
    t1 = time.perf_counter()
    eng.grad_pgs(64, "fp32", seed=inst.seed + 777)   # first call adds the derivative tables
    t2 = time.perf_counter()
    print(f"# precompute {t1 - t0:.1f} s, derivative tables + first call {t2 - t1:.1f} s", file=sys.stderr,
          flush=True)
    ref = load_ame_reference("a2a8_ctrl16_fd_gradient.json")
    results = {}
    for prec in (args.precisions or "fp32").split(","):
        for w in range(args.warmup):
            eng.grad_pgs(K, prec, seed=inst.seed + 1000 + w)
        times, outs = [], []
        for i in range(args.steps):
            torch.cuda.synchronize()
            ts = time.perf_counter()
            outs.append(eng.grad_pgs(K, prec, seed=inst.seed + i, instance_id=inst.instance_id))
            times.append(time.perf_counter() - ts)
        fwd = time_precision(eng, torch, K, prec, max(1, args.steps), 1, seed=inst.seed)
        fwd_ms = sum(fwd["event_ms"]) / len(fwd["event_ms"])
        ms = 1e3 * sum(times) / len(times)
        g = [sum(o["grad"][c] for o in outs) / len(outs) for c in range(2 * m + 1)]
        se = [math.sqrt(sum(o["grad_se"][c] ** 2 for o in outs)) / len(outs) for c in range(2 * m + 1)]
        res = {"ms": ms, "value": K * (M - 1) / (ms / 1e3), "forward_ms": fwd_ms, "grad": g, "grad_se": se,
               "P_GS_final": sum(o["value"] for o in outs) / len(outs)}
        if ref:
            col = {"A": lambda j: j, "B": lambda j: m + j, "eta": lambda j: 2 * m}
            z = {f"{k}{j}": (g[col[k](j)] - v) / se[col[k](j)] for (k, j), v in zip(ref["params"], ref["grad"])}
            res["z_vs_fd"] = z
        results[prec] = res
        print(f"# {prec}: gradient {ms:.1f} ms ({res['value']:.4g} traj-steps/s), forward run {fwd_ms:.1f} ms, "
              f"ratio {ms / fwd_ms:.2f}; P_GS(1)={res['P_GS_final']:.5f}", file=sys.stderr, flush=True)
    head_prec = "fp32" if "fp32" in results else next(iter(results))
    head = results[head_prec]
    # per trajectory-step: the replay kick, X_g products at both points (2; one product serves both
    # schedule directions and both adjoints) and the two adjoint kicks, each 4 n^2 flop; plus the
    # forward run
    per_unit = 5 * 4 * n * n + FLOP_PER_TRAJ_STEP(n)
    flops = per_unit * K * (M - 1)
    achieved = flops / (head["ms"] / 1e3)
    cpu = None if args.no_cpu else cpu_grad_baseline(inst, 16, 2)
    line = {
        "metric": "trajectory-steps/s of the adjoint gradient (forward + checkpointed adjoint) at 1 MI355X",
        "value": head["value"], "unit": "trajectory-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": head["ms"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": head_prec, "data": "synthetic",
        "config": {"workload": f"gradient of P_GS(1) w.r.t. {m}+{m} schedule control points and eta, 8-qubit "
                               f"all-to-all +-1 anneal, n=256, {M} grid points, t_f=10us, {K} trajectories",
                   "name": inst.name, "n_traj": K, "n_levels": n, "n_grid": M, "n_params": 2 * m + 1},
        "paths": results,
        "fd_reference": ({f"{k}{j}": v for (k, j), v in zip(ref["params"], ref["grad"])} if ref else None),
        "roofline": {"bound": "mfma", "achieved": achieved / 1e12, "peak": PEAK[head_prec] / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / PEAK[head_prec], "traffic": None,
                     "kernel": f"k_grad + forward run ({head_prec})",
                     "per_unit": f"{per_unit} flop per trajectory-step"},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line))


def bench_fixed(args):
    """Fixed-step unraveling on the a2a8 anneal, waiting-time aqt_run beside it."""
    import torch
    import workloads as W
    from paper_1710_03431_amd.binding import Engine
    inst = W.config_a2a8(args.n_traj or 10_000).with_(lamb_shift=args.lamb_shift)
    K, M, n, S = inst.n_traj, inst.n_grid, inst.levels, args.substeps
    eng = Engine(0)
    eng.set_instance(inst)
    t0 = time.perf_counter()
    eng.precompute(M, n)
    precompute_s = time.perf_counter() - t0
    ref = load_ame_reference(None if args.lamb_shift else "a2a8_ame_pgs.json")
    for w in range(args.warmup):
        eng.run_fixed_step(K, S, "fp32", seed=inst.seed + 100 + w)
    times, p, q = [], [], []
    for i in range(args.steps):
        torch.cuda.synchronize()
        ts = time.perf_counter()
        r = eng.run_fixed_step(K, S, "fp32", seed=inst.seed + i, instance_id=inst.instance_id)
        times.append(time.perf_counter() - ts)
        p.append(float(r["pgs_sum"][-1]) / K)
        q.append(float(r["pgs_sumsq"][-1]) / K)
    R = K * len(p)
    p_mean = sum(p) / len(p)
    p_se = math.sqrt(max((sum(q) * K - R * p_mean * p_mean) / (R - 1), 0.0) / R)
    ms = 1e3 * sum(times) / len(times)
    wt = time_precision(eng, torch, K, "fp32", max(1, args.steps), 1, seed=inst.seed)
    wt_ms = sum(wt["event_ms"]) / len(wt["event_ms"])
    flops = FLOP_PER_TRAJ_STEP(n) * K * (M - 1)
    achieved = flops / (ms / 1e3)
    print(f"# fixed-step ({S} sub-steps): {ms:.1f} ms/run, waiting-time {wt_ms:.1f} ms/run; "
          f"P_GS(1) {sum(p) / len(p):.5f} vs waiting-time {sum(wt['pgs_final']) / len(wt['pgs_final']):.5f}",
          file=sys.stderr, flush=True)
    line = {
        "metric": "grid trajectory-steps/s of the fixed-step unraveling at 1 MI355X", "value": K * (M - 1) / (ms / 1e3),
        "unit": "trajectory-steps/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "fp32", "data": "synthetic",
        "config": {"workload": f"8-qubit all-to-all +-1 anneal, n=256, {M} grid points x {S} sub-steps, t_f=10us, "
                               f"{K} trajectories" + (", Lamb shift" if args.lamb_shift else ""),
                   "substeps": S, "lamb_shift": args.lamb_shift},
        "P_GS_final": p_mean, "P_GS_final_waiting_time": sum(wt["pgs_final"]) / len(wt["pgs_final"]),
        "P_GS_final_ame": (ref["pgs"][-1] if ref else None),
        # against the split-step AME on the same grid: includes the fixed-step scheme's own
        # first-order error in the sub-step, which the waiting-time procedure does not have
        "error_vs_fp64_ame_same_grid": ({"P_GS_final": p_mean, "stderr": p_se, "abs_err": abs(p_mean - ref["pgs"][-1]),
                                         "note": "fixed-step scheme, first order in the sub-step"} if ref else None),
        "waiting_time_ms": wt_ms, "precompute_s": precompute_s,
        "roofline": {"bound": "mfma", "achieved": achieved / 1e12, "peak": PEAK["fp32"] / 1e12, "unit": "TFLOP/s",
                     "frac": achieved / PEAK["fp32"], "traffic": None, "kernel": "k_fixed_step<256, 16, float>",
                     "per_unit": f"{FLOP_PER_TRAJ_STEP(n)} flop per grid trajectory-step (the basis change)"},
        "cpu_baseline": None,
    }
    print(json.dumps(line))


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this engine runs on one GPU; runs on several GPUs are not supported",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    if args.workload == "batched":
        bench_batched(args)
        return
    if args.workload == "grad":
        bench_grad(args)
        return
    if args.workload == "fixed":
        bench_fixed(args)
        return
    import torch
    from paper_1710_03431_amd.binding import Engine

    wl = workload(args.workload, args.n_traj)
    inst = wl["inst"].with_(lamb_shift=args.lamb_shift)
    if args.bath_corr is not None:
        import numpy as np
        q = inst.n_qubits
        inst = inst.with_(bath_corr=np.array([[args.bath_corr ** abs(a - b) for b in range(q)] for a in range(q)]))
    if args.bath_terms is not None:
        import workloads as W
        inst = inst.with_(bath_terms=W.two_term_bath(inst.n_qubits, rho=args.bath_terms))
    if args.zx_coupling:
        import numpy as np
        q = inst.n_qubits
        inst = inst.with_(coupling=(np.vstack([np.eye(q), np.zeros((q, q))]),
                                    np.vstack([np.zeros((q, q)), np.eye(q)]), None))
    switches = [k for k, on in (("lamb_shift", args.lamb_shift), (f"bath_corr_{args.bath_corr}", args.bath_corr is not None),
                                (f"bath_terms_{args.bath_terms}", args.bath_terms is not None),
                                ("zx_coupling", args.zx_coupling)) if on]
    model_ref = None
    if switches:
        # the default references hold independent baths without the Lamb shift; one switch on
        # the 8-qubit workload has its own stored AME (tests/golden/a2a8_models_ame_pgs.json)
        wl["golden"] = None
        models = load_ame_reference("a2a8_models_ame_pgs.json") if args.workload == "a2a8" else None
        if models and len(switches) == 1 and switches[0] in models["models"] and same_grid_as_models(inst):
            model_ref = models["models"][switches[0]][-1]
    K = inst.n_traj
    M = inst.n_grid
    n = inst.levels
    eng = Engine(0)
    eng.set_instance(inst)
    t0 = time.perf_counter()
    eng.precompute(M, n)
    precompute_s = time.perf_counter() - t0
    print(f"# precompute {precompute_s:.2f} s ({inst.name}, n={n}, M={M})", file=sys.stderr, flush=True)

    ref = load_ame_reference(wl["golden"])
    p_ame = ref["pgs"][-1] if ref else model_ref
    results = {}
    for prec in (args.precisions or wl["precisions"]).split(","):
        r = time_precision(eng, torch, K, prec, args.steps, args.warmup, seed=inst.seed)
        ms = sum(r["event_ms"]) / len(r["event_ms"])
        mean_p = sum(r["pgs_final"]) / len(r["pgs_final"])
        # standard error of the pooled mean over all timed runs
        R = K * len(r["pgs_final"])
        var = (sum(r["pgs_sq_final"]) * K - R * mean_p * mean_p) / (R - 1)
        se = math.sqrt(max(var, 0.0) / R)
        results[prec] = {"ms": ms, "value": K * (M - 1) / (ms / 1e3), "pgs_final": mean_p, "pgs_se": se,
                         "err_vs_ame": (abs(mean_p - p_ame) if p_ame is not None else None), "wall_s": r["wall_s"],
                         "jumps_per_traj": r["jumps_per_traj"]}
        print(f"# {prec}: {ms:.2f} ms/run, {results[prec]['value']:.4g} traj-steps/s, "
              f"P_GS(1)={mean_p:.5f}+-{se:.5f}, {r['jumps_per_traj']:.1f} jumps/trajectory", file=sys.stderr,
              flush=True)

    head_prec = wl["head"] if wl["head"] in results else next(iter(results))
    head = results[head_prec]
    flops = FLOP_PER_TRAJ_STEP(n) * K * (M - 1)
    achieved = flops / (head["ms"] / 1e3)
    traffic = None
    if args.workload == "a2a8" and head_prec == "fp32" and K == 10_000:
        traffic = measured_traffic(f"k_trajectories<256, {TILE_TQ['a2a8']}, ModeF32>")
    roof = {"bound": "mfma", "achieved": achieved / 1e12, "peak": PEAK[head_prec] / 1e12, "unit": "TFLOP/s",
            "frac": achieved / PEAK[head_prec], "traffic": traffic,
            "kernel": f"k_trajectories<n={n}, {head_prec}>",
            "per_unit": f"{FLOP_PER_TRAJ_STEP(n)} flop per trajectory-step"}
    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(inst.with_(n_traj=args.cpu_traj), args.cpu_traj, args.cpu_grid or wl["cpu_grid"])
    line = {
        "metric": METRIC, "value": head["value"], "unit": "trajectory-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": head["ms"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": head_prec, "data": "synthetic",
        "config": {"workload": wl["text"] + (", Lamb shift" if args.lamb_shift else "")
                   + (f", bath correlation {args.bath_corr}^|a-b|" if args.bath_corr is not None else "")
                   + (f", bath terms 0.5^|a-b| (cutoff 8 pi) + shared {args.bath_terms} (cutoff 2 pi)"
                      if args.bath_terms is not None else "")
                   + (", sz and sx couplings (2 n_qubits channels)" if args.zx_coupling else ""),
                   "name": inst.name,
                   "n_traj": K, "n_levels": n, "n_grid": M, "precision": head_prec, "seed": inst.seed},
        # accuracy target (3 sigma + 1e-4): against the FP64 split-step AME on the same grid,
        # the exact mean of the discrete process the trajectories sample
        "error_vs_fp64_ame_same_grid": {"P_GS_final_ame": p_ame,
                                        **{p: {"P_GS_final": v["pgs_final"], "stderr": v["pgs_se"],
                                               "abs_err": v["err_vs_ame"]} for p, v in results.items()}},
        # context: the scheme's own discretisation error, against the grid-converged AME
        "error_vs_converged_ame": converged_error(inst, results),
        # jumps per second: the throughput of the jump handler, which binds the runs with
        # few levels and many jumps (their MFMA share is small)
        "paths": {p: {"value": v["value"], "ms_per_step": v["ms"], "jumps_per_traj": v["jumps_per_traj"],
                      "jumps_per_s": v["jumps_per_traj"] * K / (v["ms"] / 1e3)}
                  for p, v in results.items()},
        "precompute_s": precompute_s,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
