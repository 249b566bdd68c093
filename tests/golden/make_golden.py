"""Writes the stored expected values under tests/golden/ using only oracle/.

Run from the repository root:  python tests/golden/make_golden.py
It records
  * the seed scan that fixes the 8-qubit all-to-all instance: the first seed
    >= 1002 whose s = 1 Ising ground state is non-degenerate (so the
    "ground-state population" of Sec. V is that of a single level);
  * the split-step FP64 AME ground-state population of that instance on its
    2000-point grid (a2a8_ame_pgs.json), the reference for the stated error
    of the GPU trajectory averages (python tests/golden/make_golden.py --ame);
  * the same for the 4-qubit ring workload (small_ame_pgs.json, --ame-small);
  * central differences (h = 1e-4: absolute for control points, relative for
    eta) of that AME's final ground-state population with respect to the
    schedule control points and eta, for the 16-control-point version of the
    4-qubit ring (every parameter, --grad4) and of the 8-qubit instance (a
    subset of the parameters, --grad8; each AME solve there takes minutes);
  * the oracle's own trajectories of the 8-qubit workload (--a2a8-traj): 10^4
    trajectories with the workload's seed on its 2000-point grid, summarised as
    jump totals by kind, the histograms of net jumps into the ground cluster and
    of jump counts, the ground-cluster population sums at every grid point and
    the full jump records of a few trajectories from both ends of the batch; and
    the split-step AME's expected jumps per trajectory by kind (Sec. III,
    E[dN] = <A^dag A> dt) on the same grid (a2a8_traj.json);
  * the split-step AME ground-state population of the first eight instances of the
    batched workload (every tenth grid point and the last), the reference for the
    batched launch's per-instance errors (--batched; batched_ame_pgs.json);
  * the split-step AME ground-cluster population of the 16-qubit gadget truncated to its
    32 lowest canonical levels, on its 500-point grid (--gadget; gadget16_ame_pgs.json):
    the same tables as oracle.spectrum.table_stream, with the per-grid-point Lanczos
    solves spread over worker processes;
  * the split-step AME of the 8-qubit workload under the bench's model switches --
    correlated baths 0.5^|a-b|, bath terms (rho = 0.5), sz and sx couplings on every
    qubit (--a2a8-models; a2a8_models_ame_pgs.json: every tenth grid point and the
    last);
  * the discretisation error of the eigenbasis scheme (--discretisation): the
    split-step AME's final ground-state population on the workload grid and on
    grids with 2x and 4x the steps, first-order Richardson extrapolations from
    them, and for the 4-qubit ring also the continuous AME integrated in t
    (discretisation.json).
"""
import json
import os
import sys

if "--grad4" in sys.argv or "--grad8" in sys.argv:
    os.environ.setdefault("OMP_NUM_THREADS", "1")   # one BLAS thread per worker process
    os.environ.setdefault("OPENBLAS_NUM_THREADS", "1")

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import workloads  # noqa: E402
from oracle import model  # noqa: E402


def scan_a2a8(start=1002, stop=1100):
    rows = []
    for seed in range(start, stop):
        inst = workloads.pm1_all_to_all(8, seed)
        e = np.sort(model.hz_diag(inst.h, inst.J))
        unique = bool(e[1] - e[0] > 0.5)
        rows.append({"seed": seed, "e0": float(e[0]), "e1": float(e[1]), "unique": unique})
        if unique:
            break
    return rows


def ame_a2a8():
    from oracle import ame, spectrum
    inst = workloads.config_a2a8(10)
    P = ame.split_step(spectrum.table_stream(inst), inst)
    with open(os.path.join(HERE, "a2a8_ame_pgs.json"), "w") as f:
        json.dump({"source": "oracle.ame.split_step over oracle.spectrum.table_stream(workloads.config_a2a8())",
                   "instance": inst.name, "n_grid": inst.n_grid, "t_f": inst.t_f,
                   "pgs": [float(p) for p in P]}, f)


def ame_small():
    from oracle import ame, spectrum
    inst = workloads.config_small()
    P = ame.split_step(spectrum.table_stream(inst), inst)
    with open(os.path.join(HERE, "small_ame_pgs.json"), "w") as f:
        json.dump({"source": "oracle.ame.split_step over oracle.spectrum.table_stream(workloads.config_small())",
                   "instance": inst.name, "n_grid": inst.n_grid, "t_f": inst.t_f,
                   "pgs": [float(p) for p in P]}, f)


def _fd_worker(args):
    inst, kind, j, h = args
    from oracle import gradient
    ip, step = gradient._perturbed(inst, kind, j, +1.0, h)
    im, _ = gradient._perturbed(inst, kind, j, -1.0, h)
    return (gradient.final_pgs(ip) - gradient.final_pgs(im)) / (2.0 * step)


def fd_golden(inst, params, fname, workers):
    from concurrent.futures import ProcessPoolExecutor
    h = 1e-4
    with ProcessPoolExecutor(max_workers=workers) as ex:
        vals = list(ex.map(_fd_worker, [(inst, k, j, h) for k, j in params]))
    with open(os.path.join(HERE, fname), "w") as f:
        json.dump({"source": "central differences of oracle.gradient.final_pgs (split-step AME) over "
                             "workloads instance " + inst.name,
                   "instance": inst.name, "n_grid": inst.n_grid, "t_f": inst.t_f, "h": h,
                   "params": [[k, j] for k, j in params], "grad": [float(v) for v in vals]}, f, indent=1)


def traj_a2a8(n_traj=10_000, sample=(0, 1, 2, 3, 9996, 9997, 9998, 9999)):
    import time
    from oracle import ame, spectrum, trajectories
    inst = workloads.config_a2a8(n_traj)
    t0 = time.time()
    res = trajectories.run(spectrum.table_stream(inst), inst, n_traj, seed=inst.seed,
                           instance_id=inst.instance_id)
    print("trajectories %.0f s" % (time.time() - t0), flush=True)
    t0 = time.time()
    expected = ame.expected_jumps(spectrum.table_stream(inst), inst)
    print("expected jumps %.0f s" % (time.time() - t0), flush=True)
    counts = np.array([len(j) for j in res.jumps])
    net_vals, net_n = np.unique(res.net_gs, return_counts=True)
    cnt_vals, cnt_n = np.unique(counts, return_counts=True)
    out = {"source": "oracle.trajectories.run and oracle.ame.expected_jumps over "
                     "oracle.spectrum.table_stream(workloads.config_a2a8())",
           "instance": inst.name, "n_grid": inst.n_grid, "t_f": inst.t_f, "n_traj": n_traj,
           "seed": inst.seed, "instance_id": inst.instance_id,
           "kind_totals": [int(v) for v in res.kind_totals],
           "expected_jumps_per_traj": [float(v) for v in expected],
           "net_hist": {str(int(v)): int(c) for v, c in zip(net_vals, net_n)},
           "count_hist": {str(int(v)): int(c) for v, c in zip(cnt_vals, cnt_n)},
           "count_var": float(counts.var(ddof=1)),
           "pgs_sum": [float(v) for v in res.pgs_sum],
           "pgs_sumsq": [float(v) for v in res.pgs_sumsq],
           "sample_jumps": {str(j): [[float(r[0]), int(r[1]), int(r[2]), int(r[3]), int(r[4]), int(r[5])]
                                     for r in res.jumps[j]] for j in sample}}
    with open(os.path.join(HERE, "a2a8_traj.json"), "w") as f:
        json.dump(out, f)


def _batched_worker(k):
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    from oracle import ame, spectrum
    inst = workloads.config_batched()[k]
    P = ame.split_step(spectrum.table_stream(inst), inst)
    return k, inst.name, [float(v) for v in P]


def batched_ame(count=8):
    from concurrent.futures import ProcessPoolExecutor
    with ProcessPoolExecutor(max_workers=count) as ex:
        rows = list(ex.map(_batched_worker, range(count)))
    insts = workloads.config_batched()
    out = {"source": "oracle.ame.split_step over oracle.spectrum.table_stream(workloads.config_batched()[k])",
           "stride": 10, "instances": []}
    for k, name, P in rows:
        M = insts[k].n_grid
        idx = list(range(0, M, 10)) + ([M - 1] if (M - 1) % 10 else [])
        out["instances"].append({"index": k, "name": name, "n_grid": M, "t_f": insts[k].t_f,
                                 "grid_points": idx, "pgs": [P[i] for i in idx]})
    with open(os.path.join(HERE, "batched_ame_pgs.json"), "w") as f:
        json.dump(out, f, indent=0)


def _gadget_eigen(args):
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    inst, s, n = args
    from oracle import spectrum
    E, V, gs = spectrum.eigen(inst, s, n, 1e-8)
    return E, V, gs


def gadget_ame(workers=8):
    """oracle.ame.split_step over the tables oracle.spectrum.table_stream builds for the
    gadget, with the eigensolves of the grid points computed ahead in worker processes
    (same function, same arguments, consumed in grid order)."""
    import time
    from concurrent.futures import ProcessPoolExecutor
    from oracle import ame, spectrum
    inst = workloads.config_gadget(10)
    M, n = inst.n_grid, inst.levels
    dt = inst.t_f / (M - 1)

    def tables():
        with ProcessPoolExecutor(max_workers=workers) as ex:
            it = ex.map(_gadget_eigen, [(inst, g / (M - 1), max(n, 1)) for g in range(M)], chunksize=1)
            E0, V0, gs0 = next(it)
            if gs0 != 1:
                raise ValueError("degenerate ground state at s = 0")
            psi0 = V0[:, 0]
            Vprev = None
            t0 = time.time()
            for g, (E, V, gs) in enumerate(it, start=1):
                if g == 1:
                    c = V.T @ psi0
                    leak = 1.0 - float(c @ c)
                    cinit, O = c / np.linalg.norm(c), None
                else:
                    O, S = spectrum.polar(V.T @ Vprev)
                    leak = 1.0 - float(S.min()) ** 2
                    cinit = None
                z, R, Gamma, zdiag, d, shift = spectrum.grid_tables(inst, E, V, dt)
                Vprev = V
                if g % 25 == 0:
                    print("gadget grid point %d of %d, %.0f s" % (g, M - 1, time.time() - t0), flush=True)
                yield spectrum.GridTables(g=g, s=g / (M - 1), E=E, gs=gs, O=O, cinit=cinit, z=z, R=R, Gamma=Gamma,
                                          zdiag=zdiag, d=d, leak=leak, V=None, shift=shift, dt=dt,
                                          t0=(g - 1) * dt)

    P, leaks = [], []
    pgs = ame.split_step(tables(), inst)
    with open(os.path.join(HERE, "gadget16_ame_pgs.json"), "w") as f:
        json.dump({"source": "oracle.ame.split_step over the tables of oracle.spectrum.table_stream("
                             "workloads.config_gadget())", "instance": inst.name, "n_grid": M, "n_levels": n,
                   "t_f": inst.t_f, "pgs": [float(v) for v in pgs]}, f)


def a2a8_model(key):
    """The 8-qubit workload under one of the bench's model switches (same construction as
    bench.py's --lamb-shift, --bath-corr 0.5, --bath-terms 0.5, --zx-coupling)."""
    inst = workloads.config_a2a8(10)
    q = inst.n_qubits
    if key == "lamb_shift":
        return inst.with_(lamb_shift=True)
    if key == "bath_corr_0.5":
        return inst.with_(bath_corr=np.array([[0.5 ** abs(a - b) for b in range(q)] for a in range(q)]))
    if key == "bath_terms_0.5":
        return inst.with_(bath_terms=workloads.two_term_bath(q, rho=0.5))
    if key == "zx_coupling":
        return inst.with_(coupling=(np.vstack([np.eye(q), np.zeros((q, q))]), np.vstack([np.zeros((q, q)), np.eye(q)]),
                                    None))
    raise KeyError(key)


# The Lamb shift is left out: the oracle evaluates its principal-value integrals one
# frequency pair at a time, minutes per grid point at 256 levels (its parity is held
# on the 3- and 4-qubit rings instead).
A2A8_MODELS = ("bath_corr_0.5", "bath_terms_0.5", "zx_coupling")


def _model_worker(key):
    from oracle import ame, spectrum
    inst = a2a8_model(key)
    P = ame.split_step(spectrum.table_stream(inst), inst)
    return key, [float(v) for v in P]


def a2a8_models():
    from concurrent.futures import ProcessPoolExecutor
    with ProcessPoolExecutor(max_workers=len(A2A8_MODELS)) as ex:
        rows = list(ex.map(_model_worker, A2A8_MODELS))
    inst = workloads.config_a2a8(10)
    M = inst.n_grid
    idx = list(range(0, M, 10)) + ([M - 1] if (M - 1) % 10 else [])
    out = {"source": "oracle.ame.split_step over oracle.spectrum.table_stream of workloads.config_a2a8() with "
                     "each model switch (make_golden.a2a8_model)", "instance": inst.name, "n_grid": M,
           "grid_points": idx, "models": {k: [P[i] for i in idx] for k, P in rows}}
    with open(os.path.join(HERE, "a2a8_models_ame_pgs.json"), "w") as f:
        json.dump(out, f)


def discretisation():
    import time
    from oracle import ame, spectrum
    out = {"source": "oracle.ame.split_step at n_grid, 2 (n_grid - 1) + 1 and 4 (n_grid - 1) + 1 points; "
                     "Richardson (first order) P_inf = 2 P_2M - P_M; oracle.ame.continuous for the 4-qubit ring",
           "cases": []}
    for inst in (workloads.config_small(), workloads.config_a2a8(10)):
        steps = inst.n_grid - 1
        row = {"instance": inst.name, "n_grid": inst.n_grid, "t_f": inst.t_f, "pgs": {}}
        for mult in (1, 2, 4):
            M = mult * steps + 1
            t0 = time.time()
            P = ame.split_step(spectrum.table_stream(inst.with_(n_grid=M)), inst.with_(n_grid=M))
            row["pgs"][str(M)] = float(P[-1])
            print(inst.name, M, float(P[-1]), "%.0f s" % (time.time() - t0), flush=True)
        p1, p2, p4 = (row["pgs"][str(m * steps + 1)] for m in (1, 2, 4))
        row["richardson_from_M_2M"] = 2 * p2 - p1
        row["richardson_from_2M_4M"] = 2 * p4 - p2
        row["error_at_workload_grid"] = p1 - (2 * p4 - p2)
        if inst.n_qubits <= 4:
            t0 = time.time()
            row["continuous"] = float(ame.continuous(inst, [1.0])[-1])
            row["error_vs_continuous"] = p1 - row["continuous"]
            print(inst.name, "continuous", row["continuous"], "%.0f s" % (time.time() - t0), flush=True)
        out["cases"].append(row)
        with open(os.path.join(HERE, "discretisation.json"), "w") as f:
            json.dump(out, f, indent=1)


if __name__ == "__main__":
    if "--a2a8-models" in sys.argv:
        a2a8_models()
        sys.exit(0)
    if "--gadget" in sys.argv:
        gadget_ame()
        sys.exit(0)
    if "--batched" in sys.argv:
        batched_ame()
        sys.exit(0)
    if "--a2a8-traj" in sys.argv:
        traj_a2a8()
        sys.exit(0)
    if "--discretisation" in sys.argv:
        discretisation()
        sys.exit(0)
    if "--grad4" in sys.argv:
        from oracle import gradient
        inst = workloads.config_small_ctrl()
        fd_golden(inst, gradient.parameter_list(inst), "small_ctrl16_fd_gradient.json", 8)
        sys.exit(0)
    if "--grad8" in sys.argv:
        inst = workloads.config_gradient(10)
        params = [("A", 4), ("A", 8), ("B", 4), ("B", 8), ("eta", 0)]
        fd_golden(inst, params, "a2a8_ctrl16_fd_gradient.json", 5)
        sys.exit(0)
    if "--ame" in sys.argv:
        ame_a2a8()
        sys.exit(0)
    if "--ame-small" in sys.argv:
        ame_small()
        sys.exit(0)
    rows = scan_a2a8()
    with open(os.path.join(HERE, "a2a8_seed_scan.json"), "w") as f:
        json.dump({"source": "oracle.model.hz_diag over workloads.pm1_all_to_all(8, seed)",
                   "rows": rows, "chosen": rows[-1]["seed"]}, f, indent=1)
    print("chosen seed", rows[-1]["seed"])
