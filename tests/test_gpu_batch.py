"""Batched persistent launch (aqt_batch_*): many instances of different sizes in one
launch reproduce their individual runs, with and without graph capture.

The batched kernel is a separate instantiation of the same tile code, so the compiler
may contract or order floating-point operations differently: jump channels must agree
trajectory by trajectory (up to rare mixed-precision threshold ties), jump times to
the precision of the state arithmetic.  Replays of one batch are bit-identical."""
import numpy as np
import pytest

import workloads as W
from oracle import ame, spectrum, trajectories

from gpu_common import sigma_bound

pytestmark = pytest.mark.gpu


def make_engine(inst):
    from paper_1710_03431_amd.binding import Engine
    eng = Engine(0)
    eng.set_instance(inst)
    eng.precompute(inst.n_grid, inst.levels)
    return eng


def same_records(a, b, t_f, t_rel):
    """Fraction of trajectories with equal jump counts, channels and times within t_rel."""
    K = len(a["jump_count"])
    cap = a["jumps"].shape[1]
    ok = 0
    for j in range(K):
        n = int(a["jump_count"][j])
        if n != int(b["jump_count"][j]):
            continue
        m = min(n, cap)
        x, y = a["jumps"][j, :m], b["jumps"][j, :m]
        if any(not np.array_equal(x[f], y[f]) for f in ("step", "qubit", "kind", "from_level", "to_level")):
            continue
        if np.all(np.abs(x["t"] - y["t"]) <= t_rel * np.abs(y["t"]) + 1e-12 * t_f):
            ok += 1
    return ok / K


@pytest.fixture(scope="module")
def instances():
    insts = [W.pm1_all_to_all(6, 11, t_f=1500.0, n_grid=120, n_levels=16),
             W.pm1_all_to_all(7, 12, t_f=3000.0, n_grid=150, n_levels=32),
             W.pm1_all_to_all(6, 13, t_f=800.0, n_grid=100, n_levels=64),
             W.ring_instance(4, 1001, n_grid=200)]
    return insts, [make_engine(i) for i in insts]


@pytest.mark.parametrize("prec,graph,autotune", [("fp64", False, False), ("fp32", True, True),
                                                  ("bf16", True, True)])
def test_batch_equals_individual_runs(instances, prec, graph, autotune):
    from paper_1710_03431_amd.binding import Batch
    insts, engines = instances
    if prec == "bf16":
        keep = [k for k in range(len(insts)) if insts[k].levels >= 16]
    else:
        keep = list(range(len(insts)))
    runs = [dict(n_traj=300 + 37 * k, seed=5 + k, instance_id=k, record_capacity=32) for k in keep]
    b = Batch([engines[k] for k in keep], runs, precision=prec, graph=graph, autotune=autotune)
    b.launch()
    got = b.results()
    b.launch()          # a replay overwrites the sums and gives the same numbers
    again = b.results()
    t_rel, need = {"fp64": (1e-9, 0.999), "fp32": (1e-4, 0.98), "bf16": (1e-3, 0.97)}[prec]
    for k, r, g, g2, tile in zip(keep, runs, got, again, b.tiles):
        K = r["n_traj"]
        ref = engines[k].run(K, prec, seed=r["seed"], instance_id=k, record_capacity=32, tile=tile)
        frac = same_records(g, ref, insts[k].t_f, t_rel)
        assert frac >= need, (k, frac)
        # a trajectory that diverges moves each per-grid P_GS sum by at most 1
        diff = np.abs(g["pgs_sum"] - ref["pgs_sum"]).max()
        assert diff <= (1.0 - frac) * K + 1e-6 * K, (k, diff)
        np.testing.assert_array_equal(g2["pgs_sum"], g["pgs_sum"])
        np.testing.assert_array_equal(g2["jumps"], g["jumps"])
        np.testing.assert_array_equal(g2["jump_totals"], 2 * g["jump_totals"])   # accumulated
    b.close()


def test_bf16_sixteen_levels_matches_ame():
    """16 retained levels use the BF16 16x16x16 MFMA; the mean follows the split-step AME."""
    inst = W.pm1_all_to_all(5, 21, t_f=2000.0, n_grid=400, n_levels=16)
    tabs = spectrum.all_tables(inst)
    P = ame.split_step(tabs, inst)
    eng = make_engine(inst)
    K = 4000
    res = eng.run(K, "bf16", seed=3)
    m, se = trajectories.mean_and_stderr(res["pgs_sum"], res["pgs_sumsq"], K)
    assert np.all(np.abs(m - P) <= 3 * sigma_bound(P, se, K) + 1e-4)


def test_batch_mixes_bath_models_and_grids():
    """Instances with bath terms (one more channel than qubits), sz/sx couplings, a
    non-uniform grid and the Lamb shift in one FP64 batch: each reproduces its own
    run, so the batched kernel reads every instance's channel count, step lengths and
    phase tables."""
    from paper_1710_03431_amd.binding import Batch
    base = W.pm1_all_to_all(6, 11, t_f=1500.0, n_grid=120, n_levels=16)
    cz = np.vstack([np.eye(6), np.zeros((2, 6))])
    cx = np.zeros((8, 6))
    cx[6, 0], cx[7, 3] = 1.0, 0.5
    g = np.arange(base.n_grid) / (base.n_grid - 1)
    insts = [base.with_(bath_terms=W.two_term_bath(6)),
             base.with_(coupling=(cz, cx, None)),
             base.with_(s_grid=0.5 * (1.0 - np.cos(np.pi * g))),
             base.with_(lamb_shift=True)]
    engines = [make_engine(i) for i in insts]
    assert [e.channel_count() for e in engines] == [7, 8, 6, 6]
    runs = [dict(n_traj=256 + 29 * k, seed=7 + k, instance_id=k, record_capacity=48) for k in range(len(insts))]
    b = Batch(engines, runs, precision="fp64", graph=False, autotune=False)
    b.launch()
    got = b.results()
    for k, (r, res, tile) in enumerate(zip(runs, got, b.tiles)):
        K = r["n_traj"]
        ref = engines[k].run(K, "fp64", seed=r["seed"], instance_id=k, record_capacity=48, tile=tile)
        frac = same_records(res, ref, insts[k].t_f, 1e-9)
        assert frac >= 0.999, (k, frac)
        assert np.abs(res["pgs_sum"] - ref["pgs_sum"]).max() <= (1.0 - frac) * K + 1e-6 * K


@pytest.fixture(scope="module")
def oracle_batch():
    """Instances of 16 (truncated), 32 (truncated), 64 and 128 levels and the 4-qubit ring,
    each with oracle tables handed over through aqt_set_tables."""
    from gpu_common import engine_with_oracle_tables
    insts = [W.pm1_all_to_all(6, 11, t_f=1500.0, n_grid=120, n_levels=16),
             W.pm1_all_to_all(7, 12, t_f=3000.0, n_grid=150, n_levels=32),
             W.pm1_all_to_all(6, 13, t_f=4000.0, n_grid=100),
             W.pm1_all_to_all(7, 14, t_f=4000.0, n_grid=80),
             W.ring_instance(4, 1001, n_grid=200)]
    tabs = [spectrum.all_tables(i) for i in insts]
    return insts, tabs, [engine_with_oracle_tables(i, t) for i, t in zip(insts, tabs)]


def test_batch_fp64_matches_oracle_trajectories(oracle_batch):
    """FP64 batch of five instances (the 64- and 128-level ones run under eight wavefronts
    in the batched kernel) against oracle.trajectories.run on the same Philox streams
    (key (seed, instance id)): jump records per trajectory, totals and population sums."""
    from paper_1710_03431_amd.binding import Batch
    from gpu_common import compare_jump_records
    insts, tabs, engines = oracle_batch
    runs = [dict(n_traj=200 + 41 * k, seed=31 + k, instance_id=k, record_capacity=96) for k in range(len(insts))]
    b = Batch(engines, runs, precision="fp64", graph=True, autotune=False)
    b.launch()
    got = b.results()
    for k, (r, res) in enumerate(zip(runs, got)):
        K = r["n_traj"]
        ref = trajectories.run(tabs[k], insts[k], K, seed=r["seed"], instance_id=k)
        assert max(len(j) for j in ref.jumps) < r["record_capacity"]
        frac, worst = compare_jump_records(res["jumps"], res["jump_count"], ref.jumps, insts[k].t_f)
        assert frac >= 0.999, (k, frac, worst)
        assert np.abs(res["pgs_sum"] - ref.pgs_sum).max() <= (1.0 - frac) * K + 1e-9 * K, k
        if frac == 1.0:
            np.testing.assert_array_equal(res["jump_totals"], ref.kind_totals)
            np.testing.assert_array_equal(res["net_gs"], ref.net_gs)
    b.close()


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_batch_mixed_precision_matches_split_step_ame(oracle_batch, prec):
    """Mixed-precision batch (graph-captured, autotuned tiles): every instance's mean at
    every grid point against its split-step AME (bound of gpu_common.assert_mean_matches)."""
    from paper_1710_03431_amd.binding import Batch
    from gpu_common import assert_mean_matches
    insts, tabs, engines = oracle_batch
    runs = [dict(n_traj=3000 + 64 * k, seed=41 + k, instance_id=k) for k in range(len(insts))]
    b = Batch(engines, runs, precision=prec, graph=True, autotune=True)
    b.launch()
    got = b.results()
    for k, (r, res) in enumerate(zip(runs, got)):
        K = r["n_traj"]
        P = ame.split_step(tabs[k], insts[k])
        m, se = trajectories.mean_and_stderr(res["pgs_sum"], res["pgs_sumsq"], K)
        assert_mean_matches(m, se, P, K, (k, prec))
    b.close()


@pytest.mark.parametrize("prec", ["bf16", "fp32"])
def test_batched_workload_instances_match_stored_ame(prec):
    """The first eight instances of the batched workload (6-9 qubits, 16/32/64 retained
    levels, t_f 1-98 us, 1000 grid points, 2048 trajectories, the workload's seeds and
    instance ids), GPU precompute, one graph-captured autotuned launch: every instance's
    mean at the stored grid points (every tenth and the last) against the oracle's
    split-step AME (tests/golden/batched_ame_pgs.json), bound of
    gpu_common.assert_mean_matches."""
    import json
    import os
    from paper_1710_03431_amd.binding import Batch
    from gpu_common import assert_mean_matches
    ref = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "batched_ame_pgs.json")))
    insts = W.config_batched()
    rows = ref["instances"]
    sel = [insts[r["index"]] for r in rows]
    assert [i.name for i in sel] == [r["name"] for r in rows]
    engines = [make_engine(i) for i in sel]
    runs = [dict(n_traj=i.n_traj, seed=i.seed, instance_id=i.instance_id) for i in sel]
    b = Batch(engines, runs, precision=prec, graph=True, autotune=True)
    b.launch()
    got = b.results()
    for r, res, inst in zip(rows, got, sel):
        K = inst.n_traj
        idx = np.array(r["grid_points"])
        m, se = trajectories.mean_and_stderr(res["pgs_sum"], res["pgs_sumsq"], K)
        assert_mean_matches(m[idx], se[idx], np.array(r["pgs"]), K, (r["name"], prec))
    b.close()
