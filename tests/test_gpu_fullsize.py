"""Parity of the waiting-time trajectory kernel with the FP64 oracle at the level counts
the workloads run at: 64, 128 and 256 levels (full spectra of 6-, 7- and 8-qubit
all-to-all +-1 instances).

These sizes take code paths that 16 and 32 levels never reach: eight wavefronts per
workgroup, the overlap GEMM with every wave sharing all column tiles (B read one
chunk ahead), and the jump handler's 64-lane segment with 2 or 4 levels per lane, whose
source and target scans carry their running sums across the lane chunks.

Two kinds of checks:
  * shortened anneals (200 grid points, 50 ns steps, so most crossing steps hold
    several jumps) with oracle tables handed over through aqt_set_tables: FP64 jump
    records per trajectory against oracle.trajectories.run on the same Philox draws
    (Sec. IV waiting-time procedure; App. B eq. Pi(t)), and FP32 / BF16 means against
    the split-step AME, the exact mean of the discrete process;
  * the 8-qubit workload itself (2000 grid points, 10^4 trajectories, GPU precompute,
    the launch shapes the benchmark times) against stored oracle values written by
    tests/golden/make_golden.py: the oracle's own trajectories on the same draws (jump
    records of sampled trajectories, the net-jump and jump-count histograms, jump totals
    by kind, population sums at every grid point) and the AME (populations at every grid
    point; expected jumps by kind, Sec. III E[dN] = <A^dag A> dt).
"""
import json
import os

import numpy as np
import pytest

import workloads as W
from oracle import ame, spectrum, trajectories

from gpu_common import assert_mean_matches, compare_jump_records, engine_with_oracle_tables

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

# Tolerances.  FP64 on both sides: jump times agree to 1e-9 relative (plus 1e-12 t_f for
# times near zero) and at most 0.1% of trajectories may differ (a threshold or CDF
# boundary decided differently by rounding).  A trajectory that differs moves each
# per-grid population sum by at most 1.
FP64_SAME = 0.999


def _short(nq):
    # all levels kept; the ground-cluster population is that of the lowest s = 1 cluster
    return W.pm1_all_to_all(nq, 10 + nq - 5, t_f=1.0e4, n_grid=200)


K_SHORT = 1003   # a ragged last tile for every tile width


@pytest.fixture(scope="module", params=[6, 7, 8], ids=["n64", "n128", "n256"])
def short(request):
    inst = _short(request.param)
    tabs = spectrum.all_tables(inst)
    ref = trajectories.run(tabs, inst, K_SHORT)
    return inst, tabs, ref


def _cap(ref):
    return max(len(j) for j in ref.jumps) + 1


def _check_fp64_against_oracle(res, ref, inst, K):
    frac, worst = compare_jump_records(res["jumps"], res["jump_count"], ref.jumps, inst.t_f)
    assert frac >= FP64_SAME, (frac, worst)
    bad = int(round((1.0 - frac) * K))
    # whole-batch quantities move only through the differing trajectories
    assert np.abs(res["pgs_sum"] - ref.pgs_sum).max() <= bad + 1e-9 * K
    counts = np.array([len(j) for j in ref.jumps])
    assert np.abs(res["jump_count"] - counts).sum() <= 200 * bad
    assert np.count_nonzero(res["net_gs"] != ref.net_gs) <= bad
    hist = np.bincount(np.clip(ref.net_gs, -64, 64) + 64, minlength=129)
    assert np.abs(res["net_hist"] - hist).sum() <= 2 * bad
    if bad == 0:
        np.testing.assert_array_equal(res["jump_totals"], ref.kind_totals)
        np.testing.assert_array_equal(res["net_gs"], ref.net_gs)
        np.testing.assert_allclose(res["pgs_sum"], ref.pgs_sum, rtol=1e-9, atol=1e-9)


@pytest.mark.parametrize("tile", [0, 16])
def test_fp64_per_trajectory_parity(short, tile):
    """Automatic tile and 16 trajectories per workgroup: jump sequences and times, net
    jumps, totals and sums."""
    inst, tabs, ref = short
    K = K_SHORT
    assert ref.kind_totals[0] > 0 and ref.kind_totals[1] > 0, "the instance must relax and excite"
    eng = engine_with_oracle_tables(inst, tabs)
    res = eng.run(K, "fp64", seed=inst.seed, instance_id=inst.instance_id, record_capacity=_cap(ref),
                  tile=tile, final_state=True)
    _check_fp64_against_oracle(res, ref, inst, K)
    # amplitudes of the trajectories whose paths agree (up to a global phase after a jump)
    same = [j for j in range(K) if res["jump_count"][j] == len(ref.jumps[j])]
    pop = (res["final_state"] ** 2).sum(axis=2).T
    np.testing.assert_allclose(pop[:, same], (np.abs(ref.final_state) ** 2)[:, same], atol=1e-9)


def test_several_jumps_in_one_step(short):
    """The shortened anneals put several jumps into one step for many trajectories (the
    handler's loop over the rest of the step), so the parity above covers it."""
    inst, tabs, ref = short
    multi = sum(1 for j in ref.jumps for a, b in zip(j, j[1:]) if a[1] == b[1])
    assert multi >= 200


def _wide_tile(inst):
    """The widest tile the 8-qubit workload runs with (40 trajectories) where the level
    count allows it, else the widest allowed (32)."""
    return 40 if inst.levels >= 128 else 32


@pytest.mark.parametrize("prec,wide", [("fp32", False), ("fp32", True), ("bf16", False)])
def test_mixed_precision_mean_matches_split_step_ame(short, prec, wide):
    """FP32 (and BF16 operands with FP32 accumulation) means at every grid point against
    the split-step AME, the exact mean of the discrete process (bound of
    gpu_common.assert_mean_matches); automatic and widest tiles."""
    inst, tabs, _ = short
    P = ame.split_step(tabs, inst)
    eng = engine_with_oracle_tables(inst, tabs)
    K = 4000
    res = eng.run(K, prec, seed=inst.seed + 1, instance_id=inst.instance_id, tile=_wide_tile(inst) if wide else 0)
    m, se = trajectories.mean_and_stderr(res["pgs_sum"], res["pgs_sumsq"], K)
    assert_mean_matches(m, se, P, K, (inst.name, prec, wide))


def test_fp32_jump_records_follow_fp64(short):
    """FP32 stepping on the same draws: most trajectories reproduce the oracle's jump
    channels, with times to the state precision."""
    inst, tabs, ref = short
    K = K_SHORT
    eng = engine_with_oracle_tables(inst, tabs)
    res = eng.run(K, "fp32", seed=inst.seed, instance_id=inst.instance_id, record_capacity=_cap(ref),
                  tile=_wide_tile(inst))
    frac, _ = compare_jump_records(res["jumps"], res["jump_count"], ref.jumps, inst.t_f, rel=1e-4)
    assert frac >= 0.97, frac


# ------------------------------------------------------- the 8-qubit workload --
@pytest.fixture(scope="module")
def a2a8():
    inst = W.config_a2a8()
    from paper_1710_03431_amd.binding import Engine
    eng = Engine(0)
    eng.set_instance(inst)
    eng.precompute(inst.n_grid, inst.levels)
    traj = json.load(open(os.path.join(GOLDEN, "a2a8_traj.json")))
    amep = np.array(json.load(open(os.path.join(GOLDEN, "a2a8_ame_pgs.json")))["pgs"])
    assert traj["seed"] == inst.seed and traj["n_traj"] == inst.n_traj and traj["n_grid"] == inst.n_grid
    return inst, eng, traj, amep


def _hist(d, lo, hi):
    out = np.zeros(hi - lo + 1, dtype=np.int64)
    for k, v in d.items():
        out[min(max(int(k), lo), hi) - lo] += v
    return out


def test_workload_fp64_against_oracle_trajectories(a2a8):
    """FP64 run of the 8-qubit workload (GPU precompute; 8 trajectories per workgroup, as
    benchmarked) on the oracle's draws: the sampled trajectories' full jump records, the
    histograms, the jump totals and the population sums at every grid point."""
    inst, eng, traj, _ = a2a8
    K = inst.n_traj
    cap = 2 + max(int(k) for k in traj["count_hist"])
    res = eng.run(K, "fp64", seed=inst.seed, instance_id=inst.instance_id, record_capacity=cap)
    ids = sorted(int(j) for j in traj["sample_jumps"])
    recs = [[tuple(r) for r in traj["sample_jumps"][str(j)]] for j in ids]
    frac, worst = compare_jump_records(res["jumps"][ids], res["jump_count"][ids], recs, inst.t_f)
    assert frac == 1.0, (frac, worst)
    allowed = int((1.0 - FP64_SAME) * K)          # 10 differing trajectories
    counts = np.bincount(res["jump_count"], minlength=cap + 1)
    want_counts = _hist(traj["count_hist"], 0, cap)
    assert np.abs(counts[:cap + 1] - want_counts).sum() <= 2 * allowed
    assert np.abs(res["net_hist"] - _hist(traj["net_hist"], -64, 64)).sum() <= 2 * allowed
    assert np.abs(res["jump_totals"] - np.array(traj["kind_totals"])).sum() <= 200 * allowed
    assert np.abs(res["pgs_sum"] - np.array(traj["pgs_sum"])).max() <= allowed + 1e-9 * K


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp64"])
def test_workload_mean_at_every_grid_point(a2a8, prec):
    """The benchmarked run (10^4 trajectories, automatic tile) against the split-step
    AME at all 2000 grid points (bound of gpu_common.assert_mean_matches: the final
    population within 3 standard errors + 1e-4)."""
    inst, eng, _, amep = a2a8
    K = inst.n_traj
    res = eng.run(K, prec, seed=inst.seed + 17, instance_id=inst.instance_id)
    m, se = trajectories.mean_and_stderr(res["pgs_sum"], res["pgs_sumsq"], K)
    assert_mean_matches(m, se, amep, K, prec)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_workload_jump_statistics(a2a8, prec):
    """Mixed precision on the oracle's draws: jump totals by kind against the AME's
    expected jumps (4 standard errors), net-jump histogram close to the oracle
    trajectories' own, and jump counts per trajectory equal to the FP64 run's."""
    inst, eng, traj, _ = a2a8
    K = inst.n_traj
    res = eng.run(K, prec, seed=inst.seed, instance_id=inst.instance_id)
    r64 = eng.run(K, "fp64", seed=inst.seed, instance_id=inst.instance_id)
    expected = K * np.array(traj["expected_jumps_per_traj"])
    # standard error of a kind's total: Poisson, widened by the over-dispersion of the
    # per-trajectory counts (variance / mean of the oracle's counts, at least 1)
    counts = np.array([int(k) for k, v in traj["count_hist"].items() for _ in range(v)])
    disp = max(1.0, traj["count_var"] / counts.mean())
    se = np.sqrt(np.maximum(expected, 1.0) * disp)
    assert np.all(np.abs(res["jump_totals"] - expected) <= 4.0 * se), (res["jump_totals"], expected, se)
    agree = np.mean(res["jump_count"] == r64["jump_count"])
    assert agree >= 0.97, agree
    diff = np.abs(res["net_hist"] - _hist(traj["net_hist"], -64, 64)).sum()
    assert diff <= 2 * (1.0 - agree) * K + 2, diff


def _golden_models():
    import importlib.util
    spec = importlib.util.spec_from_file_location("make_golden", os.path.join(GOLDEN, "make_golden.py"))
    mg = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mg)
    return mg


@pytest.mark.parametrize("model", ["bath_corr_0.5", "bath_terms_0.5", "zx_coupling"])
def test_workload_model_switches_match_stored_ame(model):
    """The 8-qubit workload under the benchmark's bath-model switches (baths correlated as
    0.5^|a-b|, two bath terms per qubit at rho = 0.5, sz and sx couplings on every qubit;
    the instances are built by the same function that wrote the references), GPU
    precompute, 10^4 FP32 trajectories: the mean at the stored grid points (every tenth
    and the last) against the oracle's split-step AME of the same model
    (tests/golden/a2a8_models_ame_pgs.json), bound of gpu_common.assert_mean_matches."""
    from paper_1710_03431_amd.binding import Engine
    ref = json.load(open(os.path.join(GOLDEN, "a2a8_models_ame_pgs.json")))
    inst = _golden_models().a2a8_model(model)
    assert ref["n_grid"] == inst.n_grid
    eng = Engine(0)
    eng.set_instance(inst)
    eng.precompute(inst.n_grid, inst.levels)
    K = 10_000
    res = eng.run(K, "fp32", seed=inst.seed + 29, instance_id=inst.instance_id)
    m, se = trajectories.mean_and_stderr(res["pgs_sum"], res["pgs_sumsq"], K)
    idx = np.array(ref["grid_points"])
    assert_mean_matches(m[idx], se[idx], np.array(ref["models"][model]), K, model)
