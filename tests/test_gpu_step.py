"""Parity of the HIP trajectory kernel with the FP64 oracle, tables supplied by the oracle.

The kernel runs through the C ABI (aqt_set_tables + aqt_run); every expected
value comes from oracle/ on the same seeded inputs.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import ame, spectrum, trajectories

from gpu_common import compare_jump_records, engine_with_oracle_tables, sigma_bound

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def small():
    inst = W.config_small()
    tabs = spectrum.all_tables(inst)
    return inst, tabs


def test_tables_roundtrip_and_decay_rates(small):
    inst, tabs = small
    eng = engine_with_oracle_tables(inst, tabs)
    got = eng.get_tables()
    for T in tabs[::97]:
        np.testing.assert_allclose(got["E"][T.g], T.E, rtol=0, atol=0)
        np.testing.assert_allclose(got["Gamma"][T.g], T.Gamma, rtol=1e-13, atol=1e-18)
        if T.O is not None:
            np.testing.assert_allclose(got["O"][T.g], T.O, rtol=0, atol=1e-15)
    np.testing.assert_array_equal(got["cinit"], tabs[0].cinit)


def test_closed_system_amplitudes_fp64():
    """eta = 0: no jumps; the final amplitudes are the product of overlaps and phases.
    Checks the MFMA operand and accumulator layouts element by element (n = 16 and 32)."""
    for nq in (4, 5):
        inst = W.ring_instance(nq, 77, t_f=30.0, eta=0.0, n_grid=120)
        tabs = spectrum.all_tables(inst)
        ref = trajectories.run(tabs, inst, 5)
        eng = engine_with_oracle_tables(inst, tabs)
        res = eng.run(5, "fp64", seed=inst.seed, final_state=True)
        c = res["final_state"][..., 0] + 1j * res["final_state"][..., 1]
        np.testing.assert_allclose(c.T, ref.final_state, atol=1e-12)
        assert res["jump_totals"].sum() == 0
        for prec, tol in (("fp32", 2e-5), ("bf16", 2e-4)):
            if prec == "bf16" and nq < 5:
                continue
            r2 = eng.run(5, prec, seed=inst.seed, final_state=True)
            c2 = r2["final_state"][..., 0] + 1j * r2["final_state"][..., 1]
            assert np.abs(c2.T - ref.final_state).max() < tol, prec


def test_fp64_per_trajectory_parity(small):
    """4-qubit workload, 1000 trajectories: jump sequences identical in >= 99.9% of
    trajectories, jump times within 1e-9 relative."""
    inst, tabs = small
    K = 1000
    ref = trajectories.run(tabs, inst, K)
    eng = engine_with_oracle_tables(inst, tabs)
    cap = 64
    res = eng.run(K, "fp64", seed=inst.seed, instance_id=inst.instance_id, record_capacity=cap,
                  final_state=True)
    assert max(len(j) for j in ref.jumps) < cap
    frac, worst = compare_jump_records(res["jumps"], res["jump_count"], ref.jumps, inst.t_f)
    assert frac >= 0.999, (frac, worst)
    np.testing.assert_array_equal(res["jump_totals"], ref.kind_totals)
    np.testing.assert_array_equal(res["net_gs"], ref.net_gs)
    np.testing.assert_allclose(res["pgs_sum"], ref.pgs_sum, rtol=1e-9, atol=1e-9)
    pop_gpu = (res["final_state"] ** 2).sum(axis=2).T
    np.testing.assert_allclose(pop_gpu, np.abs(ref.final_state) ** 2, atol=1e-9)
    hist = np.bincount(np.clip(ref.net_gs, -64, 64) + 64, minlength=129)
    np.testing.assert_array_equal(res["net_hist"], hist)


@pytest.mark.parametrize("K,offset", [(1, 0), (37, 5), (16, 1000)])
def test_ragged_and_offset_tiles(small, K, offset):
    inst, tabs = small
    ref = trajectories.run(tabs, inst, K, traj_offset=offset)
    eng = engine_with_oracle_tables(inst, tabs)
    res = eng.run(K, "fp64", seed=inst.seed, traj_offset=offset, record_capacity=64)
    frac, _ = compare_jump_records(res["jumps"], res["jump_count"], ref.jumps, inst.t_f)
    assert frac == 1.0
    np.testing.assert_allclose(res["pgs_sum"], ref.pgs_sum, rtol=1e-9, atol=1e-9)


@pytest.mark.parametrize("tile", [8, 16, 32, 64])
def test_tile_shape_does_not_change_results(small, tile):
    inst, tabs = small
    eng = engine_with_oracle_tables(inst, tabs)
    a = eng.run(200, "fp64", seed=3, record_capacity=64)
    b = eng.run(200, "fp64", seed=3, record_capacity=64, tile=tile)
    np.testing.assert_array_equal(a["jump_count"], b["jump_count"])
    np.testing.assert_array_equal(a["jumps"], b["jumps"])
    np.testing.assert_allclose(a["pgs_sum"], b["pgs_sum"], rtol=1e-13)


def test_record_capacity_overflow_keeps_counts(small):
    inst, tabs = small
    eng = engine_with_oracle_tables(inst, tabs)
    full = eng.run(300, "fp64", seed=9, record_capacity=64)
    part = eng.run(300, "fp64", seed=9, record_capacity=1)
    np.testing.assert_array_equal(full["jump_count"], part["jump_count"])
    has = full["jump_count"] > 0
    np.testing.assert_array_equal(part["jumps"][has, 0], full["jumps"][has, 0])
    # the overflow is reported through the context's run status (aqt_run_status)
    assert full["jump_count"].max() > 1
    assert not full["records_truncated"] and part["records_truncated"]


def test_step_decay_beyond_the_precision_is_rejected():
    """Rates far too large for the step (Gamma dt about 4e4): the decay of one step
    underflows the state, so every run entry point refuses the tables with AQT_ENUMERIC
    instead of stepping; a grid fine enough for the rates runs."""
    from paper_1710_03431_amd.binding import AQT_ENUMERIC, AqtError
    inst = W.two_level_fixed(A=0.3, t_f=1.0e4, n_grid=3, eta=1.0)
    tabs = spectrum.all_tables(inst)
    assert tabs[-1].Gamma.max() * tabs[-1].dt > 1e4
    eng = engine_with_oracle_tables(inst, tabs)
    for prec in ("fp64", "fp32"):
        with pytest.raises(AqtError) as e:
            eng.run(8, prec, seed=1)
        assert e.value.status == AQT_ENUMERIC
        with pytest.raises(AqtError) as e:
            eng.run_fixed_step(8, 2, prec, seed=1)
        assert e.value.status == AQT_ENUMERIC
    fine = inst.with_(t_f=200.0, n_grid=101)
    eng2 = engine_with_oracle_tables(fine, spectrum.all_tables(fine))
    res = eng2.run(64, "fp32", seed=1)
    assert res["jump_totals"].sum() > 64 and np.all(np.isfinite(res["pgs_sum"]))


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_mixed_precision_matches_ame(prec):
    """5-qubit ring (n = 32): trajectory mean within 3 sigma + 1e-4 of the split-step AME."""
    inst = W.ring_instance(5, 1001, t_f=1000.0, n_grid=801)
    tabs = spectrum.all_tables(inst)
    P = ame.split_step(tabs, inst)
    eng = engine_with_oracle_tables(inst, tabs)
    K = 4000
    res = eng.run(K, prec, seed=11)
    m, se = trajectories.mean_and_stderr(res["pgs_sum"], res["pgs_sumsq"], K)
    assert np.all(np.abs(m - P) <= 3 * sigma_bound(P, se, K) + 1e-4)
    # the same draws in FP64 give nearly the same jump counts
    r64 = eng.run(K, "fp64", seed=11)
    same = np.mean(res["jump_count"] == r64["jump_count"])
    assert same > 0.95


def test_fp32_matches_ame_small(small):
    inst, tabs = small
    P = ame.split_step(tabs, inst)
    eng = engine_with_oracle_tables(inst, tabs)
    K = 4000
    res = eng.run(K, "fp32", seed=21)
    m, se = trajectories.mean_and_stderr(res["pgs_sum"], res["pgs_sumsq"], K)
    assert np.all(np.abs(m - P) <= 3 * sigma_bound(P, se, K) + 1e-4)
