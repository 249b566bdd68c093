"""Fixed-step unraveling (App. B) on the GPU against the FP64 oracle's fixed-step code."""
import numpy as np
import pytest

import workloads as W
from oracle import ame, spectrum, trajectories

from gpu_common import compare_jump_records, sigma_bound

pytestmark = pytest.mark.gpu


def _engine(inst):
    from paper_1710_03431_amd.binding import Engine
    eng = Engine(0)
    eng.set_instance(inst)
    eng.precompute(inst.n_grid, inst.levels)
    return eng


@pytest.fixture(scope="module")
def fast():
    inst = W.ring_instance(3, 8, t_f=1.5, eta=0.1, n_grid=101)
    return inst, spectrum.all_tables(inst)


def test_fixed_step_fp64_per_trajectory(fast):
    """Same draws: identical jump sequences (sub-step start times) and final states."""
    inst, tabs = fast
    K, S = 300, 4
    ref = trajectories.run_fixed_step(tabs, inst, K, S)
    eng = _engine(inst)
    res = eng.run_fixed_step(K, S, "fp64", seed=inst.seed, instance_id=inst.instance_id, record_capacity=64,
                             final_state=True)
    frac, worst = compare_jump_records(res["jumps"], res["jump_count"], ref.jumps, inst.t_f)
    assert frac >= 0.99, (frac, worst)
    assert ref.kind_totals.sum() > K
    same = [j for j in range(K) if res["jump_count"][j] == len(ref.jumps[j])]
    pop = (res["final_state"] ** 2).sum(axis=2).T
    np.testing.assert_allclose(pop[:, same], (np.abs(ref.final_state) ** 2)[:, same], atol=1e-9)
    if frac == 1.0:
        np.testing.assert_array_equal(res["jump_totals"], ref.kind_totals)
        np.testing.assert_array_equal(res["net_gs"], ref.net_gs)
        np.testing.assert_allclose(res["pgs_sum"], ref.pgs_sum, rtol=1e-9)


def test_fixed_step_two_level_chain():
    """10^6 FP32 trajectories of the frozen two-level system follow the discrete chain of
    the fixed-step law and are excluded from the AME's exponential relaxation."""
    inst = W.two_level_fixed(A=0.3, t_f=20.0, n_grid=11, eta=1e-2)
    tabs = spectrum.all_tables(inst)
    S, K = 2, 1_000_000
    res = _engine(inst).run_fixed_step(K, S, "fp32", seed=inst.seed, instance_id=inst.instance_id)
    T = tabs[0]
    W10, W01 = T.R[:, 0, 1].sum(), T.R[:, 1, 0].sum()
    h = inst.t_f / (inst.n_grid - 1) / S
    p, chain = 1.0, [1.0]
    for _ in range(1, inst.n_grid):
        for _ in range(S):
            p = p * (1 - h * W10) + (1 - p) * h * W01
        chain.append(p)
    chain = np.array(chain)
    m, se = trajectories.mean_and_stderr(res["pgs_sum"], res["pgs_sumsq"], K)
    assert np.all(np.abs(m - chain)[1:] <= 3 * se[1:] + 1e-6)
    P = ame.split_step(tabs, inst)
    assert np.max(np.abs(m - P)[1:] / se[1:]) > 20


def test_fixed_step_converges_to_the_ame():
    """First order in h (coarse grid, 20 steps): with 64 sub-steps per grid step the mean of
    10^6 FP32 trajectories sits on the split-step AME, with one it is visibly off."""
    inst = W.ring_instance(3, 8, t_f=1.5, eta=0.1, n_grid=21)
    P = ame.split_step(spectrum.all_tables(inst), inst)
    eng = _engine(inst)
    K = 1_000_000
    err = {}
    for S in (1, 64):
        res = eng.run_fixed_step(K, S, "fp32", seed=inst.seed + S, instance_id=inst.instance_id)
        m, se = trajectories.mean_and_stderr(res["pgs_sum"], res["pgs_sumsq"], K)
        sig = sigma_bound(P, se, K)
        err[S] = np.max(np.abs(m - P)[1:] / sig[1:])
    assert err[64] <= 4.0, err
    assert err[1] > 10.0, err


def test_fixed_step_argument_errors(fast):
    from paper_1710_03431_amd.binding import AqtError
    inst, _ = fast
    eng = _engine(inst)
    with pytest.raises(AqtError):
        eng.run_fixed_step(8, 0, "fp64")
    with pytest.raises(AqtError):
        eng.run_fixed_step(8, 2, "bf16")



@pytest.fixture(scope="module", params=[7, 8], ids=["n128", "n256"])
def full_fixed(request):
    """128 and 256 levels (2 and 4 levels per lane in the sub-step loop, whose scans carry
    across lane chunks), 4 sub-steps per grid step, 1003 trajectories, oracle tables."""
    nq = request.param
    inst = W.pm1_all_to_all(nq, 10 + nq - 5, t_f=1.0e4, n_grid=120)
    tabs = spectrum.all_tables(inst)
    K, S = 1003, 4
    ref = trajectories.run_fixed_step(tabs, inst, K, S)
    return inst, tabs, ref, K, S


def test_fixed_step_fp64_per_trajectory_full_spectrum(full_fixed):
    """Identical jump sequences in >= 99.9% of trajectories, final populations of those,
    sums and totals through the differing ones."""
    from gpu_common import engine_with_oracle_tables
    inst, tabs, ref, K, S = full_fixed
    assert ref.kind_totals[0] > 0 and ref.kind_totals[1] > 0
    cap = max(len(j) for j in ref.jumps) + 1
    eng = engine_with_oracle_tables(inst, tabs)
    res = eng.run_fixed_step(K, S, "fp64", seed=inst.seed, instance_id=inst.instance_id, record_capacity=cap,
                             final_state=True)
    frac, worst = compare_jump_records(res["jumps"], res["jump_count"], ref.jumps, inst.t_f)
    assert frac >= 0.999, (frac, worst)
    bad = int(round((1.0 - frac) * K))
    assert np.abs(res["pgs_sum"] - ref.pgs_sum).max() <= bad + 1e-9 * K
    same = [j for j in range(K) if res["jump_count"][j] == len(ref.jumps[j])]
    pop = (res["final_state"] ** 2).sum(axis=2).T
    np.testing.assert_allclose(pop[:, same], (np.abs(ref.final_state) ** 2)[:, same], atol=1e-9)
    if bad == 0:
        np.testing.assert_array_equal(res["jump_totals"], ref.kind_totals)
        np.testing.assert_array_equal(res["net_gs"], ref.net_gs)


def test_fixed_step_fp32_full_spectrum_follows_oracle(full_fixed):
    """FP32 (the benchmarked precision) on the oracle's draws: at least 97% of the
    trajectories repeat the oracle's jump channels with sub-step start times to 1e-4
    relative; the population sums move only through the others."""
    from gpu_common import engine_with_oracle_tables
    inst, tabs, ref, K, S = full_fixed
    cap = max(len(j) for j in ref.jumps) + 1
    eng = engine_with_oracle_tables(inst, tabs)
    res = eng.run_fixed_step(K, S, "fp32", seed=inst.seed, instance_id=inst.instance_id, record_capacity=cap)
    frac, _ = compare_jump_records(res["jumps"], res["jump_count"], ref.jumps, inst.t_f, rel=1e-4)
    assert frac >= 0.97, frac
    assert np.abs(res["pgs_sum"] - ref.pgs_sum).max() <= (1.0 - frac) * K + 1e-4 * K
