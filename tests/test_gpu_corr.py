"""Correlated baths (gamma_ab(w) = C_ab gamma(w)) on the GPU against the FP64 oracle.

The oracle builds the jump channels from the Cholesky factor of C and is pinned to
the double-sum form of the master equation (no factorisation); the GPU forms the
same channel couplings as weighted products over the eigenvectors.
"""
import numpy as np
import pytest

import workloads as W
from oracle import ame, gradient, spectrum, trajectories

from gpu_common import compare_jump_records, sigma_bound

pytestmark = pytest.mark.gpu

C3 = np.array([[0.5 ** abs(i - j) for j in range(3)] for i in range(3)])


@pytest.fixture(scope="module")
def corr_case():
    inst = W.ring_instance(3, 8, t_f=1.5, eta=0.1, n_grid=101, bath_corr=C3)
    return inst, spectrum.all_tables(inst)


def _engine(inst):
    from paper_1710_03431_amd.binding import Engine
    eng = Engine(0)
    eng.set_instance(inst)
    eng.precompute(inst.n_grid, inst.levels)
    return eng


def test_correlated_channel_tables(corr_case):
    inst, tabs = corr_case
    got = _engine(inst).get_tables(("R", "zdiag", "Gamma"))
    rmax = max(np.abs(T.R).max() for T in tabs)
    for T in tabs:
        np.testing.assert_allclose(got["R"][T.g], T.R, rtol=0, atol=1e-12 * rmax)
        np.testing.assert_allclose(got["zdiag"][T.g], T.zdiag, rtol=0, atol=1e-12)
        np.testing.assert_allclose(got["Gamma"][T.g], T.Gamma, rtol=1e-12, atol=1e-15)
    plain = _engine(inst.with_(bath_corr=None)).get_tables(("R",))
    assert np.abs(plain["R"] - got["R"]).max() > 1e-2 * rmax


def test_correlated_fp64_per_trajectory(corr_case):
    inst, tabs = corr_case
    K = 400
    ref = trajectories.run(tabs, inst, K)
    res = _engine(inst).run(K, "fp64", seed=inst.seed, instance_id=inst.instance_id, record_capacity=32)
    frac, worst = compare_jump_records(res["jumps"], res["jump_count"], ref.jumps, inst.t_f)
    assert frac >= 0.99, (frac, worst)


def test_correlated_average_matches_ame(corr_case):
    inst, tabs = corr_case
    P = ame.split_step(tabs, inst)
    plain = inst.with_(bath_corr=None)
    P0 = ame.split_step(spectrum.all_tables(plain), plain)
    K = 1_000_000
    res = _engine(inst).run(K, "fp32", seed=inst.seed + 9, instance_id=inst.instance_id)
    m, se = trajectories.mean_and_stderr(res["pgs_sum"], res["pgs_sumsq"], K)
    sig = sigma_bound(P, se, K)
    assert np.all(np.abs(m - P) <= 3 * sig + 1e-4)
    assert np.max(np.abs(m - P0)[1:] / sig[1:]) > 8   # grid 0 is the initial state


def test_correlated_gradient_per_trajectory(corr_case):
    inst, _ = corr_case
    A, B = W.linear_schedule(3)
    inst = inst.with_(A_ctrl=A, B_ctrl=B)
    K = 48
    ref = gradient.trajectory_gradients(inst, K)
    eng = _engine(inst)
    out = eng.grad_pgs(K, "fp64", seed=inst.seed, instance_id=inst.instance_id, per_trajectory=True)
    pt = out["per_traj"]
    P = pt.shape[1] // 2 - 1
    res = eng.run(K, "fp64", seed=inst.seed, instance_id=inst.instance_id, record_capacity=32)
    same = [j for j in range(K)
            if compare_jump_records(res["jumps"][j:j + 1], res["jump_count"][j:j + 1], ref["jumps"][j:j + 1],
                                    inst.t_f)[0] == 1.0]
    assert len(same) >= K - 2
    for got, want in ((pt[same, 1:P + 1], ref["g"][same]), (pt[same, P + 2:], ref["score"][same])):
        scale = np.maximum(np.abs(want).max(axis=0), 1e-3)
        assert (np.abs(got - want) / scale).max() <= 2e-6


def test_correlation_argument_errors():
    from paper_1710_03431_amd.binding import AqtError, Engine
    eng = Engine(0)
    inst = W.ring_instance(3, 8, t_f=1.5, eta=0.1, n_grid=21)
    eng.set_instance(inst)
    with pytest.raises(AqtError):
        eng.set_bath_correlation(np.array([[1.0, 0.2, 0.0], [0.3, 1.0, 0.0], [0.0, 0.0, 1.0]]))   # not symmetric
    with pytest.raises(AqtError):
        eng.set_bath_correlation(np.ones((3, 3)))                                                # singular
    eng.set_bath_correlation(np.eye(3))
    eng.precompute(21, 8)
    a = eng.get_tables(("R",))["R"]
    eng.set_bath_correlation(None)
    eng.precompute(21, 8)
    np.testing.assert_array_equal(eng.get_tables(("R",))["R"], a)
