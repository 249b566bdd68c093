"""Frequency-dependent bath correlations, gamma_ab(w) = sum_m C_m[a, b] gamma(w; omega_c,m),
on the GPU against the FP64 oracle.

The oracle builds one jump channel per kept column of each term's semidefinite
Cholesky factor, each with its term's cutoff, and is pinned to the double-sum form of
the master equation with gamma_ab(w) taken from its definition; the GPU forms the same
channel couplings as weighted products over the eigenvectors and rates with per-channel
cutoffs.  The case used here has non-commuting terms (the eigenvectors of gamma(w) turn
with w) and a rank-one shared bath (one channel for it).
"""
import numpy as np
import pytest

import workloads as W
from oracle import ame, spectrum, trajectories

from gpu_common import compare_jump_records, sigma_bound

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def terms_case():
    inst = W.ring_instance(3, 8, t_f=1.5, eta=0.1, n_grid=101, bath_terms=W.two_term_bath(3, rho=0.8))
    return inst, spectrum.all_tables(inst)


def _engine(inst):
    from paper_1710_03431_amd.binding import Engine
    eng = Engine(0)
    eng.set_instance(inst)
    eng.precompute(inst.n_grid, inst.levels)
    return eng


def test_bath_terms_channel_tables(terms_case):
    inst, tabs = terms_case
    eng = _engine(inst)
    assert eng.channel_count() == tabs[1].R.shape[0] == 4
    got = eng.get_tables(("R", "zdiag", "Gamma"))
    rmax = max(np.abs(T.R).max() for T in tabs)
    for T in tabs:
        np.testing.assert_allclose(got["R"][T.g], T.R, rtol=0, atol=1e-12 * rmax)
        np.testing.assert_allclose(got["zdiag"][T.g], T.zdiag, rtol=0, atol=1e-12)
        np.testing.assert_allclose(got["Gamma"][T.g], T.Gamma, rtol=1e-12, atol=1e-15)


def test_bath_terms_fp64_per_trajectory(terms_case):
    """Same Philox draws: the same channels, targets and jump times as the oracle."""
    inst, tabs = terms_case
    K = 400
    ref = trajectories.run(tabs, inst, K)
    res = _engine(inst).run(K, "fp64", seed=inst.seed, instance_id=inst.instance_id, record_capacity=32)
    frac, worst = compare_jump_records(res["jumps"], res["jump_count"], ref.jumps, inst.t_f)
    assert frac >= 0.99, (frac, worst)
    assert max(int(j["qubit"]) for r, c in zip(res["jumps"], res["jump_count"]) for j in r[:c]) == 3


def test_bath_terms_average_matches_ame(terms_case):
    """10^6 FP32 trajectories within 3 sigma + 1e-4 of the split-step AME at every grid
    point, and far from the same local baths without the shared term."""
    inst, tabs = terms_case
    P = ame.split_step(tabs, inst)
    local = inst.with_(bath_terms=None, bath_corr=inst.bath_terms[0][0])
    P0 = ame.split_step(spectrum.all_tables(local), local)
    K = 1_000_000
    res = _engine(inst).run(K, "fp32", seed=inst.seed + 9, instance_id=inst.instance_id)
    m, se = trajectories.mean_and_stderr(res["pgs_sum"], res["pgs_sumsq"], K)
    sig = sigma_bound(P, se, K)
    assert np.all(np.abs(m - P) <= 3 * sig + 1e-4)
    assert np.max(np.abs(m - P0)[1:] / sig[1:]) > 8


def test_bath_terms_fixed_step_per_trajectory(terms_case):
    inst, tabs = terms_case
    K, S = 200, 3
    ref = trajectories.run_fixed_step(tabs, inst, K, S)
    res = _engine(inst).run_fixed_step(K, S, "fp64", seed=inst.seed, instance_id=inst.instance_id,
                                       record_capacity=64)
    frac, worst = compare_jump_records(res["jumps"], res["jump_count"], ref.jumps, inst.t_f)
    assert frac >= 0.99, (frac, worst)


def test_bath_terms_gradient_per_trajectory(terms_case):
    """Per-trajectory gradient estimates with the per-term channels (each rate's
    derivative with its own cutoff) against the oracle's path-weight differences."""
    _gradient_matches_oracle_per_trajectory(terms_case[0])


def test_bath_terms_with_lamb_shift():
    """Lamb shift with per-term cutoffs (one S table per cutoff): shifts against the
    oracle's quadrature, and FP64 trajectories against the oracle's."""
    inst = W.ring_instance(3, 8, t_f=1.5, eta=0.1, n_grid=41, bath_terms=W.two_term_bath(3, rho=0.8),
                           lamb_shift=True)
    tabs = spectrum.all_tables(inst)
    eng = _engine(inst)
    got = eng.get_lamb_shift()
    scale = max(np.abs(T.shift).max() for T in tabs)
    assert scale > 1.0
    for T in tabs:
        np.testing.assert_allclose(got[T.g], T.shift, rtol=0, atol=1e-9 * scale)
    K = 300
    ref = trajectories.run(tabs, inst, K)
    res = eng.run(K, "fp64", seed=inst.seed, instance_id=inst.instance_id, record_capacity=32)
    frac, worst = compare_jump_records(res["jumps"], res["jump_count"], ref.jumps, inst.t_f)
    assert frac >= 0.99, (frac, worst)


def test_bath_terms_argument_errors():
    from paper_1710_03431_amd.binding import AqtError, Engine
    inst = W.ring_instance(3, 8, t_f=1.5, eta=0.1, n_grid=21)
    eng = Engine(0)
    eng.set_instance(inst)
    C0, C1 = np.eye(3), np.ones((3, 3))
    with pytest.raises(AqtError):
        eng.set_bath_terms(((C0, 8.0), (np.diag([1.0, -1.0, 1.0]), 2.0)))    # not semidefinite
    with pytest.raises(AqtError):
        eng.set_bath_terms(((C0, 0.0),))                                      # cutoff
    with pytest.raises(AqtError):
        eng.set_bath_terms(((np.array([[1.0, 0.2, 0.0], [0.3, 1.0, 0.0], [0.0, 0.0, 1.0]]), 8.0),))
    eng.set_bath_terms(((C0, 8.0), (C1, 2.0)))
    assert eng.channel_count() == 4
    eng.precompute(21, 8)
    # channels beyond the padded level count (16 here): six full-rank terms, 18 channels
    eng.set_bath_terms(tuple((C0, 8.0 + m) for m in range(6)))
    assert eng.channel_count() == 18
    with pytest.raises(AqtError):
        eng.precompute(21, 8)
    # no terms: the independent baths again, bit for bit
    eng.set_bath_terms(None)
    eng.precompute(21, 8)
    a = eng.get_tables(("R",))["R"]
    plain = Engine(0)
    plain.set_instance(inst)
    plain.precompute(21, 8)
    np.testing.assert_array_equal(a, plain.get_tables(("R",))["R"])


def _gradient_matches_oracle_per_trajectory(inst, K=48):
    from oracle import gradient
    A, B = W.linear_schedule(3)
    inst = inst.with_(A_ctrl=A, B_ctrl=B)
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
