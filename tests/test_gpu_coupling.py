"""Coupling operators other than sz on the GPU against the FP64 oracle.

Channel k couples through sum_a (cz[k][a] sz_a + cx[k][a] sx_a) to its own Ohmic bath.
The oracle applies sx as a row permutation of the eigenvectors and is pinned to the
Lindblad form built from dense Kronecker-product Pauli matrices and to the two-level
closed form; the GPU builds the operands O_k V in one kernel and multiplies by V^T.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import ame, spectrum, trajectories

from gpu_common import compare_jump_records, sigma_bound

pytestmark = pytest.mark.gpu

CZ = np.array([[1.0, 0.0, 0.0], [0.0, 0.7, 0.0], [0.0, 0.0, 0.0], [0.5, 0.0, -0.5]])
CX = np.array([[0.0, 0.0, 0.0], [0.0, 0.7, 0.0], [0.0, 0.0, 1.0], [0.0, 0.4, 0.0]])
WC = np.array([8.0 * math.pi, 8.0 * math.pi, 3.0, 8.0 * math.pi])


@pytest.fixture(scope="module")
def mixed_case():
    inst = W.ring_instance(3, 8, t_f=1.5, eta=0.1, n_grid=101, coupling=(CZ, CX, WC))
    return inst, spectrum.all_tables(inst)


def _engine(inst):
    from paper_1710_03431_amd.binding import Engine
    eng = Engine(0)
    eng.set_instance(inst)
    eng.precompute(inst.n_grid, inst.levels)
    return eng


def test_coupling_channel_tables(mixed_case):
    inst, tabs = mixed_case
    eng = _engine(inst)
    assert eng.channel_count() == 4
    got = eng.get_tables(("R", "zdiag", "Gamma"))
    rmax = max(np.abs(T.R).max() for T in tabs)
    for T in tabs:
        np.testing.assert_allclose(got["R"][T.g], T.R, rtol=0, atol=1e-12 * rmax)
        np.testing.assert_allclose(got["zdiag"][T.g], T.zdiag, rtol=0, atol=1e-12)
        np.testing.assert_allclose(got["Gamma"][T.g], T.Gamma, rtol=1e-12, atol=1e-15)


def test_coupling_fp64_per_trajectory(mixed_case):
    inst, tabs = mixed_case
    K = 400
    ref = trajectories.run(tabs, inst, K)
    res = _engine(inst).run(K, "fp64", seed=inst.seed, instance_id=inst.instance_id, record_capacity=32)
    frac, worst = compare_jump_records(res["jumps"], res["jump_count"], ref.jumps, inst.t_f)
    assert frac >= 0.99, (frac, worst)


def test_coupling_average_matches_ame(mixed_case):
    """10^6 FP32 trajectories within 3 sigma + 1e-4 of the split-step AME, and far from
    the default sz couplings."""
    inst, tabs = mixed_case
    P = ame.split_step(tabs, inst)
    plain = inst.with_(coupling=None)
    P0 = ame.split_step(spectrum.all_tables(plain), plain)
    K = 1_000_000
    res = _engine(inst).run(K, "fp32", seed=inst.seed + 9, instance_id=inst.instance_id)
    m, se = trajectories.mean_and_stderr(res["pgs_sum"], res["pgs_sumsq"], K)
    sig = sigma_bound(P, se, K)
    assert np.all(np.abs(m - P) <= 3 * sig + 1e-4)
    assert np.max(np.abs(m - P0)[1:] / sig[1:]) > 8


@pytest.fixture(scope="module")
def wide_case():
    """Twenty channels on a 5-qubit ring kept at all 32 levels: a crossing is handled
    by 16 lanes, so the channel draw spans two chunks of lanes."""
    nq, nch = 5, 20
    rng = np.random.default_rng(5)
    cz, cx = np.zeros((nch, nq)), np.zeros((nch, nq))
    for k in range(nq):
        cz[k, k] = 1.0
        cx[nq + k, k] = 1.0
    cz[2 * nq:] = rng.uniform(-0.5, 0.5, (nch - 2 * nq, nq))
    cx[2 * nq:] = rng.uniform(-0.5, 0.5, (nch - 2 * nq, nq))
    inst = W.ring_instance(nq, 8, t_f=1.5, eta=0.1, n_grid=101, coupling=(cz, cx, np.full(nch, 8.0 * math.pi)))
    return inst, spectrum.all_tables(inst)


def test_more_channels_than_handler_lanes_per_trajectory(wide_case):
    """FP64 jump records against the oracle trajectory by trajectory; channels beyond
    the first 16 are among those drawn."""
    inst, tabs = wide_case
    K = 400
    ref = trajectories.run(tabs, inst, K)
    eng = _engine(inst)
    assert eng.channel_count() == 20
    res = eng.run(K, "fp64", seed=inst.seed, instance_id=inst.instance_id, record_capacity=64)
    frac, worst = compare_jump_records(res["jumps"], res["jump_count"], ref.jumps, inst.t_f)
    assert frac >= 0.99, (frac, worst)
    drawn = {int(res["jumps"][j, m]["qubit"]) for j in range(K) for m in range(min(int(res["jump_count"][j]), 64))}
    assert max(drawn) >= 16 and len(drawn) == 20, sorted(drawn)


def test_more_channels_than_handler_lanes_average(wide_case):
    """10^5 FP32 trajectories of the same instance within 3 sigma + 1e-4 of the split-step AME."""
    inst, tabs = wide_case
    P = ame.split_step(tabs, inst)
    K = 100_000
    res = _engine(inst).run(K, "fp32", seed=inst.seed + 3, instance_id=inst.instance_id)
    m, se = trajectories.mean_and_stderr(res["pgs_sum"], res["pgs_sumsq"], K)
    assert np.all(np.abs(m - P) <= 3 * sigma_bound(P, se, K) + 1e-4)


def test_sx_coupling_of_a_fixed_sx_hamiltonian_only_dephases():
    """H = -A sx fixed and coupling sx: the coupling commutes with H, every jump is an
    omega = 0 jump and the ground-state population stays 1."""
    inst = W.two_level_fixed(A=0.3, t_f=200.0, n_grid=41, eta=2e-2, coupling=([[0.0]], [[1.0]], None))
    res = _engine(inst).run(20000, "fp64", seed=inst.seed, instance_id=inst.instance_id)
    tot = np.asarray(res["jump_totals"])
    assert tot[0] == 0 and tot[1] == 0 and tot[2] > 1000
    np.testing.assert_allclose(np.asarray(res["pgs_sum"]) / 20000, 1.0, atol=1e-12)


def test_coupling_gradient_per_trajectory(mixed_case):
    """Per-trajectory gradient estimates with sz/sx channel operators (dz = z X - X z
    for any fixed operator) against the oracle's path-weight differences."""
    _gradient_matches_oracle_per_trajectory(mixed_case[0])


def test_coupling_argument_errors():
    from paper_1710_03431_amd.binding import AqtError, Engine
    inst = W.ring_instance(3, 8, t_f=1.5, eta=0.1, n_grid=21)
    eng = Engine(0)
    eng.set_instance(inst)
    with pytest.raises(AqtError):
        eng.set_coupling(np.zeros((2, 3)), np.array([[1.0, 0, 0], [0, 0, 0]]))       # channel 1 is zero
    with pytest.raises(AqtError):
        eng.set_coupling(np.eye(3), None, [1.0, -1.0, 2.0])                           # cutoff
    with pytest.raises(AqtError):
        eng.set_coupling(np.ones((65, 3)))                                            # too many channels
    eng.set_coupling(CZ, CX, WC)
    eng.precompute(21, 8)
    # cz = I, no sx part: the default channels bit for bit
    eng.set_coupling(np.eye(3))
    eng.precompute(21, 8)
    a = eng.get_tables(("R",))["R"]
    eng.set_coupling(None, None)
    eng.precompute(21, 8)
    np.testing.assert_allclose(a, eng.get_tables(("R",))["R"], rtol=1e-14, atol=1e-300)


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
