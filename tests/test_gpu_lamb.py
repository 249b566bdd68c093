"""Lamb shift (Sec. II eq. ME2-H) on the GPU against the FP64 oracle.

The oracle evaluates S(w) by adaptive quadrature of the principal-value integral
for every Bohr frequency (pinned to the zero-temperature closed form and to
S(0) = -eta wc); the GPU tabulates S once per precompute and interpolates.
"""
import numpy as np
import pytest

import workloads as W
from oracle import ame, spectrum, trajectories

from gpu_common import compare_jump_records, sigma_bound

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lamb_case():
    """Fast, strongly coupled 3-qubit anneal: shifts of several rad/ns that move P_GS."""
    inst = W.ring_instance(3, 8, t_f=1.5, eta=0.1, n_grid=101, lamb_shift=True)
    return inst, spectrum.all_tables(inst)


def _engine(inst):
    from paper_1710_03431_amd.binding import Engine
    eng = Engine(0)
    eng.set_instance(inst)
    eng.precompute(inst.n_grid, inst.levels)
    return eng


def test_lamb_shift_tables(lamb_case):
    inst, tabs = lamb_case
    eng = _engine(inst)
    got = eng.get_lamb_shift()
    scale = max(np.abs(T.shift).max() for T in tabs)
    assert scale > 1.0
    for T in tabs:
        np.testing.assert_allclose(got[T.g], T.shift, rtol=0, atol=1e-9 * scale)
    np.testing.assert_array_equal(got[0], 0.0)
    eng.set_lamb_shift(False)
    eng.precompute(inst.n_grid, inst.levels)
    np.testing.assert_array_equal(eng.get_lamb_shift(), 0.0)


def test_lamb_shift_fp64_per_trajectory(lamb_case):
    inst, tabs = lamb_case
    K = 400
    ref = trajectories.run(tabs, inst, K)
    eng = _engine(inst)
    res = eng.run(K, "fp64", seed=inst.seed, instance_id=inst.instance_id, record_capacity=32, final_state=True)
    frac, worst = compare_jump_records(res["jumps"], res["jump_count"], ref.jumps, inst.t_f)
    assert frac >= 0.99, (frac, worst)
    np.testing.assert_allclose(res["pgs_sum"], ref.pgs_sum, atol=K * (1 - frac) + 1e-6 * K)


def test_lamb_shift_average_matches_ame(lamb_case):
    """10^6 FP32 trajectories against the split-step AME with H_LS at every grid point;
    the same AME without H_LS is excluded at some grid point (the shift is resolved)."""
    inst, tabs = lamb_case
    P = ame.split_step(tabs, inst)
    plain = inst.with_(lamb_shift=False)
    P0 = ame.split_step(spectrum.all_tables(plain), plain)
    eng = _engine(inst)
    K = 1_000_000
    res = eng.run(K, "fp32", seed=inst.seed + 5, instance_id=inst.instance_id)
    m, se = trajectories.mean_and_stderr(res["pgs_sum"], res["pgs_sumsq"], K)
    sig = sigma_bound(P, se, K)
    assert np.all(np.abs(m - P) <= 3 * sig + 1e-4)
    assert np.max(np.abs(m - P0)[1:] / sig[1:]) > 8   # grid 0 is the initial state, P = 1 exactly


def test_lamb_shift_gradient_per_trajectory():
    """Gradient with the Lamb shift on (2-qubit ring, 3 + 3 controls): per-trajectory FP64
    estimates against the oracle's central differences of each path's log weight, whose
    perturbed tables re-evaluate S(w) by quadrature; the GPU differentiates the
    interpolated S table and scales the shift with eta."""
    from oracle import gradient
    A, B = W.linear_schedule(3)
    inst = W.ring_instance(2, 5, t_f=1.5, eta=0.1, n_grid=21, A_ctrl=A, B_ctrl=B, lamb_shift=True)
    K = 32
    ref = gradient.trajectory_gradients(inst, K)
    eng = _engine(inst)
    out = eng.grad_pgs(K, "fp64", seed=inst.seed, instance_id=inst.instance_id, per_trajectory=True)
    pt = out["per_traj"]
    P = pt.shape[1] // 2 - 1
    res = eng.run(K, "fp64", seed=inst.seed, instance_id=inst.instance_id, record_capacity=32)
    same = [j for j in range(K)
            if compare_jump_records(res["jumps"][j:j + 1], res["jump_count"][j:j + 1], ref["jumps"][j:j + 1],
                                    inst.t_f)[0] == 1.0]
    assert len(same) >= K - 1
    np.testing.assert_allclose(pt[same, 0], ref["f"][same], atol=1e-10)
    for got, want in ((pt[same, 1:P + 1], ref["g"][same]), (pt[same, P + 2:], ref["score"][same])):
        scale = np.maximum(np.abs(want).max(axis=0), 1e-3)
        err = np.abs(got - want) / scale
        assert err.max() <= 2e-6, (err.max(axis=0), np.unravel_index(err.argmax(), err.shape))
