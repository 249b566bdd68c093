"""Parity of the HIP adjoint gradient (aqt_grad_pgs) with the FP64 oracle.

The oracle's per-trajectory estimates are central differences of each path's own
log weight (jump times and channels held fixed), rebuilt from perturbed tables;
its mean is pinned to the central differences of the split-step AME.  The GPU
evaluates the same estimator by an adjoint sweep, so in FP64 the two agree per
trajectory wherever the jump sequences agree, and the FP32 mean agrees with the
AME differences within the statistical error.
"""
import numpy as np
import pytest

import workloads as W
from oracle import gradient

from gpu_common import compare_jump_records

pytestmark = pytest.mark.gpu


def _engine(inst):
    from paper_1710_03431_amd.binding import Engine
    eng = Engine(0)
    eng.set_instance(inst)
    eng.precompute(inst.n_grid, inst.levels)
    return eng


def _ring3(n_ctrl=3):
    A, B = W.linear_schedule(n_ctrl)
    return W.ring_instance(3, 8, t_f=1.5, eta=0.1, n_grid=101, A_ctrl=A, B_ctrl=B)


def _matched(eng, inst, K, ref_jumps):
    """Indices of trajectories whose GPU jump sequence equals the oracle's (FP64 run)."""
    cap = max(8, max(len(j) for j in ref_jumps) + 1)
    res = eng.run(K, "fp64", seed=inst.seed, instance_id=inst.instance_id, record_capacity=cap)
    frac, _ = compare_jump_records(res["jumps"], res["jump_count"], ref_jumps, inst.t_f)
    same = []
    for j in range(K):
        one, _ = compare_jump_records(res["jumps"][j:j + 1], res["jump_count"][j:j + 1], ref_jumps[j:j + 1],
                                      inst.t_f)
        if one == 1.0:
            same.append(j)
    return np.array(same), frac


@pytest.mark.parametrize("inst_fn,K", [(_ring3, 96), (lambda: _ring3(5), 48)])
def test_fp64_per_trajectory_gradient(inst_fn, K):
    """3-qubit ring, fast strongly coupled anneal (about two jumps per trajectory, jumps
    from superpositions and omega = 0 jumps): f and every component of g per trajectory."""
    inst = inst_fn()
    ref = gradient.trajectory_gradients(inst, K)
    eng = _engine(inst)
    out = eng.grad_pgs(K, "fp64", seed=inst.seed, instance_id=inst.instance_id, per_trajectory=True)
    pt = out["per_traj"]
    P = pt.shape[1] // 2 - 1
    same, frac = _matched(eng, inst, K, ref["jumps"])
    assert frac >= 0.97 and len(same) >= K - 2, frac
    np.testing.assert_allclose(pt[same, 0], ref["f"][same], atol=1e-11)
    np.testing.assert_array_equal(pt[:, P + 1], 1.0)
    for got, want in ((pt[same, 1:P + 1], ref["g"][same]), (pt[same, P + 2:], ref["score"][same])):
        scale = np.maximum(np.abs(want).max(axis=0), 1e-3)
        err = np.abs(got - want) / scale
        assert err.max() <= 2e-6, (err.max(axis=0), np.unravel_index(err.argmax(), err.shape))
    # host reductions of the same per-trajectory values (control variate with the score)
    g, sc = pt[:, 1:P + 1], pt[:, P + 2:]
    cov = ((g - g.mean(0)) * (sc - sc.mean(0))).sum(0) / (K - 1)
    c = cov / sc.var(axis=0, ddof=1)
    np.testing.assert_allclose(out["value"], pt[:, 0].mean(), rtol=1e-12)
    np.testing.assert_allclose(out["grad"], g.mean(0) - c * sc.mean(0), rtol=1e-9, atol=1e-13)
    np.testing.assert_allclose(out["grad_se"], (g - c * sc).std(axis=0, ddof=1) / np.sqrt(K), rtol=1e-6)


def test_fp64_two_level_gradient_per_trajectory():
    """Fixed two-level relaxation (one qubit, B = 0): no field, so every d/dB_j is zero."""
    inst = W.two_level_fixed(A=0.3, t_f=150.0, n_grid=41, eta=2e-3)
    K = 64
    ref = gradient.trajectory_gradients(inst, K)
    eng = _engine(inst)
    out = eng.grad_pgs(K, "fp64", seed=inst.seed, instance_id=inst.instance_id, per_trajectory=True)
    pt = out["per_traj"]
    P = pt.shape[1] // 2 - 1
    same, frac = _matched(eng, inst, K, ref["jumps"])
    assert len(same) >= K - 1
    for got, want in ((pt[same, 1:P + 1], ref["g"][same]), (pt[same, P + 2:], ref["score"][same])):
        scale = np.maximum(np.abs(want).max(axis=0), 1e-3)
        assert (np.abs(got - want) / scale).max() <= 2e-6
    np.testing.assert_array_equal(pt[:, 3:5], 0.0)
    np.testing.assert_array_equal(pt[:, P + 4:P + 6], 0.0)


@pytest.mark.parametrize("prec,K", [("fp32", 20000), ("fp64", 20000)])
def test_gradient_mean_matches_ame_differences(prec, K):
    """The estimator's mean against central differences of the FP64 split-step AME,
    within 3.5 standard errors per component (plus 1e-3 of the largest component in FP32)."""
    inst = _ring3()
    fd = gradient.fd_gradient(inst)
    ref = np.concatenate([fd["dA"], fd["dB"], [fd["deta"]]])
    eng = _engine(inst)
    out = eng.grad_pgs(K, prec, seed=inst.seed, instance_id=inst.instance_id)
    tol = 3.5 * out["grad_se"] + (1e-3 * np.abs(ref).max() if prec == "fp32" else 1e-5)
    assert np.all(np.abs(out["grad"] - ref) <= tol), (out["grad"], ref, out["grad_se"])
    assert np.sum(np.abs(ref) > 5.0 * out["grad_se"]) >= 4


def test_gradient_argument_errors():
    from paper_1710_03431_amd.binding import AqtError, Engine
    inst = W.ring_instance(3, 8, t_f=1.5, eta=0.1, n_grid=21)
    eng = Engine(0)
    eng.set_instance(inst)
    eng.precompute(21, 4)                     # truncated spectrum
    with pytest.raises(AqtError):
        eng.grad_pgs(16, "fp32")
    eng.precompute(21, 8)
    with pytest.raises(AqtError):
        eng.grad_pgs(16, "bf16")
    with pytest.raises(AqtError):
        eng.grad_pgs(1, "fp32")
    t = eng.get_tables(("E", "gs", "O", "cinit", "R", "zdiag"))
    eng.set_tables(t["E"], t["gs"], t["O"], t["cinit"], t["R"], t["zdiag"])
    with pytest.raises(AqtError):              # no eigenvectors behind host tables
        eng.grad_pgs(16, "fp32")
    eng.precompute(21, 8)
    out = eng.grad_pgs(16, "fp32")
    assert np.all(np.isfinite(out["grad"]))


def test_gradient_matches_stored_ame_differences_4q():
    """4-qubit ring workload with 16 + 16 control points: every component of the FP32
    estimate from 10^5 trajectories against the stored central differences of the FP64
    split-step AME (tests/golden/make_golden.py --grad4) within four standard errors per
    component (33 components: about 0.2% chance of a false alarm)."""
    import json
    import os
    ref = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "small_ctrl16_fd_gradient.json")))
    inst = W.config_small_ctrl(100_000)
    eng = _engine(inst)
    out = eng.grad_pgs(inst.n_traj, "fp32", seed=inst.seed, instance_id=inst.instance_id)
    fd = np.array(ref["grad"])
    assert len(fd) == len(out["grad"])
    tol = 4.0 * out["grad_se"] + 1e-3 * np.abs(fd[:-1]).max() * np.r_[np.ones(len(fd) - 1), 0.0]
    assert np.all(np.abs(out["grad"] - fd) <= tol), (out["grad"], fd, out["grad_se"])
    assert np.sum(np.abs(fd) > 5.0 * out["grad_se"]) >= 5


@pytest.mark.parametrize("segment", [1, 7, 33])
def test_checkpoint_segments_do_not_change_results(segment):
    """The sweep keeps every post-kick state here; forcing checkpoint segments (a forward
    pass storing every segment-th state, then a replay per segment) reproduces the
    same per-trajectory values bit for bit, including a ragged last tile."""
    inst = _ring3()
    eng = _engine(inst)
    K = 40
    a = eng.grad_pgs(K, "fp64", seed=inst.seed, instance_id=inst.instance_id, per_trajectory=True)
    b = eng.grad_pgs(K, "fp64", seed=inst.seed, instance_id=inst.instance_id, per_trajectory=True,
                     segment=segment)
    np.testing.assert_array_equal(a["per_traj"], b["per_traj"])
    c = eng.grad_pgs(K, "fp32", seed=inst.seed, instance_id=inst.instance_id, per_trajectory=True,
                     segment=segment)
    d = eng.grad_pgs(K, "fp32", seed=inst.seed, instance_id=inst.instance_id, per_trajectory=True)
    np.testing.assert_array_equal(c["per_traj"], d["per_traj"])


def test_autograd_function_matches_the_entry_point():
    """The torch.autograd.Function wrapper returns aqt_grad_pgs's value and gradient."""
    import torch
    from paper_1710_03431_amd import binding
    inst = _ring3()
    A = torch.tensor(inst.A_ctrl, dtype=torch.float64, requires_grad=True)
    B = torch.tensor(inst.B_ctrl, dtype=torch.float64, requires_grad=True)
    eta = torch.tensor(inst.eta, dtype=torch.float64, requires_grad=True)
    eng = _engine(inst)
    v = binding.pgs(eng, A, B, eta, t_f=inst.t_f, omega_c=inst.omega_c, T=inst.T, n_grid=inst.n_grid,
                    n_levels=inst.levels, n_traj=4000, precision="fp64", seed=inst.seed)
    (3.0 * v).backward()
    ref = _engine(inst).grad_pgs(4000, "fp64", seed=inst.seed)
    assert abs(float(v) - ref["value"]) <= 1e-12
    m = len(inst.A_ctrl)
    np.testing.assert_allclose(A.grad.numpy(), 3.0 * ref["grad"][:m], rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(B.grad.numpy(), 3.0 * ref["grad"][m:2 * m], rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(float(eta.grad), 3.0 * ref["grad"][2 * m], rtol=1e-12)


def _ring8():
    """8-qubit ring (256 levels, U[-1,1] couplings) on a fast anneal with three control
    points per schedule, B(0) > 0 and A(1) well away from zero: the smallest gap on the
    grid is about 8e-4 rad/ns, so the oracle's central differences at h = 1e-4 are in the
    linear regime (halving h moves every estimate by less than 1e-7 of its scale)."""
    A = np.array([2.0 * np.pi, np.pi, 2.5])
    B = np.array([0.6, np.pi, 2.0 * np.pi])
    return W.ring_instance(8, 3, t_f=40.0, eta=2e-2, n_grid=30, A_ctrl=A, B_ctrl=B)


@pytest.fixture(scope="module")
def ring8():
    inst = _ring8()
    K = 27     # a ragged last tile for the FP64 (8) and FP32 (16) sweeps
    return inst, K, gradient.trajectory_gradients(inst, K)


@pytest.mark.parametrize("prec,tol", [("fp64", 2e-6), ("fp32", 2e-4)])
def test_per_trajectory_gradient_256_levels(ring8, prec, tol):
    """The 256-level sweeps (eight FP64 or sixteen FP32 trajectories per workgroup, four
    rows per lane, chunked operand loads) per trajectory against the oracle's estimates,
    on the trajectories whose jump sequences agree.  FP32 tolerance: unit roundoff 6e-8
    grown over 256-term sums, 29 steps and five products per step, with a margin."""
    inst, K, ref = ring8
    eng = _engine(inst)
    out = eng.grad_pgs(K, prec, seed=inst.seed, instance_id=inst.instance_id, per_trajectory=True)
    pt = out["per_traj"]
    P = pt.shape[1] // 2 - 1
    assert P == len(ref["params"])
    cap = max(len(j) for j in ref["jumps"]) + 1
    res = eng.run(K, prec, seed=inst.seed, instance_id=inst.instance_id, record_capacity=cap)
    rel = 1e-9 if prec == "fp64" else 1e-4
    same = [j for j in range(K)
            if compare_jump_records(res["jumps"][j:j + 1], res["jump_count"][j:j + 1], ref["jumps"][j:j + 1],
                                    inst.t_f, rel=rel)[0] == 1.0]
    assert len(same) >= (K if prec == "fp64" else K - 2), len(same)
    assert sum(len(ref["jumps"][j]) for j in same) > 10 * len(same)
    np.testing.assert_allclose(pt[same, 0], ref["f"][same], atol=1e-10 if prec == "fp64" else 1e-5)
    for got, want in ((pt[same, 1:P + 1], ref["g"][same]), (pt[same, P + 2:], ref["score"][same])):
        scale = np.maximum(np.abs(want).max(axis=0), 1e-3)
        err = np.abs(got - want) / scale
        assert err.max() <= tol, (err.max(axis=0), np.unravel_index(err.argmax(), err.shape))


def test_gradient_matches_stored_ame_differences_8q():
    """The 8-qubit workload with 16 + 16 control points (config 5): the FP32 estimate from
    10^5 trajectories against the stored central differences of the FP64 split-step AME
    for five parameters (tests/golden/make_golden.py --grad8), within four standard
    errors each.  At 10^5 trajectories only eta is resolved (about 2.5 standard errors),
    which keeps the comparison from being vacuous."""
    import json
    import os
    ref = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "a2a8_ctrl16_fd_gradient.json")))
    inst = W.config_gradient(100_000)
    eng = _engine(inst)
    out = eng.grad_pgs(inst.n_traj, "fp32", seed=inst.seed, instance_id=inst.instance_id)
    m = len(inst.A_ctrl)
    idx = [j if k == "A" else (m + j if k == "B" else 2 * m) for k, j in ref["params"]]
    got, se, fd = out["grad"][idx], out["grad_se"][idx], np.array(ref["grad"])
    assert np.all(np.abs(got - fd) <= 4.0 * se), (got, fd, se)
    assert np.abs(fd[-1]) > 2.0 * se[-1]
