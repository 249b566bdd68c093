"""Non-uniform s-grids on the GPU against the FP64 oracle.

The grid used here follows the App. B time-step bound (eq. B7): its local step is
proportional to the bound's instantaneous value (the oracle's bound_grid, pinned to a
closed form).  Steps of different lengths change the step tables, the jump times and
the gradient's hat-function weights; exact-mean parity with the split-step AME on the
same grid holds for any grid.
"""
import numpy as np
import pytest

import workloads as W
from oracle import ame, gradient, spectrum, trajectories

from gpu_common import compare_jump_records, sigma_bound

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def grid_case():
    inst = W.ring_instance(3, 8, t_f=1.5, eta=0.1, n_grid=61)
    inst = inst.with_(s_grid=spectrum.bound_grid(inst, 61, n_probe=121))
    return inst, spectrum.all_tables(inst)


def _engine(inst):
    from paper_1710_03431_amd.binding import Engine
    eng = Engine(0)
    eng.set_instance(inst)
    eng.precompute(inst.n_grid, inst.levels)
    return eng


def test_grid_fp64_per_trajectory(grid_case):
    inst, tabs = grid_case
    steps = np.diff(inst.s_grid)
    assert steps.max() > 1.5 * steps.min()
    K = 400
    ref = trajectories.run(tabs, inst, K)
    res = _engine(inst).run(K, "fp64", seed=inst.seed, instance_id=inst.instance_id, record_capacity=32)
    frac, worst = compare_jump_records(res["jumps"], res["jump_count"], ref.jumps, inst.t_f)
    assert frac >= 0.99, (frac, worst)
    if frac == 1.0:
        np.testing.assert_allclose(res["pgs_sum"], ref.pgs_sum, rtol=1e-9)


def test_grid_average_matches_ame(grid_case):
    inst, tabs = grid_case
    P = ame.split_step(tabs, inst)
    K = 1_000_000
    res = _engine(inst).run(K, "fp32", seed=inst.seed + 9, instance_id=inst.instance_id)
    m, se = trajectories.mean_and_stderr(res["pgs_sum"], res["pgs_sumsq"], K)
    sig = sigma_bound(P, se, K)
    assert np.all(np.abs(m - P) <= 3 * sig + 1e-4)


def test_grid_fixed_step_per_trajectory(grid_case):
    inst, tabs = grid_case
    K, S = 200, 3
    ref = trajectories.run_fixed_step(tabs, inst, K, S)
    res = _engine(inst).run_fixed_step(K, S, "fp64", seed=inst.seed, instance_id=inst.instance_id,
                                       record_capacity=64)
    frac, worst = compare_jump_records(res["jumps"], res["jump_count"], ref.jumps, inst.t_f)
    assert frac >= 0.99, (frac, worst)


def test_grid_gradient_per_trajectory(grid_case):
    """Per-trajectory gradient estimates on the non-uniform grid (5 control points, whose
    hat functions are sampled at the grid points)."""
    inst, _ = grid_case
    A, B = W.linear_schedule(5)
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


def test_grid_argument_errors_and_equidistant_default():
    from paper_1710_03431_amd.binding import AqtError, Engine
    inst = W.ring_instance(3, 8, t_f=1.5, eta=0.1, n_grid=21)
    eng = Engine(0)
    eng.set_instance(inst)
    for bad in ([0.0, 0.5, 0.4, 1.0], [0.1, 0.5, 1.0], [0.0, 0.5, 0.9], [0.0]):
        with pytest.raises(AqtError):
            eng.set_grid(np.array(bad))
    eng.set_grid(np.linspace(0.0, 1.0, 11))
    with pytest.raises(AqtError):            # n_grid differs from the grid's point count
        eng.precompute(21, 8)
    eng.set_grid(np.linspace(0.0, 1.0, 21))
    eng.precompute(21, 8)
    a = eng.run(256, "fp64", seed=3)
    eng.set_grid(None)
    eng.precompute(21, 8)
    b = eng.run(256, "fp64", seed=3)
    np.testing.assert_allclose(a["pgs_sum"], b["pgs_sum"], rtol=1e-9)


@pytest.mark.parametrize("case", ["ring3", "pm1_6q", "ring4_bath_terms"])
def test_library_step_bound_and_grid_match_the_oracle(case):
    """aqt_step_bound and aqt_bound_grid (App. B eq. B7) against oracle.spectrum.step_bound
    and bound_grid: the bound at every probe to 1e-8 relative (the library's operator norm
    comes from a power iteration stopped at 1e-13 in the squared norm), the grid points to
    1e-8.  Bath terms enter through the decay rates."""
    insts = {"ring3": W.ring_instance(3, 8, t_f=1.5, eta=0.1, n_grid=61),
             "pm1_6q": W.pm1_all_to_all(6, 11, t_f=40.0, eta=1e-3, n_grid=61),
             "ring4_bath_terms": W.ring_instance(4, 1001, t_f=30.0, eta=1e-2, n_grid=41,
                                                 bath_terms=W.two_term_bath(4))}
    inst = insts[case]
    P = 121
    from paper_1710_03431_amd.binding import Engine
    eng = Engine(0)
    eng.set_instance(inst)
    got = eng.step_bound(P)
    want = spectrum.step_bound(inst, np.linspace(0.0, 1.0, P))
    np.testing.assert_allclose(got, want, rtol=1e-8)
    g = eng.bound_grid(inst.n_grid, P)
    np.testing.assert_allclose(g, spectrum.bound_grid(inst, inst.n_grid, n_probe=P), rtol=0, atol=1e-8)
    assert np.diff(g).max() > 1.2 * np.diff(g).min()
    # the grid is only returned: the context's own grid and tables are untouched
    eng.set_grid(g)
    eng.precompute(inst.n_grid, inst.levels)
    assert eng.get_tables(("E",))["E"].shape == (inst.n_grid, inst.levels)


@pytest.mark.parametrize("case", ["ring3", "pm1_6q"])
@pytest.mark.parametrize("fraction", [0.37, 2.5])
def test_library_bound_grid_points_match_the_oracle(case, fraction):
    """aqt_bound_grid_points, the step control drawn from the App. B bound (eq. B7):
    n_grid - 1 = ceil(t_f F(1) / fraction), F(1) the trapezoid integral of 1 / bound over
    the probes, against the same integral of oracle.spectrum.step_bound; on the grid that
    aqt_bound_grid returns for that count every step stays within the fraction of the
    oracle's bound at the step's midpoint (interpolated from the probes, 2% for the
    linear interpolations), and most steps use more than 90% of it."""
    insts = {"ring3": W.ring_instance(3, 8, t_f=1.5, eta=0.1, n_grid=61),
             "pm1_6q": W.pm1_all_to_all(6, 11, t_f=40.0, eta=1e-3, n_grid=61)}
    inst = insts[case]
    P = 121
    from paper_1710_03431_amd.binding import Engine
    eng = Engine(0)
    eng.set_instance(inst)
    M = eng.bound_grid_points(fraction, P)
    sp = np.linspace(0.0, 1.0, P)
    b = spectrum.step_bound(inst, sp)
    F = float(np.sum(0.5 * (1.0 / b[1:] + 1.0 / b[:-1]) * np.diff(sp)))
    x = inst.t_f * F / fraction
    want = max(2, int(np.ceil(x)) + 1)
    assert M == want or (abs(x - round(x)) < 1e-6 and abs(M - want) <= 1), (M, want, x)
    g = eng.bound_grid(M, P)
    ratio = inst.t_f * np.diff(g) / (fraction * np.interp(0.5 * (g[1:] + g[:-1]), sp, b))
    assert ratio.max() <= 1.02, ratio.max()
    assert np.median(ratio) > 0.9, np.median(ratio)


def test_library_bound_grid_argument_errors():
    from paper_1710_03431_amd.binding import AqtError, Engine
    eng = Engine(0)
    with pytest.raises(AqtError):
        eng.step_bound(11)                          # nothing set
    inst = W.pm1_all_to_all(9, 11, t_f=40.0, n_grid=11)
    eng.set_instance(inst)
    with pytest.raises(AqtError):
        eng.step_bound(11)                          # 512 basis states: beyond the full-spectrum limit
    eng.set_instance(W.ring_instance(3, 8, t_f=1.5, eta=0.1, n_grid=61))
    with pytest.raises(AqtError):
        eng.step_bound(2)
    with pytest.raises(AqtError):
        eng.bound_grid(1, 11)
    for bad in (0.0, -1.0, float("inf"), float("nan")):
        with pytest.raises(AqtError):
            eng.bound_grid_points(bad, 11)
    with pytest.raises(AqtError):
        eng.bound_grid_points(1e-9, 11)              # more than 10^7 points
