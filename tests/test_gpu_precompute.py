"""Parity of the GPU eigensystem and AME tables (aqt_precompute) with the FP64 oracle."""
import numpy as np
import pytest

import workloads as W
from oracle import ame, spectrum, trajectories

from gpu_common import compare_jump_records, sigma_bound

pytestmark = pytest.mark.gpu


def gpu_tables(inst, n_grid=None, n_levels=None, deg_tol=1e-8):
    from paper_1710_03431_amd.binding import Engine
    eng = Engine(0)
    eng.set_instance(inst)
    eng.precompute(n_grid or inst.n_grid, n_levels or inst.levels, deg_tol)
    return eng


def level_condition(E, deg_tol=1e-8):
    """First-order eigenvector error bound per level: eps |H| / (distance to the nearest
    level outside its cluster).  Both eigensolvers are backward stable, so eigenvector
    entries of two correct solvers may differ by about this much."""
    eps_h = 2.2e-16 * max(np.abs(E).max(), 1.0)
    n = len(E)
    gap = np.full(n, np.inf)
    for a in range(n):
        d = np.abs(E - E[a])
        d = d[d >= deg_tol]
        if d.size:
            gap[a] = d.min()
    return eps_h / gap


def check_tables(got, tabs, scale, safety=200.0):
    """E to 1e-12 of the spectral scale; overlaps, matrix-element rates, decay and zdiag
    to 1e-10 plus the first-order eigenvector-conditioning bound of the levels involved."""
    for T in tabs:
        g = T.g
        np.testing.assert_allclose(got["E"][g], T.E, atol=1e-12 * scale, rtol=0, err_msg=f"E g={g}")
        assert got["gs"][g] == T.gs, g
        kap = safety * level_condition(T.E)
        pair = kap[:, None] + kap[None, :]
        if T.O is not None:
            err = np.abs(got["O"][g] - T.O)
            assert np.all(err <= 1e-10 + pair), (g, (err - pair).max())
        rmax = max(T.R.max(), 1e-300)
        for i in range(T.R.shape[0]):
            # R[b][a] = gamma z_ab^2: error <= 2 gamma |z_ab| dz with dz <= pair bound
            gam_over = T.R[i] / np.maximum(np.abs(T.z[i].T) ** 2, 1e-300)
            bound = 1e-10 * rmax + 2.0 * gam_over * np.abs(T.z[i].T) * pair.T + 1e-12 * rmax
            err = np.abs(got["R"][g][i] - T.R[i])
            assert np.all(err <= bound), (g, i, float((err - bound).max()), float(rmax))
        np.testing.assert_array_less(np.abs(got["zdiag"][g] - T.zdiag), 1e-10 + 2 * kap[None, :] + 1e-300,
                                     err_msg=f"zdiag g={g}")
        gmax = T.Gamma.max()
        assert np.all(np.abs(got["Gamma"][g] - T.Gamma) <= 1e-10 * gmax + 2 * gmax * kap.max() * len(T.E)), g
        assert abs(got["leak"][g] - T.leak) < 1e-10 + 2 * kap.max(), g


def test_small_full_spectrum_tables():
    inst = W.config_small()
    tabs = spectrum.all_tables(inst)
    eng = gpu_tables(inst)
    got = eng.get_tables()
    np.testing.assert_allclose(got["cinit"], tabs[0].cinit, atol=1e-12)
    check_tables(got, tabs, scale=10.0)


def test_a2a8_full_spectrum_tables_sampled():
    """8 qubits, n = 256, 2000 grid points; sampled grid points incl. s = 1 (degenerate
    Ising levels in the canonical basis) and the first two."""
    inst = W.config_a2a8(10)
    grids = {1, 2, 3, 700, 1001, 1500, 1998, 1999}
    tabs = list(spectrum.table_stream(inst, grids=grids))
    eng = gpu_tables(inst)
    got = eng.get_tables()
    check_tables(got, tabs, scale=100.0)


def test_truncated_tables_polar():
    """6 qubits truncated to 16 levels: polar overlaps, leakage and rates."""
    inst = W.pm1_all_to_all(6, 5, t_f=2000.0, n_grid=300, n_levels=16)
    grids = {1, 2, 57, 150, 298, 299}
    tabs = list(spectrum.table_stream(inst, grids=grids))
    eng = gpu_tables(inst)
    got = eng.get_tables()
    check_tables(got, tabs, scale=50.0)


def test_end_to_end_small_per_trajectory():
    """GPU precompute + FP64 stepping vs the oracle's tables + trajectories (4-qubit workload)."""
    inst = W.config_small()
    tabs = spectrum.all_tables(inst)
    K = 1000
    ref = trajectories.run(tabs, inst, K)
    eng = gpu_tables(inst)
    res = eng.run(K, "fp64", seed=inst.seed, instance_id=inst.instance_id, record_capacity=64)
    frac, worst = compare_jump_records(res["jumps"], res["jump_count"], ref.jumps, inst.t_f)
    assert frac >= 0.999, (frac, worst)
    P = ame.split_step(tabs, inst)
    m, se = trajectories.mean_and_stderr(res["pgs_sum"], res["pgs_sumsq"], K)
    assert np.all(np.abs(m - P) <= 3 * sigma_bound(P, se, K) + 1e-4)


def test_degenerate_initial_state_is_rejected():
    from paper_1710_03431_amd.binding import AqtError, AQT_ENUMERIC
    inst = W.ring_instance(4, 3)
    inst = inst.with_(h=np.zeros(4), A_ctrl=np.array([0.0, 0.0]), B_ctrl=np.array([1.0, 1.0]))
    with pytest.raises(AqtError) as e:
        gpu_tables(inst, n_grid=5)
    assert e.value.status == AQT_ENUMERIC
