"""Helpers shared by the GPU tests: oracle tables stacked for aqt_set_tables,
GPU-vs-oracle jump-record comparison and the statistical acceptance bound."""
import numpy as np

import workloads as W
from oracle import ame, spectrum, trajectories


def stack_tables(tabs, inst, n_grid=None):
    """Stack a list of oracle GridTables (g = 1..M-1) into aqt_set_tables arrays."""
    M = n_grid or inst.n_grid
    n = len(tabs[0].E)
    nq = inst.n_qubits
    E = np.zeros((M, n))
    gs = np.ones(M, dtype=np.int32)
    O = np.zeros((M, n, n))
    R = np.zeros((M, nq, n, n))
    zd = np.zeros((M, nq, n))
    cinit = None
    for T in tabs:
        E[T.g] = T.E
        gs[T.g] = T.gs
        R[T.g] = T.R
        zd[T.g] = T.zdiag
        if T.O is not None:
            O[T.g] = T.O
        if T.cinit is not None:
            cinit = T.cinit
    return dict(E=E, gs=gs, O=O, cinit=cinit, R=R, zdiag=zd)


def engine_with_oracle_tables(inst, tabs, n_grid=None):
    from paper_1710_03431_amd.binding import Engine
    eng = Engine(0)
    eng.set_instance(inst)
    eng.set_tables(**stack_tables(tabs, inst, n_grid))
    return eng


def compare_jump_records(gpu_jumps, gpu_count, oracle_jumps, t_f, rel=1e-9):
    """Fraction of trajectories whose jump sequences agree (channel and time)."""
    K = len(oracle_jumps)
    same = 0
    worst = 0.0
    for j in range(K):
        o = oracle_jumps[j]
        if gpu_count[j] != len(o):
            continue
        ok = True
        for m, rec in enumerate(o):
            g = gpu_jumps[j, m]
            if (int(g["qubit"]), int(g["from_level"]), int(g["to_level"]), int(g["kind"])) != \
               (rec[2], rec[3], rec[4], rec[5]):
                ok = False
                break
            dt = abs(float(g["t"]) - rec[0])
            worst = max(worst, dt / (abs(rec[0]) + 1e-300))
            if dt > rel * abs(rec[0]) + 1e-12 * t_f:
                ok = False
                break
        same += ok
    return same / K, worst


def sigma_bound(P, se, K):
    """Standard error of the mean, floored by the Bernoulli bound sqrt(P(1-P)/K)
    (a sample with no events yet has zero sample variance)."""
    return np.maximum(se, np.sqrt(np.clip(P * (1 - P), 0, None) / K))


def family_z(n_points, alpha=1e-3):
    """Two-sided normal critical value for n_points comparisons at family-wise false-alarm
    rate alpha (Bonferroni): 4.06 for 200 points, 4.56 for 2000."""
    from scipy.stats import norm
    return float(norm.isf(alpha / (2.0 * n_points)))


def assert_mean_matches(m, se, P, K, what=""):
    """Trajectory means m (standard errors se, K trajectories) against exact means P.

    Every grid point: |m - P| <= z_M sigma + 1e-4, with z_M the Bonferroni critical value
    for the M points at a family-wise false-alarm rate of 1e-3 (the points share their
    trajectories, so the bound is conservative); the final point, the reported value:
    |m - P| <= 3 sigma + 1e-4.  sigma is the sample standard error floored by the
    Bernoulli bound sqrt(P(1-P)/K), since a sample in which a rare event has not yet
    happened has zero sample variance but not zero uncertainty."""
    sig = sigma_bound(P, se, K)
    err = np.abs(m - P)
    z = family_z(len(P))
    bad = np.nonzero(err > z * sig + 1e-4)[0]
    assert len(bad) == 0, (what, "grid points", bad[:10], err[bad[:10]], sig[bad[:10]], z)
    assert err[-1] <= 3.0 * sig[-1] + 1e-4, (what, "final", m[-1], P[-1], sig[-1])
