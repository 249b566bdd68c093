"""Quantum-jump trajectories of the adiabatic master equation (FP64 oracle).

TEST INFRASTRUCTURE: only tests/, the smoke check and the bench's cpu_baseline
leg may import anything under oracle/.

Follows the waiting-time procedure of Sec. IV (validity for time-dependent
operators shown in App. C) in the instantaneous eigenbasis:

  * draw a threshold r; propagate the unnormalised state with H_eff until its
    squared norm reaches r (eq. Schr, eq. squareofnorm);
  * pick the jump type with probability <A_i^dag A_i> / lambda (App. B,
    eq. Pi(t)); apply A_i and renormalise (eq. jump);
  * draw a new threshold and continue until t_f.

In the eigenbasis H_eff is diagonal (energies e_b, decay rates Gamma_b; see
oracle.spectrum), so between grid points the no-jump propagator is the
diagonal exp(-i e_b tau - Gamma_b tau / 2) and the squared norm is exactly
sum_b |c_b|^2 exp(-Gamma_b tau).  The generator is frozen at the right end
point of each step; the basis change between grid points is the overlap
O_g (unitary, so it leaves the norm unchanged).

Jump type sampling is two-level and exact: the source level b with weight
q_b Gamma_b (q = current populations), then (qubit i, target a) with weight
R[i, b, a]; a == b selects the omega = 0 operator of qubit i, which acts as
c_x <- z_i[x, x] c_x on every component.  A jump a != b leaves e_a.

Within a step the phases exp(-i e_b dt) are applied once, at the end; this
is exact up to a global phase because the omega = 0 operators commute with
the diagonal propagator and an a != b jump leaves a single component.

Random draws: Philox4x64-10 (oracle.philox); draw 0 is the first threshold,
jump m uses draws 3m+1 (source), 3m+2 (qubit and target), 3m+3 (next
threshold).  Newton's method on log(norm^2) from tau = 0 finds the crossing
time (monotone convergence because log-sum-exp is convex).
"""
from __future__ import annotations

import dataclasses
from typing import Iterable, List, Optional

import numpy as np

from . import philox

KIND_RELAX, KIND_EXCITE, KIND_DEPHASE = 0, 1, 2


@dataclasses.dataclass
class TrajectoryResult:
    pgs_sum: np.ndarray          # [M]  sum over trajectories of ground-cluster population
    pgs_sumsq: np.ndarray        # [M]
    jumps: Optional[List[list]]  # per trajectory: list of (t, step, qubit, from_b, to_a, kind)
    net_gs: np.ndarray           # [K] net jumps into the ground cluster
    kind_totals: np.ndarray      # [3]
    final_state: np.ndarray      # [n, K] complex (unnormalised as carried)
    n_traj: int


def crossing_time(w: np.ndarray, Gam: np.ndarray, r: float, tau_max: float, dt: float) -> float:
    """Smallest tau in (0, tau_max] with sum_b w_b exp(-Gam_b tau) = r (Newton on the log)."""
    tau = 0.0
    logr = np.log(r)
    for _ in range(100):
        e = w * np.exp(-Gam * tau)
        g = e.sum()
        f = np.log(g) - logr
        fp = -(Gam * e).sum() / g
        if fp == 0.0:
            return tau_max
        step = -f / fp
        if not step > 0.0:
            break
        tau_new = min(tau + step, tau_max)
        if tau_new - tau <= 1e-15 * dt:
            tau = tau_new
            break
        tau = tau_new
        if tau >= tau_max:
            break
    return tau


def pick(weights: np.ndarray, u: float) -> int:
    """First index whose running (left-to-right) sum exceeds u * total."""
    cum = np.cumsum(weights)
    idx = int(np.searchsorted(cum, u * cum[-1], side="right"))
    if idx >= len(weights):
        idx = int(np.nonzero(weights > 0)[0][-1])
    return idx


def run(tables: Iterable, inst, n_traj: int, *, n_grid: Optional[int] = None, seed: Optional[int] = None,
        instance_id: Optional[int] = None, traj_offset: int = 0, record: bool = True,
        n_levels: Optional[int] = None) -> TrajectoryResult:
    M = n_grid or inst.n_grid
    seed = inst.seed if seed is None else seed
    iid = inst.instance_id if instance_id is None else instance_id
    K = n_traj
    tid = np.arange(traj_offset, traj_offset + K, dtype=np.uint64)
    r = philox.draw(seed, iid, tid, 0)
    m = np.zeros(K, dtype=np.int64)
    pgs_sum = np.zeros(M)
    pgs_sumsq = np.zeros(M)
    pgs_sum[0] = K       # the initial state is the ground state of H(0)
    pgs_sumsq[0] = K
    jumps = [[] for _ in range(K)] if record else None
    net = np.zeros(K, dtype=np.int64)
    kinds = np.zeros(3, dtype=np.int64)
    c = None
    for T in tables:
        g = T.g
        k = g - 1
        t_k, dt = T.t0, T.dt
        if g == 1:
            c = np.repeat(T.cinit.astype(np.complex128)[:, None], K, axis=1)
        else:
            c = T.O @ c
        Gam = T.Gamma
        nu_end = (np.abs(c) ** 2 * np.exp(-Gam * dt)[:, None]).sum(axis=0)
        cross = nu_end <= r
        c[:, ~cross] *= np.exp(-0.5 * Gam * dt)[:, None]
        for j in np.nonzero(cross)[0]:
            cj = c[:, j].copy()
            tau_e = 0.0
            while True:
                rem = dt - tau_e
                w = np.abs(cj) ** 2
                if (w * np.exp(-Gam * rem)).sum() > r[j]:
                    cj *= np.exp(-0.5 * Gam * rem)
                    break
                tau = crossing_time(w, Gam, r[j], rem, dt)
                cj *= np.exp(-0.5 * Gam * tau)
                tau_e += tau
                q = np.abs(cj) ** 2
                u1 = philox.draw_scalar(seed, iid, tid[j], 3 * m[j] + 1)
                u2 = philox.draw_scalar(seed, iid, tid[j], 3 * m[j] + 2)
                b = pick(q * Gam, float(u1))
                ia = pick(T.R[:, b, :].ravel(), float(u2))
                i, a = divmod(ia, len(Gam))
                if a != b:
                    cj = np.zeros_like(cj)
                    cj[a] = 1.0
                    kind = KIND_RELAX if T.E[a] <= T.E[b] else KIND_EXCITE
                    if a < T.gs <= b:
                        net[j] += 1
                    elif b < T.gs <= a:
                        net[j] -= 1
                else:
                    cj = T.zdiag[i] * cj
                    kind = KIND_DEPHASE
                cj /= np.linalg.norm(cj)
                kinds[kind] += 1
                if record:
                    jumps[j].append((t_k + tau_e, k, int(i), int(b), int(a), kind))
                m[j] += 1
                r[j] = philox.draw_scalar(seed, iid, tid[j], 3 * m[j])
            c[:, j] = cj
        c *= np.exp(-1j * T.Eph * dt)[:, None]
        pop = np.abs(c) ** 2
        p = pop[:T.gs].sum(axis=0) / pop.sum(axis=0)
        pgs_sum[g] = p.sum()
        pgs_sumsq[g] = (p * p).sum()
    return TrajectoryResult(pgs_sum=pgs_sum, pgs_sumsq=pgs_sumsq, jumps=jumps, net_gs=net,
                            kind_totals=kinds, final_state=c, n_traj=K)


def mean_and_stderr(sum_, sumsq, R: int):
    """Sample mean and standard error of the mean (Sec. VI, eq. stderror)."""
    mean = sum_ / R
    var = (sumsq - R * mean * mean) / (R - 1)
    return mean, np.sqrt(np.maximum(var, 0.0) / R)


def run_fixed_step(tables: Iterable, inst, n_traj: int, substeps: int, *, n_grid: Optional[int] = None,
                   seed: Optional[int] = None, instance_id: Optional[int] = None, traj_offset: int = 0,
                   record: bool = True) -> TrajectoryResult:
    """Fixed-step quantum-jump unraveling (App. B, "to jump or not to jump"): each grid step
    of length dt is cut into `substeps` sub-steps of length h with the generator frozen at
    the grid point (as in run).  Per sub-step the normalised state has jump probability
    dp = h sum_b |c_b|^2 Gamma_b (eq. lambda); a uniform eps decides: eps >= dp evolves
    with the no-jump propagator exp(-i e h - Gamma h / 2) and renormalises, eps < dp
    applies the jump operator drawn with probability proportional to its rate (eq. Pi(t):
    source b with weight |c_b|^2 Gamma_b, then qubit and target by R, as in run) and
    renormalises.  First order in h: the mean approaches the master equation as h -> 0.

    Draws: sub-step u = (g - 1) substeps + s of trajectory j uses draws 3u (eps), 3u + 1
    (source) and 3u + 2 (qubit and target).  Jump records carry the sub-step's start time."""
    M = n_grid or inst.n_grid
    seed = inst.seed if seed is None else seed
    iid = inst.instance_id if instance_id is None else instance_id
    K = n_traj
    tid = np.arange(traj_offset, traj_offset + K, dtype=np.uint64)
    pgs_sum = np.zeros(M)
    pgs_sumsq = np.zeros(M)
    pgs_sum[0] = K
    pgs_sumsq[0] = K
    jumps = [[] for _ in range(K)] if record else None
    net = np.zeros(K, dtype=np.int64)
    kinds = np.zeros(3, dtype=np.int64)
    c = None
    for T in tables:
        g = T.g
        k = g - 1
        h = T.dt / substeps
        if g == 1:
            c = np.repeat(T.cinit.astype(np.complex128)[:, None], K, axis=1)
        else:
            c = T.O @ c
        Gam = T.Gamma
        dsub = np.exp(-1j * T.Eph * h - 0.5 * Gam * h)
        for s in range(substeps):
            u = k * substeps + s
            pop = np.abs(c) ** 2
            dp = h * (pop * Gam[:, None]).sum(axis=0) / pop.sum(axis=0)
            eps = philox.draw(seed, iid, tid, np.uint64(3 * u))
            jump = eps < dp
            stay = ~jump
            c[:, stay] *= dsub[:, None]
            c[:, stay] /= np.linalg.norm(c[:, stay], axis=0)[None, :]
            for j in np.nonzero(jump)[0]:
                cj = c[:, j]
                q = np.abs(cj) ** 2
                u1 = philox.draw_scalar(seed, iid, tid[j], 3 * u + 1)
                u2 = philox.draw_scalar(seed, iid, tid[j], 3 * u + 2)
                b = pick(q * Gam, float(u1))
                ia = pick(T.R[:, b, :].ravel(), float(u2))
                i, a = divmod(ia, len(Gam))
                if a != b:
                    cj = np.zeros_like(cj)
                    cj[a] = 1.0
                    kind = KIND_RELAX if T.E[a] <= T.E[b] else KIND_EXCITE
                    if a < T.gs <= b:
                        net[j] += 1
                    elif b < T.gs <= a:
                        net[j] -= 1
                else:
                    cj = T.zdiag[i] * cj
                    kind = KIND_DEPHASE
                c[:, j] = cj / np.linalg.norm(cj)
                kinds[kind] += 1
                if record:
                    jumps[j].append((T.t0 + s * h, k, int(i), int(b), int(a), kind))
        pop = np.abs(c) ** 2
        p = pop[:T.gs].sum(axis=0) / pop.sum(axis=0)
        pgs_sum[g] = p.sum()
        pgs_sumsq[g] = (p * p).sum()
    return TrajectoryResult(pgs_sum=pgs_sum, pgs_sumsq=pgs_sumsq, jumps=jumps, net_gs=net,
                            kind_totals=kinds, final_state=c, n_traj=K)
