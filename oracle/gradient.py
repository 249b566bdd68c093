"""Gradients of the final ground-state population (FP64 oracle).

TEST INFRASTRUCTURE: only tests/, the smoke check and the bench's cpu_baseline
leg may import anything under oracle/.

Parameters theta = (A_1..A_m, B_1..B_m, eta): the control points of the
piecewise-linear schedules A(s), B(s) (Sec. V schedules, written as controls)
and the system-bath coupling eta of the Ohmic spectral density (Sec. V, g^2).
Control points move by an absolute step h (rad/ns), eta by a relative step h;
all differences are central, (F(x + h) - F(x - h)) / 2h.

Two quantities are differentiated:

* fd_gradient: P(theta) = P_GS(1) of the split-step AME (ame.split_step), the
  exact mean of the discrete trajectory process.

* trajectory_gradients: one estimate per trajectory.  A trajectory of the
  waiting-time procedure (Sec. IV) is a path: its jump times and channels.
  Paths have density |psi~|^2 with respect to a measure that does not depend on
  theta (Lebesgue measure on the times, counting measure on the channels), where
  psi~ is the unnormalised amplitude built from the no-jump propagators, the
  basis changes and the jump operators sqrt(gamma) A along the path (Sec. III,
  eqs. Heff and jump; App. B).  Hence E[P_GS] = integral of <psi~|Pi|psi~> over
  paths, and its derivative is E[g] with

      g = d<psi~|Pi|psi~>/dtheta / |psi~|^2 = f * d log <psi~|Pi|psi~> / dtheta,

  f = <psi~|Pi|psi~> / |psi~|^2 the trajectory's own final ground-cluster
  population.  Here the derivative is taken by central differences of the log
  weight of the trajectory's own path (times and channels held fixed), rebuilt
  from the tables of the perturbed instance.  The same with Pi replaced by the
  identity gives s = d log |psi~|^2 / dtheta, the score of the path density,
  whose mean is zero (the derivative of the total probability 1).
"""
from __future__ import annotations

from collections import defaultdict

import numpy as np

from . import ame, spectrum, trajectories


def final_pgs(inst) -> float:
    """P_GS at s = 1 of the split-step AME of the instance."""
    P = ame.split_step(spectrum.table_stream(inst), inst)
    return float(P[-1])


def _perturbed(inst, kind: str, j: int, sign: float, h: float):
    """The instance with parameter (kind, j) moved by sign * step; returns (inst, step)."""
    if kind == "A":
        v = np.array(inst.A_ctrl, dtype=np.float64)
        v[j] += sign * h
        return inst.with_(A_ctrl=v), h
    if kind == "B":
        v = np.array(inst.B_ctrl, dtype=np.float64)
        v[j] += sign * h
        return inst.with_(B_ctrl=v), h
    return inst.with_(eta=inst.eta * (1.0 + sign * h)), inst.eta * h


def parameter_list(inst, which=("A", "B", "eta")):
    """[(kind, index)] in output order: A controls, B controls, eta."""
    out = []
    if "A" in which:
        out += [("A", j) for j in range(len(inst.A_ctrl))]
    if "B" in which:
        out += [("B", j) for j in range(len(inst.B_ctrl))]
    if "eta" in which:
        out.append(("eta", 0))
    return out


def fd_gradient(inst, h: float = 1e-4, which=("A", "B", "eta")) -> dict:
    """Central-difference gradient of final_pgs.  Returns dA, dB (arrays) and deta."""
    out = {}
    for kind in ("A", "B"):
        if kind in which:
            m = len(inst.A_ctrl if kind == "A" else inst.B_ctrl)
            g = np.zeros(m)
            for j in range(m):
                ip, step = _perturbed(inst, kind, j, +1.0, h)
                im, _ = _perturbed(inst, kind, j, -1.0, h)
                g[j] = (final_pgs(ip) - final_pgs(im)) / (2.0 * step)
            out["d" + kind] = g
    if "eta" in which:
        ip, step = _perturbed(inst, "eta", 0, +1.0, h)
        im, _ = _perturbed(inst, "eta", 0, -1.0, h)
        out["deta"] = (final_pgs(ip) - final_pgs(im)) / (2.0 * step)
    return out


def replay_log_weight(tables, inst, paths, n_grid=None):
    """Rebuild the unnormalised amplitude psi~ of each fixed path with the given tables.

    paths[j] is trajectory j's list of jumps (t, step, qubit, from_b, to_a, kind) in
    time order, as recorded by trajectories.run.  Between jumps the state evolves by
    the diagonal no-jump propagator (decay exp(-Gamma tau / 2); the phases exp(-i e dt)
    are applied at the end of each step, which changes psi~ by a global phase only);
    at a grid point by the overlap O_g; a jump b -> a (a != b) of qubit i multiplies by
    the operator sqrt(R[i, b, a]) |a><b| and the omega = 0 operator of qubit i by
    sqrt(gamma(0)) diag(z_i), whose squared action is sum_x R[i, x, x] |c_x|^2.  The
    state is carried normalised after each jump with the logs of the norms summed.

    Returns (log <psi~|Pi|psi~>, log <psi~|psi~>, final carried states [n, K]) with Pi
    the projector on the ground cluster of the last grid point."""
    K = len(paths)
    first = defaultdict(list)            # step -> [(trajectory, index of its first jump in the step)]
    for j, p in enumerate(paths):
        for m, rec in enumerate(p):
            if m == 0 or p[m - 1][1] != rec[1]:
                first[rec[1]].append((j, m))
    logs = np.zeros(K)
    C = None
    gs = 1
    for T in tables:
        k = T.g - 1
        t_k, dt = T.t0, T.dt
        C = np.repeat(T.cinit.astype(np.complex128)[:, None], K, axis=1) if T.g == 1 else T.O @ C
        starts = first.get(k, [])
        saved = [C[:, j].copy() for j, _ in starts]
        C *= np.exp(-0.5 * T.Gamma * dt)[:, None]
        for (j, m), c in zip(starts, saved):
            p = paths[j]
            tau_e = 0.0
            while m < len(p) and p[m][1] == k:
                t, _, i, b, a, _ = p[m]
                tau = t - t_k
                c = c * np.exp(-0.5 * T.Gamma * (tau - tau_e))
                tau_e = tau
                if a != b:
                    logs[j] += 0.5 * np.log(T.R[i, b, a]) + np.log(abs(c[b]))
                    c = np.zeros_like(c)
                    c[a] = 1.0
                else:
                    logs[j] += 0.5 * np.log(np.sum(np.diag(T.R[i]) * np.abs(c) ** 2))
                    y = T.zdiag[i] * c
                    c = y / np.linalg.norm(y)
                m += 1
            C[:, j] = c * np.exp(-0.5 * T.Gamma * (dt - tau_e))
        C *= np.exp(-1j * T.Eph * dt)[:, None]
        gs = T.gs
    pop = np.abs(C) ** 2
    with np.errstate(divide="ignore"):   # log 0 = -inf: the path ends outside the ground cluster
        logW = 2.0 * logs + np.log(pop[:gs].sum(axis=0))
    return logW, 2.0 * logs + np.log(pop.sum(axis=0)), C


def trajectory_gradients(inst, n_traj: int, h: float = 1e-4, which=("A", "B", "eta"),
                         traj_offset: int = 0) -> dict:
    """Per-trajectory gradient estimates g[j, p] and path-density scores score[j, p]
    (module docstring) for the parameters of parameter_list(inst, which), from
    trajectories.run on the instance's tables.  Also returns f[j] (final ground-cluster
    population), the recorded paths and the final states of the replay."""
    tabs = spectrum.all_tables(inst)
    res = trajectories.run(tabs, inst, n_traj, record=True, traj_offset=traj_offset)
    logW, logN, C = replay_log_weight(tabs, inst, res.jumps)
    f = np.exp(logW - logN)
    params = parameter_list(inst, which)
    g = np.zeros((n_traj, len(params)))
    score = np.zeros((n_traj, len(params)))
    for col, (kind, j) in enumerate(params):
        ip, step = _perturbed(inst, kind, j, +1.0, h)
        im, _ = _perturbed(inst, kind, j, -1.0, h)
        lp, np_, _ = replay_log_weight(spectrum.all_tables(ip), ip, res.jumps)
        lm, nm_, _ = replay_log_weight(spectrum.all_tables(im), im, res.jumps)
        score[:, col] = (np_ - nm_) / (2.0 * step)
        # a path that ends outside the ground cluster has zero weight for every theta
        with np.errstate(invalid="ignore"):
            g[:, col] = np.where(f > 0.0, f * (lp - lm) / (2.0 * step), 0.0)
    return {"f": f, "g": g, "score": score, "params": params, "jumps": res.jumps, "replay_state": C,
            "final_state": res.final_state}
