"""Gradient of the final ground-state population by central differences (FP64 oracle).

TEST INFRASTRUCTURE: only tests/, the smoke check and the bench's cpu_baseline
leg may import anything under oracle/.

The quantity differentiated is the exact mean of the discrete trajectory process,
the split-step AME (ame.split_step), at s = 1:

    P(theta) = P_GS(1),  theta = (A_1..A_m, B_1..B_m, eta),

with A(s), B(s) piecewise linear through the m control points (Sec. V schedules,
written as controls) and eta the system-bath coupling of the Ohmic spectral
density (Sec. V, g^2).  Control points move by an absolute step h (rad/ns) and eta
by a relative step h, both central: (P(x + h) - P(x - h)) / 2h.  The adjoint
estimator of the trajectory average is checked against these numbers.
"""
from __future__ import annotations

import numpy as np

from . import ame, spectrum


def final_pgs(inst) -> float:
    """P_GS at s = 1 of the split-step AME of the instance."""
    P = ame.split_step(spectrum.table_stream(inst), inst)
    return float(P[-1])


def fd_gradient(inst, h: float = 1e-4, which=("A", "B", "eta")) -> dict:
    """Central-difference gradient of final_pgs with respect to the control points
    (absolute step h) and eta (relative step h).  Returns dA, dB (arrays) and deta."""
    out = {}
    A = np.asarray(inst.A_ctrl, dtype=np.float64)
    B = np.asarray(inst.B_ctrl, dtype=np.float64)
    if "A" in which:
        g = np.zeros(len(A))
        for j in range(len(A)):
            Ap, Am = A.copy(), A.copy()
            Ap[j] += h
            Am[j] -= h
            g[j] = (final_pgs(inst.with_(A_ctrl=Ap)) - final_pgs(inst.with_(A_ctrl=Am))) / (2.0 * h)
        out["dA"] = g
    if "B" in which:
        g = np.zeros(len(B))
        for j in range(len(B)):
            Bp, Bm = B.copy(), B.copy()
            Bp[j] += h
            Bm[j] -= h
            g[j] = (final_pgs(inst.with_(B_ctrl=Bp)) - final_pgs(inst.with_(B_ctrl=Bm))) / (2.0 * h)
        out["dB"] = g
    if "eta" in which:
        e = inst.eta
        out["deta"] = (final_pgs(inst.with_(eta=e * (1 + h))) - final_pgs(inst.with_(eta=e * (1 - h)))) / (2.0 * e * h)
    return out
