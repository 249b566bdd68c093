"""Density-matrix solvers of the adiabatic master equation (FP64 oracle).

TEST INFRASTRUCTURE: only tests/, the smoke check and the bench's cpu_baseline
leg may import anything under oracle/.

Three independent routes to the AME of Sec. II (eqs. ME2-H, ME2-L, Lindblad2,
dissdiag).  The Lamb shift is zero unless the instance asks for it (the paper gives no
S(w); model.lamb_S is the Ohmic bath's); split_step and liouvillian include it then,
continuous does not support it:

split_step   -- the exact mean of the trajectory process on the same grid:
                rho <- O_g rho O_g^T, then rho <- exp(L_g dt) rho with L_g the
                Lindbladian frozen at s_g, written in the eigenbasis where it
                decouples: populations evolve with the rate matrix
                W[a, b] = sum_i R[i, b, a] (b -> a), coherences a != b decay as
                exp(-i(e_a - e_b) dt - (Gamma_a + Gamma_b) dt / 2
                    + gamma(0) sum_i z_i[a,a] z_i[b,b] dt).
                (Averaging trajectories gives the master equation, App. B.)
liouvillian  -- the Lindbladian as an explicit n^2 x n^2 matrix built from the
                operators L_{i,w} of eq. Lindblad2 grouped by Bohr frequency
                (pairs a != b kept as separate operators, the a == b terms
                of each qubit form one w = 0 operator) for small checks.
continuous   -- the lab-frame N x N equation integrated with an adaptive
                Runge-Kutta (DOP853), rebuilding the eigenbasis and the jump
                operators from numpy eigh at every right-hand-side call.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
from scipy.integrate import solve_ivp

from . import model


def rate_matrix(T) -> np.ndarray:
    """W[a, b]: transition rate b -> a (a != b); columns sum to zero."""
    W = T.R.sum(axis=0).T.copy()
    np.fill_diagonal(W, 0.0)
    W -= np.diag(W.sum(axis=0))
    return W


def coherence_factor(T, inst, dt: float) -> np.ndarray:
    g0 = float(model.gamma_ohmic(0.0, inst.eta, inst.omega_c, inst.T))
    E, Gam, zd = T.Eph, T.Gamma, T.zdiag
    cross = g0 * (zd.T @ zd)                      # gamma(0) sum_i z_aa z_bb
    rate = (-1j * (E[:, None] - E[None, :]) - 0.5 * (Gam[:, None] + Gam[None, :]) + cross)
    return np.exp(rate * dt)


def step_map(rho: np.ndarray, T, inst, dt: float) -> np.ndarray:
    """exp(L_g dt) applied to rho in the eigenbasis of grid g."""
    p = np.real(np.diag(rho)).copy()
    p = sla.expm(rate_matrix(T) * dt) @ p
    out = rho * coherence_factor(T, inst, dt)
    out[np.diag_indices_from(out)] = p
    return out


def split_step(tables, inst, n_grid=None, keep_rho=False):
    """P_GS(s_g) for g = 0..M-1 (and optionally the final rho) of the split-step AME."""
    M = n_grid or inst.n_grid
    P = np.zeros(M)
    P[0] = 1.0
    rho = None
    for T in tables:
        if T.g == 1:
            rho = np.outer(T.cinit, T.cinit).astype(np.complex128)
        else:
            rho = T.O @ rho @ T.O.T
        rho = step_map(rho, T, inst, T.dt)
        P[T.g] = float(np.real(np.trace(rho[:T.gs, :T.gs])))
    return (P, rho) if keep_rho else P


def expected_jumps(tables, inst, n_grid=None):
    """Mean number of jumps per trajectory by kind (relax, excite, omega = 0).

    Sec. III: E[dN_i] = <A_i^dag A_i> dt, so the expected count of a channel is
    the time integral of tr(A_i rho A_i^dag).  For a != b channels that is
    R[i, b, a] rho_bb; for the omega = 0 operator of qubit i it is
    gamma(0) sum_b z_i[b, b]^2 rho_bb.  Within a step the populations follow
    expm(W tau) p, integrated exactly with an augmented matrix exponential.
    """
    out = np.zeros(3)
    rho = None
    for T in tables:
        dt = T.dt
        if T.g == 1:
            rho = np.outer(T.cinit, T.cinit).astype(np.complex128)
        else:
            rho = T.O @ rho @ T.O.T
        n = len(T.E)
        p = np.real(np.diag(rho))
        aug = np.zeros((n + 1, n + 1))
        aug[:n, :n] = rate_matrix(T)
        aug[:n, n] = p
        ip = sla.expm(aug * dt)[:n, n]            # integral over the step of p(tau)
        off = T.R.copy()
        for i in range(off.shape[0]):
            np.fill_diagonal(off[i], 0.0)
        flow = off.sum(axis=0) * ip[:, None]        # [b, a] expected b -> a jumps
        lower = T.E[None, :] <= T.E[:, None]        # target energy <= source energy
        out[0] += flow[lower].sum()
        out[1] += flow[~lower].sum()
        out[2] += sum(T.R[i].diagonal() @ ip for i in range(T.R.shape[0]))
        rho = step_map(rho, T, inst, dt)
    return out


def lindblad_operators(T, inst, tol: float = 1e-9):
    """Jump operators (already scaled by sqrt(gamma)) in the eigenbasis of grid g.

    eq. Lindblad2 with A_alpha = sz_alpha: for each qubit, terms with equal
    Bohr frequency belong to one operator.  Distinct a != b pairs are kept
    apart (generic spectra never share a non-zero Bohr frequency); the a == b
    terms share w = 0 and are summed into one diagonal operator.
    """
    n = len(T.E)
    ops = []
    wc = model.bath_channels(inst)[1]
    g0 = float(model.gamma_ohmic(0.0, inst.eta, inst.omega_c, inst.T))
    for i in range(len(T.z)):
        z = T.z[i]
        for a in range(n):
            for b in range(n):
                if a == b:
                    continue
                w = T.E[b] - T.E[a]
                gam = float(model.gamma_ohmic(w, inst.eta, wc[i], inst.T))
                L = np.zeros((n, n))
                L[a, b] = z[a, b]
                ops.append(np.sqrt(gam) * L)
        ops.append(np.sqrt(g0) * np.diag(np.diag(z)))
    return ops


def lamb_hamiltonian(T, inst) -> np.ndarray:
    """H_LS = sum_i sum_w S(w) A_i,w^dag A_i,w (eq. ME2-H) as a matrix, built from the
    unscaled operators of lindblad_operators' grouping (one per a != b pair, one omega = 0
    operator per channel; S with the channel's cutoff)."""
    n = len(T.E)
    H = np.zeros((n, n))
    wc = model.bath_channels(inst)[1]
    for i in range(len(T.z)):
        z = T.z[i]
        for a in range(n):
            for b in range(n):
                if a == b:
                    continue
                A = np.zeros((n, n))
                A[a, b] = z[a, b]
                H += model.lamb_S(float(T.E[b] - T.E[a]), inst.eta, float(wc[i]), inst.T) * (A.T @ A)
        A0 = np.diag(np.diag(z))
        H += model.lamb_S(0.0, inst.eta, float(wc[i]), inst.T) * (A0.T @ A0)
    return H


def liouvillian_correlated(T, inst, zq) -> np.ndarray:
    """Eq. ME2-L with the bath model's gamma_ab(w) (model.gamma_matrix: C_ab gamma(w), or
    a sum of such terms with their own cutoffs), written as the double sum over qubits
    a, b of sum_w gamma_ab(w) (L_b,w rho L_a,w^dag - {L_a,w^dag L_b,w, rho} / 2), with
    the per-qubit operators of the Bohr-frequency grouping (one per a != b pair of
    levels, one omega = 0 operator) built from zq[q] = <a|sz_q|b>; no factorisation of
    gamma_ab(w).  Column-stacked superoperator (no Lamb shift)."""
    n = len(T.E)
    nq = inst.n_qubits
    I = np.eye(n)
    H = np.diag(T.E).astype(np.complex128)
    Lsup = -1j * (np.kron(I, H) - np.kron(H.T, I))

    def add(ops, w):
        nonlocal Lsup
        G = model.gamma_matrix(inst, w)
        for qa in range(nq):
            for qb in range(nq):
                c = G[qa, qb]
                if c == 0.0:
                    continue
                La, Lb = ops[qa], ops[qb]
                LdL = La.conj().T @ Lb
                Lsup = Lsup + c * (np.kron(La.conj(), Lb) - 0.5 * (np.kron(I, LdL) + np.kron(LdL.T, I)))

    for a in range(n):
        for b in range(n):
            if a == b:
                continue
            ops = []
            for q in range(nq):
                L = np.zeros((n, n))
                L[a, b] = zq[q][a, b]
                ops.append(L)
            add(ops, float(T.E[b] - T.E[a]))
    add([np.diag(np.diag(zq[q])) for q in range(nq)], 0.0)
    return Lsup


def liouvillian(T, inst) -> np.ndarray:
    """Superoperator of drho/dt = -i[H, rho] + sum_k (L rho L^+ - {L^+L, rho}/2), column-stacked."""
    n = len(T.E)
    I = np.eye(n)
    H = np.diag(T.E).astype(np.complex128)
    if getattr(inst, "lamb_shift", False):
        H = H + lamb_hamiltonian(T, inst)
    Lsup = -1j * (np.kron(I, H) - np.kron(H.T, I))
    for L in lindblad_operators(T, inst):
        LdL = L.conj().T @ L
        Lsup += np.kron(L.conj(), L) - 0.5 * (np.kron(I, LdL) + np.kron(LdL.T, I))
    return Lsup


def continuous(inst, s_eval, rtol=1e-10, atol=1e-12):
    """Lab-frame AME integrated in t; returns instantaneous ground-state populations at s_eval."""
    if getattr(inst, "lamb_shift", False):
        raise NotImplementedError("the continuous AME is built without the Lamb shift")
    nq, N = inst.n_qubits, inst.dim
    HX = model.hx_dense(nq)
    HZ = model.hz_dense(inst.h, inst.J)
    WC = model.bath_channels(inst)[1]                 # cutoff of each channel
    g0 = float(model.gamma_ohmic(0.0, inst.eta, inst.omega_c, inst.T))

    def H_at(t):
        a, b = model.schedule(inst.A_ctrl, inst.B_ctrl, t / inst.t_f)
        return a * HX + b * HZ

    def rhs(t, y):
        rho = y.reshape(N, N)
        E, V = np.linalg.eigh(H_at(t))
        rt = V.T @ rho @ V                      # eigenbasis
        d = -1j * (E[:, None] - E[None, :]) * rt
        omega = E[None, :] - E[:, None]
        p = np.real(np.diag(rt))
        zs = model.channel_matrix_elements(inst, V)
        for i in range(len(zs)):
            gam = model.gamma_ohmic(omega, inst.eta, WC[i], inst.T)
            np.fill_diagonal(gam, g0)
            z = zs[i]
            R = gam * z * z                      # R[a, b]: rate b -> a (diag: g0 z_bb^2)
            zd = np.diag(z)
            # pair channels a != b: A = sqrt(R_ab)|a><b|
            Roff = R.copy()
            np.fill_diagonal(Roff, 0.0)
            gain = Roff @ p
            loss = Roff.sum(axis=0)              # sum_a R[a, b] for each b
            d += np.diag(gain)
            d -= 0.5 * (loss[:, None] + loss[None, :]) * rt
            # omega = 0 channel: D = sqrt(g0) diag(z)
            d += g0 * (zd[:, None] * rt * zd[None, :]) - 0.5 * g0 * (zd[:, None] ** 2 + zd[None, :] ** 2) * rt
        return (V @ d @ V.T).ravel()

    E0, V0 = np.linalg.eigh(H_at(0.0))
    psi0 = V0[:, 0].astype(np.complex128)
    y0 = np.outer(psi0, psi0.conj()).ravel()
    t_eval = np.asarray(s_eval) * inst.t_f
    sol = solve_ivp(rhs, (0.0, inst.t_f), y0, method="DOP853", t_eval=t_eval, rtol=rtol, atol=atol)
    out = []
    for t, y in zip(sol.t, sol.y.T):
        E, V = np.linalg.eigh(H_at(t))
        rho = y.reshape(N, N)
        out.append(float(np.real(V[:, 0] @ rho @ V[:, 0])))
    return np.array(out)


def closed_system_lab(inst, s_eval, rtol=1e-11, atol=1e-13):
    """Schrodinger evolution in the lab frame; instantaneous ground-state population at s_eval."""
    nq = inst.n_qubits
    HX = model.hx_dense(nq)
    HZ = model.hz_dense(inst.h, inst.J)

    def H_at(t):
        a, b = model.schedule(inst.A_ctrl, inst.B_ctrl, t / inst.t_f)
        return a * HX + b * HZ

    E0, V0 = np.linalg.eigh(H_at(0.0))
    psi0 = V0[:, 0].astype(np.complex128)
    sol = solve_ivp(lambda t, y: -1j * (H_at(t) @ y), (0.0, inst.t_f), psi0, method="DOP853",
                    t_eval=np.asarray(s_eval) * inst.t_f, rtol=rtol, atol=atol)
    out = []
    for t, y in zip(sol.t, sol.y.T):
        E, V = np.linalg.eigh(H_at(t))
        out.append(float(np.abs(V[:, 0] @ y) ** 2))
    return np.array(out)
