"""Model layer of the FP64 oracle: Ising Hamiltonian, schedule, Ohmic bath.

TEST INFRASTRUCTURE: only tests/, the smoke check and the bench's cpu_baseline
leg may import anything under oracle/.

Sources in the paper:
  * transverse-field Ising Hamiltonian H_S = A H_X + B H_Z  (Sec. V, eq. H_S)
  * independent bosonic baths coupled through sz_i          (Sec. V, eq. SBm)
  * Ohmic rates gamma(w) = 2 pi g^2 w e^{-|w|/wc} / (1 - e^{-beta w})  (Sec. V)
  * KMS detailed balance gamma(-w) = e^{-beta w} gamma(w)   (Sec. II, eq. KMS)
Field-sign reading: H_Z = +sum h_i sz_i + sum_{i<j} J_ij sz_i sz_j (the paper
writes -sum h sz; the two differ by h -> -h).
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp

SX = np.array([[0.0, 1.0], [1.0, 0.0]])
SZ = np.array([[1.0, 0.0], [0.0, -1.0]])
I2 = np.eye(2)


def pauli_on(op: np.ndarray, i: int, n: int) -> np.ndarray:
    """Dense 2^n x 2^n operator acting with `op` on qubit i (bit i of the index)."""
    # np.kron puts its first factor on the most significant bits.
    return np.kron(np.kron(np.eye(1 << (n - 1 - i)), op), np.eye(1 << i))


def pauli_on_sparse(op: np.ndarray, i: int, n: int):
    return sp.kron(sp.kron(sp.identity(1 << (n - 1 - i), format="csr"), sp.csr_matrix(op)),
                   sp.identity(1 << i, format="csr"), format="csr")


def hx_dense(n: int) -> np.ndarray:
    return -sum(pauli_on(SX, i, n) for i in range(n))


def hz_dense(h: np.ndarray, J: np.ndarray) -> np.ndarray:
    n = len(h)
    H = sum(h[i] * pauli_on(SZ, i, n) for i in range(n))
    for i in range(n):
        for j in range(i + 1, n):
            if J[i, j] != 0.0:
                H = H + J[i, j] * (pauli_on(SZ, i, n) @ pauli_on(SZ, j, n))
    return H


def hx_sparse(n: int):
    return -sum(pauli_on_sparse(SX, i, n) for i in range(n))


def hz_diag(h: np.ndarray, J: np.ndarray) -> np.ndarray:
    """Diagonal of H_Z in the computational basis (sz eigenvalue +1 for bit 0)."""
    n = len(h)
    x = np.arange(1 << n)
    sig = 1.0 - 2.0 * ((x[None, :] >> np.arange(n)[:, None]) & 1)   # [n, N]
    e = (h[:, None] * sig).sum(axis=0)
    for i in range(n):
        for j in range(i + 1, n):
            if J[i, j] != 0.0:
                e = e + J[i, j] * sig[i] * sig[j]
    return e


def sz_diag(i: int, n: int) -> np.ndarray:
    x = np.arange(1 << n)
    return 1.0 - 2.0 * ((x >> i) & 1)


def schedule(A_ctrl: np.ndarray, B_ctrl: np.ndarray, s):
    """Piecewise-linear A(s), B(s) through control points at s_j = j/(n_ctrl - 1)."""
    A_ctrl = np.asarray(A_ctrl, dtype=np.float64)
    B_ctrl = np.asarray(B_ctrl, dtype=np.float64)
    knots = np.linspace(0.0, 1.0, len(A_ctrl))
    return np.interp(s, knots, A_ctrl), np.interp(s, knots, B_ctrl)


def hamiltonian_dense(inst, s: float) -> np.ndarray:
    a, b = schedule(inst.A_ctrl, inst.B_ctrl, s)
    return a * hx_dense(inst.n_qubits) + b * hz_dense(inst.h, inst.J)


def hamiltonian_sparse(inst, s: float):
    a, b = schedule(inst.A_ctrl, inst.B_ctrl, s)
    return (a * hx_sparse(inst.n_qubits) + sp.diags(b * hz_diag(inst.h, inst.J))).tocsr()


def gamma_ohmic(omega, eta: float, omega_c: float, T: float):
    """Ohmic bath correlation function (Sec. V) with g^2 = eta; gamma(0) is its limit 2 pi eta T."""
    omega = np.asarray(omega, dtype=np.float64)
    beta = 1.0 / T
    out = np.empty_like(omega)
    nz = omega != 0.0
    w = omega[nz]
    with np.errstate(over="ignore"):   # expm1 -> inf far below zero frequency: gamma -> 0
        out[nz] = 2.0 * math.pi * eta * w * np.exp(-np.abs(w) / omega_c) / (-np.expm1(-beta * w))
    out[~nz] = 2.0 * math.pi * eta / beta
    return out


def lamb_S(omega: float, eta: float, omega_c: float, T: float) -> float:
    """Lamb-shift function of the Ohmic bath: the principal value
    S(w) = (1/2pi) P int gamma(w') / (w - w') dw' (the imaginary part of the one-sided
    transform of the bath correlation function, whose real part is gamma / 2), written
    with w' = w -+ u as the regular integral (1/2pi) int_0^inf [gamma(w - u) - gamma(w + u)] / u du.
    gamma has a kink at zero frequency (the |w| of the cutoff), i.e. at u = |w|: the
    integral is split there."""
    import warnings
    import scipy.integrate as si
    w = float(omega)

    def f(u):
        return float(gamma_ohmic(w - u, eta, omega_c, T) - gamma_ohmic(w + u, eta, omega_c, T)) / u

    a = abs(w)
    edges = [0.0, a] if a > 0.0 else [0.0]
    edges += [a + 40.0 * T, a + 40.0 * T + 60.0 * omega_c]
    total = 0.0
    with warnings.catch_warnings():   # quad reports rounding once the 1e-13 target is reached
        warnings.simplefilter("ignore", si.IntegrationWarning)
        for lo, hi in zip(edges[:-1], edges[1:]):
            total += si.quad(f, lo, hi, epsabs=1e-16, epsrel=1e-13, limit=400)[0]
        total += si.quad(f, edges[-1], np.inf, epsabs=1e-16, epsrel=1e-13, limit=200)[0]
    return total / (2.0 * math.pi)


def lamb_S_zero_temperature(omega, eta: float, omega_c: float):
    """S(w) of the Ohmic bath at T = 0 in closed form: eta (-wc + w e^{-w/wc} Ei(w/wc))."""
    import scipy.special as ss
    w = np.asarray(omega, dtype=np.float64)
    return eta * (-omega_c + w * np.exp(-w / omega_c) * ss.expi(w / omega_c))


def psd_factor(C, rel_tol: float = 1e-12) -> np.ndarray:
    """F with C = F F^T for a symmetric positive semidefinite C: the Cholesky recursion
    column by column in natural order, where a column whose pivot falls to
    rel_tol * max(diag C) or below is dropped (its entries vanish for a semidefinite C),
    so F has one column per direction of the range of C."""
    C = np.asarray(C, dtype=np.float64)
    q = C.shape[0]
    tol = rel_tol * float(np.max(np.diag(C)))
    L = np.zeros((q, q))
    keep = []
    for j in range(q):
        d = C[j, j] - sum(L[j, k] ** 2 for k in keep)
        if d <= tol:
            continue
        L[j, j] = math.sqrt(d)
        for i in range(j + 1, q):
            L[i, j] = (C[i, j] - sum(L[i, k] * L[j, k] for k in keep)) / L[j, j]
        keep.append(j)
    return L[:, keep]


def bath_channels(inst):
    """Jump channels of the bath model (Sec. II eq. ME2-L): diagonal coupling operators
    [n_channels, 2^n] and the cutoff frequency of each channel's Ohmic rate.

    Independent baths: sz_i of each qubit.  Correlated baths gamma_ab(w) = C_ab gamma(w):
    with C = L L^T (Cholesky; C positive definite) the double sum over qubits becomes a sum
    over channels k with operators sum_a L[a, k] sz_a, each with rate gamma(w).
    Frequency-dependent correlations gamma_ab(w) = sum_m C_m[a, b] gamma(w; omega_c,m)
    (the bath terms; each C_m positive semidefinite): the same construction per term with
    C_m = F_m F_m^T (psd_factor), channels in term order, each term's columns with its own
    cutoff.  In every case sum_k F[a, k] F[b, k] gamma_k(w) = gamma_ab(w), so the channels
    give the dissipator of the double sum at every Bohr frequency; they stand in for the
    frequency-dependent rotation u(w) that diagonalises gamma_ab(w)."""
    n = inst.n_qubits
    sz = np.stack([sz_diag(i, n) for i in range(n)])
    terms = getattr(inst, "bath_terms", None)
    C = getattr(inst, "bath_corr", None)
    cp = getattr(inst, "coupling", None)
    if cp is not None:
        if C is not None or terms is not None:
            raise ValueError("give one of coupling, bath correlation or bath terms")
        cz = np.asarray(cp[0], dtype=np.float64)
        wc = np.full(len(cz), float(inst.omega_c)) if cp[2] is None else np.asarray(cp[2], dtype=np.float64)
        return cz @ sz, wc
    if terms is not None:
        if C is not None:
            raise ValueError("give either a constant correlation or bath terms")
        ws, wcs = [], []
        for Cm, wc in terms:
            F = psd_factor(Cm)
            ws.append(F.T @ sz)
            wcs += [float(wc)] * F.shape[1]
        return np.concatenate(ws), np.array(wcs)
    if C is None:
        return sz, np.full(n, float(inst.omega_c))
    L = np.linalg.cholesky(np.asarray(C, dtype=np.float64))
    return L.T @ sz, np.full(n, float(inst.omega_c))


def channel_sx(inst):
    """sx coefficients of the channels' coupling operators, [n_channels, n_qubits], or None
    when every channel couples through sz only.  A coupling (cz, cx, omega_c) gives channel
    k the operator sum_a (cz[k, a] sz_a + cx[k, a] sx_a) (Sec. II: the system part of the
    system-bath coupling; real, so every matrix element in the real eigenbasis is real)."""
    cp = getattr(inst, "coupling", None)
    if cp is None or cp[1] is None:
        return None
    cx = np.asarray(cp[1], dtype=np.float64)
    return None if not np.any(cx) else cx


def channel_matrix_elements(inst, V: np.ndarray) -> np.ndarray:
    """z[k] = V^T O_k V for each channel operator O_k (bath_channels' diagonal part plus
    channel_sx's sx part, sx_a V permuting the rows x -> x ^ 2^a), [n_channels, n, n]."""
    w, _ = bath_channels(inst)
    cx = channel_sx(inst)
    x = np.arange(V.shape[0])
    z = np.empty((len(w), V.shape[1], V.shape[1]))
    for k in range(len(w)):
        OV = w[k][:, None] * V
        if cx is not None:
            for a in range(inst.n_qubits):
                if cx[k, a] != 0.0:
                    OV = OV + cx[k, a] * V[x ^ (1 << a)]
        z[k] = V.T @ OV
    return z


def channel_weights(inst) -> np.ndarray:
    """The channels' diagonal coupling operators, [n_channels, 2^n] (bath_channels)."""
    return bath_channels(inst)[0]


def gamma_matrix(inst, omega: float) -> np.ndarray:
    """gamma_ab(w) of the bath model as an n_qubits x n_qubits matrix, from its definition
    (no factorisation): gamma(w) I, C gamma(w), or sum_m C_m gamma(w; omega_c,m)."""
    n = inst.n_qubits
    terms = getattr(inst, "bath_terms", None)
    if terms is not None:
        out = np.zeros((n, n))
        for Cm, wc in terms:
            out += np.asarray(Cm, dtype=np.float64) * float(gamma_ohmic(omega, inst.eta, float(wc), inst.T))
        return out
    C = getattr(inst, "bath_corr", None)
    C = np.eye(n) if C is None else np.asarray(C, dtype=np.float64)
    return C * float(gamma_ohmic(omega, inst.eta, inst.omega_c, inst.T))
