"""Spectral layer of the FP64 oracle: instantaneous eigenbasis and AME tables.

TEST INFRASTRUCTURE: only tests/, the smoke check and the bench's cpu_baseline
leg may import anything under oracle/.

What is computed, per grid point s_g = g/(M-1), g = 0..M-1, t = s t_f:

* eigenpairs of H(s_g) in ascending order (numpy eigh for dense sizes, scipy
  eigsh from a seeded random start for the 2^16 gadget), the "instantaneous energy eigenstates" of
  Sec. II (eq. Lindblad2);
* clusters: maximal runs of consecutive levels whose gaps are below deg_tol.
  Inside a cluster the basis is rotated to the eigenbasis of the projected
  diagonal operator W = diag(x) (x = computational basis index), ordered by
  its eigenvalue, and the energies become Rayleigh quotients.  This makes the
  basis reproducible when levels are (numerically) degenerate; at s = 1 it is
  the computational basis.  Reading of the paper's Kronecker delta over Bohr
  frequencies: a != b pairs are separate channels, the a == b terms of each
  qubit form the single omega = 0 operator;
* column signs: the first component whose magnitude is within 1e-9 of the
  column maximum is made positive (a gauge choice; no physical result
  depends on it);
* truncation to the n lowest levels;
* per grid g >= 1 the tables used by the step that ends at s_g (generator
  frozen at the right end point):
    O_g     = polar factor of V_g^T V_{g-1}     (basis change, g >= 2; directions
              with singular value <= 1e-4, lost by the truncation, are completed
              in a canonical basis so that O_g stays orthogonal)
    c_init  = V_1^T psi_0 / |V_1^T psi_0|      (g = 1; psi_0 = ground state of H(s_0))
    z_g[i,a,b] = <a| sz_i |b>                   (eq. Lindblad2 matrix elements)
    R_g[i,b,a] = gamma(e_b - e_a) z^2 (a != b), gamma(0) z_bb^2 (a == b)
                 = |A_i psi|^2 per unit population of level b (eq. Aired, eq. 12)
    Gamma_g[b] = sum_{i,a} R_g[i,b,a]          (diagonal of sum_i A_i^dag A_i, eq. Heff)
    d_g[b]     = exp(-i e_b dt - Gamma_b dt / 2)
    leak_g     = 1 - sigma_min(V_g^T V_{g-1})^2  (diagnostic of truncation)
"""
from __future__ import annotations

import dataclasses
from typing import Iterator, Optional

import numpy as np
import scipy.sparse.linalg as spla

from . import model


@dataclasses.dataclass
class GridTables:
    g: int
    s: float
    E: np.ndarray            # [n]
    gs: int                  # size of the ground cluster
    O: Optional[np.ndarray]  # [n, n] (None at g = 1)
    cinit: Optional[np.ndarray]  # [n] (g = 1 only)
    z: np.ndarray            # [nq, n, n]
    R: np.ndarray            # [nq, n(b), n(a)]
    Gamma: np.ndarray        # [n]
    zdiag: np.ndarray        # [nq, n]
    d: np.ndarray            # [n] complex
    leak: float
    V: Optional[np.ndarray] = None   # [N, n] (kept only on request)
    shift: Optional[np.ndarray] = None   # [n] Lamb shift of each level (zeros when off)
    dt: float = 0.0          # length of the step into this grid point (ns)
    t0: float = 0.0          # time at its start (ns)

    @property
    def Eph(self) -> np.ndarray:
        """Energies that set the phases: e_b plus the Lamb shift."""
        return self.E if self.shift is None else self.E + self.shift


def clusters(E: np.ndarray, deg_tol: float):
    """List of (start, stop) index ranges of consecutive levels closer than deg_tol."""
    out = []
    a0 = 0
    for a in range(1, len(E) + 1):
        if a == len(E) or E[a] - E[a - 1] >= deg_tol:
            out.append((a0, a))
            a0 = a
    return out


def canonicalize(E: np.ndarray, V: np.ndarray, deg_tol: float):
    """Rotate degenerate clusters to the W = diag(x) eigenbasis; fix column signs.

    Returns (E, V, clusters) with the clusters found before the rotation.
    """
    E = E.copy()
    V = V.copy()
    w = np.arange(V.shape[0], dtype=np.float64)
    cl = clusters(E, deg_tol)
    for a0, a1 in cl:
        if a1 - a0 < 2:
            continue
        Vc = V[:, a0:a1]
        G = Vc.T @ (w[:, None] * Vc)
        _, Q = np.linalg.eigh(0.5 * (G + G.T))
        V[:, a0:a1] = Vc @ Q
        E[a0:a1] = (Q * Q).T @ E[a0:a1]
    mags = np.abs(V)
    mx = mags.max(axis=0)
    first = np.argmax(mags >= (1.0 - 1e-9) * mx[None, :], axis=0)
    sgn = np.sign(V[first, np.arange(V.shape[1])])
    sgn[sgn == 0] = 1.0
    return E, V * sgn[None, :], cl


def eigen(inst, s: float, n_keep: int, deg_tol: float, guard: int = 16, method: str = "auto"):
    """Lowest n_keep canonical eigenpairs of H(s) plus the ground-cluster size.

    Dense eigh up to 4096 states, else ARPACK Lanczos (eigsh).  Lanczos starts from a
    seeded random vector: a structured start such as the uniform superposition lies in
    one symmetry sector of H (for instance the qubit-permutation symmetric sector of the
    two-cluster gadget) and would miss every level outside it.  A single Krylov sequence
    also resolves degenerate levels only through its restarts, which needs room: it is
    asked for 2 (n_keep + guard) pairs, of which the lowest n_keep + guard are used."""
    N = inst.dim
    if method == "dense" or (method == "auto" and N <= 4096):
        E, V = np.linalg.eigh(model.hamiltonian_dense(inst, s))
    else:
        k = min(N - 2, 2 * (n_keep + guard))
        H = model.hamiltonian_sparse(inst, s)
        v0 = np.random.default_rng(20171009).standard_normal(N)
        E, V = spla.eigsh(H, k=k, which="SA", tol=1e-13, v0=v0)
        o = np.argsort(E)[: n_keep + guard]
        E, V = E[o], V[:, o]
    E, V, cl = canonicalize(E, V, deg_tol)
    gs = cl[0][1] - cl[0][0]
    return E[:n_keep], V[:, :n_keep], gs


def _sign_fixed(v: np.ndarray) -> np.ndarray:
    mags = np.abs(v)
    first = int(np.argmax(mags >= (1.0 - 1e-9) * mags.max()))
    return v if v[first] >= 0 else -v


def _canonical_basis(P: np.ndarray, k: int) -> np.ndarray:
    """k orthonormal columns spanning the range of the projector P, made unique by
    diagonalising P diag(1..n) P (generic weights) and the column sign rule."""
    n = P.shape[0]
    K = P @ np.diag(np.arange(1.0, n + 1.0)) @ P
    w, Q = np.linalg.eigh(0.5 * (K + K.T))
    cols = [_sign_fixed(Q[:, j]) for j in range(n - k, n)]   # the k non-zero eigenvalues, ascending
    return np.stack(cols, axis=1)


def polar(M: np.ndarray, tau: float = 1e-4):
    """Polar factor U W^T of M (SVD).  Directions with singular value <= tau carry no
    overlap (the retained subspace lost them); they are mapped onto the left directions
    not reached by the others, both taken in the canonical basis above, so the factor
    stays orthogonal and reproducible."""
    U, S, Wt = np.linalg.svd(M)
    good = S > tau
    P = U[:, good] @ Wt[good]
    k = int((~good).sum())
    if k:
        n = M.shape[0]
        right = _canonical_basis(Wt[~good].T @ Wt[~good], k)
        left = _canonical_basis(np.eye(n) - U[:, good] @ U[:, good].T, k)
        P = P + left @ right.T
    return P, S


def grid_tables(inst, E: np.ndarray, V: np.ndarray, dt: float):
    n = len(E)
    wc = model.bath_channels(inst)[1]                    # cutoff of each channel
    z = model.channel_matrix_elements(inst, V)           # [channel, a, b]
    nch = len(z)
    omega = E[None, :] - E[:, None]                      # omega[a, b] = E_b - E_a
    R = np.empty((nch, n, n))
    for i in range(nch):
        gam = model.gamma_ohmic(omega, inst.eta, wc[i], inst.T)
        np.fill_diagonal(gam, model.gamma_ohmic(0.0, inst.eta, wc[i], inst.T))
        R[i] = (gam * z[i] ** 2).T                        # R[i, b, a]
    Gamma = R.sum(axis=(0, 2))
    zdiag = np.stack([np.diag(z[i]) for i in range(nch)])
    shift = lamb_shift(inst, E, z) if getattr(inst, "lamb_shift", False) else np.zeros(n)
    d = np.exp(-1j * (E + shift) * dt - 0.5 * Gamma * dt)
    return z, R, Gamma, zdiag, d, shift


def lamb_shift(inst, E: np.ndarray, z: np.ndarray) -> np.ndarray:
    """Diagonal of H_LS = sum_i sum_w S(w) A_i,w^dag A_i,w in the eigenbasis (Sec. II,
    eq. ME2-H; the operators of the Bohr-frequency reading): level b collects
    S(e_b - e_a) z_i[a,b]^2 from every a != b and S(0) z_i[b,b]^2 from the omega = 0
    operator of each jump channel i, S taken with that channel's cutoff."""
    n = len(E)
    wc = model.bath_channels(inst)[1]                  # each channel's S uses its cutoff
    cache = {}

    def S(w, c):
        key = (w, float(c))
        if key not in cache:
            cache[key] = model.lamb_S(w, inst.eta, float(c), inst.T)
        return cache[key]

    out = np.zeros(n)
    for b in range(n):
        acc = 0.0
        for i in range(len(z)):
            for a in range(n):
                w = 0.0 if a == b else float(E[b] - E[a])
                acc += S(w, wc[i]) * z[i, a, b] ** 2
        out[b] = acc
    return out


def grid_points(inst, M: int):
    """The instance's s-grid (None: equidistant), checked: M points from 0 to 1, increasing."""
    sg = getattr(inst, "s_grid", None)
    if sg is None:
        return None
    sg = np.asarray(sg, dtype=np.float64)
    if len(sg) != M or sg[0] != 0.0 or sg[-1] != 1.0 or not np.all(np.diff(sg) > 0.0):
        raise ValueError("s_grid must hold n_grid increasing points from 0 to 1")
    return sg


def step_bound(inst, s: np.ndarray, deg_tol: float = 1e-8) -> np.ndarray:
    """The time-step bound of App. B (eq. B7) at the points s (full spectrum):
    min{ |H_eff| / |dH_eff/dt|, 1 / |H_eff|, |lambda / (lambda^2 - dlambda/dt)| } with
    |.| the operator norm.  H_eff = H - (i/2) sum A^dag A is diag(e - i Gamma / 2) in the
    eigenbasis (the decay is diagonal there), so |H_eff| = max_b |e_b - i Gamma_b / 2|
    and the lab-frame H_eff = V diag(e - i Gamma / 2) V^T; its time derivative is taken
    by central differences in s (one-sided at the ends).  lambda, the jump rate, depends
    on the trajectory's state; the bound uses its largest value, max_b Gamma_b."""
    n = inst.dim
    Hs, lam, nrm = [], [], []
    for x in s:
        E, V, _ = eigen(inst, float(x), n, deg_tol)
        _, _, Gamma, _, _, _ = grid_tables(inst, E, V, 1.0)
        h = E - 0.5j * Gamma
        Hs.append((V * h[None, :]) @ V.T)
        nrm.append(float(np.abs(h).max()))
        lam.append(float(Gamma.max()))
    Hs, lam, nrm = np.array(Hs), np.array(lam), np.array(nrm)
    t = np.asarray(s, dtype=np.float64) * inst.t_f
    dH = np.gradient(Hs, t, axis=0)
    dlam = np.gradient(lam, t)
    dHn = np.array([np.linalg.norm(m, 2) for m in dH])
    with np.errstate(divide="ignore", invalid="ignore"):
        b1 = np.where(dHn > 0.0, nrm / dHn, np.inf)
        b2 = 1.0 / nrm
        den = lam * lam - dlam
        b3 = np.where(den != 0.0, np.abs(lam / den), np.inf)
    return np.minimum(np.minimum(b1, b2), b3)


def bound_grid(inst, n_grid: int, n_probe: int = 401, deg_tol: float = 1e-8) -> np.ndarray:
    """An s-grid whose local step follows the App. B bound (eq. B7): the density of
    grid points is 1 / bound(s), equidistributed -- s_g solves F(s_g) = g F(1) / (M - 1)
    with F(s) = int_0^s ds' / bound(s'), the integral by the trapezoid rule on
    n_probe equidistant points and the inverse by linear interpolation."""
    sp = np.linspace(0.0, 1.0, n_probe)
    rho = 1.0 / step_bound(inst, sp, deg_tol)
    F = np.concatenate([[0.0], np.cumsum(0.5 * (rho[1:] + rho[:-1]) * np.diff(sp))])
    target = np.linspace(0.0, F[-1], n_grid)
    out = np.interp(target, F, sp)
    out[0], out[-1] = 0.0, 1.0
    return out


def n_steps_dt(inst, n_grid: int):
    return n_grid - 1, inst.t_f / (n_grid - 1)


def table_stream(inst, n_grid: Optional[int] = None, n_levels: Optional[int] = None,
                 deg_tol: float = 1e-8, keep_V: bool = False,
                 grids: Optional[set] = None) -> Iterator[GridTables]:
    """Yield GridTables for g = 1..M-1 in order (or only those in `grids`, still in order)."""
    M = n_grid or inst.n_grid
    n = n_levels or inst.levels
    sg = grid_points(inst, M)
    dt = inst.t_f / (M - 1)
    E0, V0, gs0 = eigen(inst, 0.0, max(n, 1), deg_tol)
    if gs0 != 1:
        raise ValueError("ground state of H(s=0) is degenerate; initial state undefined")
    psi0 = V0[:, 0]
    Vprev = None
    for g in range(1, M):
        if sg is None:      # equidistant: s_g = g / (M - 1), steps of t_f / (M - 1)
            s, s_prev, t0, dtg = g / (M - 1), (g - 1) / (M - 1), (g - 1) * dt, dt
        else:
            # The factor of grid point g (its phases and decay) acts between the basis
            # changes into g and out of g, so it covers half of each neighbouring step:
            # (h_g + h_{g+1}) / 2, h_g = t_f (s_g - s_{g-1}); the last point takes
            # (h_{M-1} + h_1) / 2, the half step the first point's factor leaves out,
            # so the lengths add up to t_f.  A symmetric splitting of each step, which
            # on equidistant points gives h as above.
            s, s_prev = float(sg[g]), float(sg[g - 1])
            s_next = float(sg[g + 1]) if g < M - 1 else 1.0 + float(sg[1])
            t0 = 0.5 * inst.t_f * (s_prev + s - float(sg[1]))
            dtg = 0.5 * inst.t_f * (s_next - s_prev)
        need_prev = grids is not None and (g + 1) in grids
        if grids is not None and g not in grids and not need_prev:
            Vprev = None
            continue
        E, V, gs = eigen(inst, s, n, deg_tol)
        if g == 1:
            c = V.T @ psi0
            leak = 1.0 - float(c @ c)
            cinit, O = c / np.linalg.norm(c), None
        else:
            if Vprev is None:
                _, Vp, _ = eigen(inst, s_prev, n, deg_tol)
            else:
                Vp = Vprev
            O, S = polar(V.T @ Vp)
            leak = 1.0 - float(S.min()) ** 2
            cinit = None
        z, R, Gamma, zdiag, d, shift = grid_tables(inst, E, V, dtg)
        Vprev = V
        if grids is None or g in grids:
            yield GridTables(g=g, s=s, E=E, gs=gs, O=O, cinit=cinit, z=z, R=R, Gamma=Gamma,
                             zdiag=zdiag, d=d, leak=leak, V=V if keep_V else None, shift=shift,
                             dt=dtg, t0=t0)


def all_tables(inst, **kw):
    return list(table_stream(inst, **kw))

