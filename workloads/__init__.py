"""Seeded synthetic workloads for the adiabatic quantum-trajectory engine.

This module only draws inputs: Ising fields and couplings, schedule control
points, bath constants and run sizes.  It holds none of the method's
arithmetic, so both the FP64 CPU oracle and the GPU library may consume it.

Units follow the paper (hbar = k_B = 1): energies, rates and temperatures are
angular frequencies in rad/ns, times are in ns.  The paper quotes its
temperatures as "GHz" in these units; 12 mK maps to 1.57 and 20 mK to 2.62
(Sec. V, the 8-qubit and 16-qubit case studies), which is the angular reading
implemented by `kelvin_to_rad_per_ns`.

Hamiltonian convention used throughout the project:
    H(s) = A(s) * (-sum_i sx_i) + B(s) * (sum_i h_i sz_i + sum_{i<j} J_ij sz_i sz_j)
with bit i of a basis index x carrying qubit i and sz_i|x> = (1 - 2 bit_i(x))|x>.
The paper writes the field term with a minus sign (Sec. V, transverse-field
Ising model); passing -h reproduces that convention exactly.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

K_B = 1.380649e-23          # J/K (exact, SI 2019)
HBAR = 1.054571817e-34      # J s (exact, SI 2019)

TWO_PI = 2.0 * math.pi


def kelvin_to_rad_per_ns(t_kelvin: float) -> float:
    """Temperature k_B T / hbar expressed in rad/ns."""
    return K_B * t_kelvin / HBAR * 1e-9


@dataclasses.dataclass
class Instance:
    """One annealing instance plus the run parameters quoted with it."""
    name: str
    n_qubits: int
    h: np.ndarray                 # [n_qubits] float64
    J: np.ndarray                 # [n_qubits, n_qubits] float64, upper triangle (i<j) used
    t_f: float                    # ns
    A_ctrl: np.ndarray            # schedule control points, rad/ns, at s_j = j/(n_ctrl-1)
    B_ctrl: np.ndarray
    eta: float = 1e-4             # dimensionless coupling (the paper's g^2)
    omega_c: float = 8.0 * math.pi
    T: float = kelvin_to_rad_per_ns(0.012)
    lamb_shift: bool = False      # include the Lamb-shift Hamiltonian of the Ohmic bath
    bath_corr: Optional[np.ndarray] = None   # [n_qubits, n_qubits] correlation C of the baths
                                             # (gamma_ab(w) = C_ab gamma(w)); None = independent
    bath_terms: Optional[tuple] = None       # ((C_m, omega_c_m), ...): gamma_ab(w) =
                                             # sum_m C_m[a, b] gamma(w; omega_c_m), C_m PSD
    coupling: Optional[tuple] = None         # (cz, cx, omega_c): channel k couples through
                                             # sum_a cz[k][a] sz_a + cx[k][a] sx_a with an
                                             # independent bath (cutoff omega_c[k]; None = omega_c)
    n_grid: int = 1001            # s-grid points (n_grid - 1 steps)
    s_grid: Optional[np.ndarray] = None   # [n_grid] grid points 0 = s_0 < ... < s_{M-1} = 1;
                                          # None = equidistant
    n_levels: int = 0             # retained levels; 0 = full spectrum
    n_traj: int = 1000
    seed: int = 0                 # trajectory-stream seed (Philox key word 0)
    instance_id: int = 0          # Philox key word 1

    @property
    def dim(self) -> int:
        return 1 << self.n_qubits

    @property
    def levels(self) -> int:
        return self.n_levels if self.n_levels > 0 else self.dim

    def with_(self, **kw) -> "Instance":
        return dataclasses.replace(self, **kw)


def linear_schedule(n_ctrl: int = 2):
    """A(s) = 2*pi*(1-s), B(s) = 2*pi*s rad/ns sampled at n_ctrl equispaced points."""
    s = np.linspace(0.0, 1.0, n_ctrl)
    return TWO_PI * (1.0 - s), TWO_PI * s


def _edges_ring(n: int):
    return sorted({(min(i, (i + 1) % n), max(i, (i + 1) % n)) for i in range(n)})


def _edges_all(n: int):
    return [(i, j) for i in range(n) for j in range(i + 1, n)]


def _draw(rng, n, edges, kind):
    """Draw h_0..h_{n-1} first, then J over the edge list (i<j, lexicographic)."""
    if kind == "uniform":
        h = rng.uniform(-1.0, 1.0, size=n)
        jv = rng.uniform(-1.0, 1.0, size=len(edges))
    elif kind == "pm1":
        h = rng.choice(np.array([-1.0, 1.0]), size=n)
        jv = rng.choice(np.array([-1.0, 1.0]), size=len(edges))
    else:
        raise ValueError(kind)
    J = np.zeros((n, n))
    for (i, j), v in zip(edges, jv):
        J[i, j] = v
    return h.astype(np.float64), J


def ring_instance(n_qubits=4, seed=1001, **kw) -> Instance:
    rng = np.random.default_rng(seed)
    h, J = _draw(rng, n_qubits, _edges_ring(n_qubits), "uniform")
    A, B = linear_schedule()
    base = dict(name=f"ring{n_qubits}-seed{seed}", n_qubits=n_qubits, h=h, J=J,
                t_f=1000.0, A_ctrl=A, B_ctrl=B, n_grid=1001, n_traj=1000, seed=seed)
    base.update(kw)
    return Instance(**base)


def pm1_all_to_all(n_qubits, seed, **kw) -> Instance:
    rng = np.random.default_rng(seed)
    h, J = _draw(rng, n_qubits, _edges_all(n_qubits), "pm1")
    A, B = linear_schedule()
    base = dict(name=f"a2a{n_qubits}-seed{seed}", n_qubits=n_qubits, h=h, J=J,
                t_f=1.0e4, A_ctrl=A, B_ctrl=B, seed=seed)
    base.update(kw)
    return Instance(**base)


# Seed of the 8-qubit all-to-all +-1 instance: the first seed >= 1002 whose
# final (s = 1) Ising ground state is non-degenerate.  Chosen once by
# tests/golden/make_golden.py (which scans seeds with the oracle) and stored
# here as a plain constant.
A2A8_SEED = 1007


def config_small() -> Instance:
    """4-qubit ring, U[-1,1] couplings, full spectrum, 1000 trajectories x 1000 steps, FP64."""
    return ring_instance(4, 1001)


def config_a2a8(n_traj: int = 10_000) -> Instance:
    """8-qubit all-to-all +-1 instance, full spectrum (n = 256), 2000 grid points, t_f = 10 us."""
    return pm1_all_to_all(8, A2A8_SEED, n_grid=2000, n_traj=n_traj, t_f=1.0e4)


def config_gradient(n_traj: int = 100_000, n_ctrl: int = 16) -> Instance:
    """The 8-qubit all-to-all anneal with A(s) and B(s) given by n_ctrl piecewise-linear
    control points each (initialised to the linear schedule): the gradient workload."""
    A, B = linear_schedule(n_ctrl)
    return config_a2a8(n_traj).with_(A_ctrl=A, B_ctrl=B, name=f"a2a8-seed{A2A8_SEED}-ctrl{n_ctrl}")


def config_small_ctrl(n_traj: int = 100_000, n_ctrl: int = 16) -> Instance:
    """The 4-qubit ring workload with n_ctrl control points per schedule (gradient checks)."""
    A, B = linear_schedule(n_ctrl)
    return config_small().with_(A_ctrl=A, B_ctrl=B, n_traj=n_traj, name=f"ring4-seed1001-ctrl{n_ctrl}")


def gadget_instance(m: int, n_levels: int = 32, n_grid: int = 500, t_f: float = 1.0e4,
                    n_traj: int = 100_000, seed: int = 1604) -> Instance:
    """Two-cluster tunnelling gadget on 2m qubits: cluster A = qubits 0..m-1 (field
    +0.44), cluster B = qubits m..2m-1 (field -1); all-to-all J = -1 inside each cluster
    and J_{i,i+m} = -1 between them.  Permuting the qubits of A together with the same
    permutation of B is a symmetry, so H(s) has degenerate levels at every s."""
    n = 2 * m
    h = np.array([0.44] * m + [-1.0] * m)
    J = np.zeros((n, n))
    for c in (0, m):
        for i in range(c, c + m):
            for j in range(i + 1, c + m):
                J[i, j] = -1.0
    for i in range(m):
        J[i, i + m] = -1.0
    A, B = linear_schedule()
    return Instance(name=f"gadget{n}", n_qubits=n, h=h, J=J, t_f=t_f, A_ctrl=A, B_ctrl=B,
                    n_grid=n_grid, n_levels=n_levels, n_traj=n_traj, seed=seed)


def config_gadget(n_traj: int = 100_000) -> Instance:
    """16-qubit two-cluster tunnelling gadget truncated to the 32 lowest levels, 500 grid
    points, t_f = 10 us."""
    return gadget_instance(8, n_traj=n_traj)


def config_batched(n_instances: int = 256, seed: int = 2024, n_traj: int = 2048,
                   n_grid: int = 1000) -> List[Instance]:
    """Many small instances: n_q ~ U{6..10}, n ~ U{16,32,64}, t_f ~ 10^U[0,2] us, +-1 all-to-all."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n_instances):
        nq = int(rng.integers(6, 11))
        n = int(rng.choice([16, 32, 64]))
        tf = 1000.0 * 10.0 ** rng.uniform(0.0, 2.0)
        inst_seed = int(rng.integers(0, 2**31 - 1))
        inst = pm1_all_to_all(nq, inst_seed, t_f=tf, n_grid=n_grid, n_levels=min(n, 1 << nq),
                              n_traj=n_traj)
        inst = inst.with_(name=f"batch{k}-nq{nq}-n{n}", instance_id=k, seed=seed)
        out.append(inst)
    return out


def config_controls(n_ctrl: int = 16, n_traj: int = 100_000) -> Instance:
    """8-qubit instance with A(s), B(s) given by n_ctrl piecewise-linear control points."""
    base = config_a2a8(n_traj)
    A, B = linear_schedule(n_ctrl)
    return base.with_(A_ctrl=A, B_ctrl=B, name=base.name + f"-ctrl{n_ctrl}")


def two_level_fixed(A: float = 0.3, t_f: float = 200.0, n_grid: int = 101, **kw) -> Instance:
    """One qubit, H = -A sx held fixed (B = 0): the textbook two-level relaxation case."""
    base = dict(name="qubit-fixed", n_qubits=1, h=np.zeros(1), J=np.zeros((1, 1)), t_f=t_f,
                A_ctrl=np.array([A, A]), B_ctrl=np.array([0.0, 0.0]), n_grid=n_grid)
    base.update(kw)
    return Instance(**base)


def case0989() -> Instance:
    """The 8-qubit non-adiabatic instance printed in Sec. V (fields and couplings x 1/3).

    The paper prints it in its own convention (H_Z = -sum h sz + sum J sz sz); the
    field signs are flipped here to express it in this project's +h convention.
    Qubits are numbered 0..7 as in the printed couplings.
    """
    h_paper = np.array([-2, -2, 2, -3, 1, 3, -3, 3], dtype=np.float64) / 3.0
    J = np.zeros((8, 8))
    rows = {0: [1, -3, -1, -1], 1: [-1, -2, 2, -3], 2: [-2, -1, -3, -2], 3: [-3, -3, -1, -3]}
    for i, vals in rows.items():
        for j, v in zip(range(4, 8), vals):
            J[i, j] = v / 3.0
    A, B = linear_schedule()
    return Instance(name="case0989-linear", n_qubits=8, h=-h_paper, J=J, t_f=1.0e4,
                    A_ctrl=A, B_ctrl=B, n_grid=2000, T=kelvin_to_rad_per_ns(0.012))


def two_term_bath(n_qubits: int, rho: float = 0.5, common_cutoff: float = 2.0 * math.pi,
                  local_cutoff: float = 8.0 * math.pi, xi: float = 0.5):
    """A frequency-dependent bath correlation: local baths correlated as xi^|a-b| with the
    standard cutoff, plus one bath shared by all qubits (rank one, weight rho) with a
    lower cutoff.  The two correlation matrices do not commute, so the eigenvectors of
    gamma_ab(w) turn with w."""
    q = n_qubits
    C0 = np.array([[xi ** abs(a - b) for b in range(q)] for a in range(q)])
    C1 = rho * np.ones((q, q))
    return ((C0, local_cutoff), (C1, common_cutoff))
