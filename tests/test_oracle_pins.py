"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Each test names the passage or property it checks.  None of them retypes the
oracle's formula: they compare with closed forms, symmetries, brute-force
constructions, independent library routines or statistical laws.
"""
import dataclasses
import math

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.optimize as so
import scipy.stats as st

import workloads as W
from oracle import ame, model, philox, spectrum, trajectories


# ---------------------------------------------------------------- RNG -------
def _numpy_block(ctr, key):
    """numpy's Philox increments its counter before each block: start one below."""
    v = sum(int(c) << (64 * i) for i, c in enumerate(ctr)) - 1
    cm1 = np.array([(v >> (64 * i)) & (2**64 - 1) for i in range(4)], dtype=np.uint64)
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=cm1)
    return [int(x) for x in bg.random_raw(4)]


@pytest.mark.parametrize("ctr,key", [((1, 0, 0, 0), (0, 0)), ((5, 7, 0, 0), (123, 456)),
                                     ((2**64 - 1, 3, 0, 0), (2**63 + 5, 99)),
                                     ((977, 2**40 + 3, 0, 0), (1007, 0))])
def test_philox_matches_numpy(ctr, key):
    mine = [int(w) for w in philox.philox4x64_10([np.uint64(c) for c in ctr], key)]
    assert mine == _numpy_block(ctr, key)


def test_draw_map_and_open_interval():
    u = philox.uniform_from_word(np.array([0, 2**64 - 1], dtype=np.uint64))
    assert 0.0 < u[0] < 1e-15 and 1.0 - 1e-15 < u[1] < 1.0
    # draw idx uses word idx & 3 of block idx >> 2
    words = philox.philox4x64_10([np.uint64(11), np.uint64(2), np.uint64(0), np.uint64(0)], (5, 6))
    for w in range(4):
        assert philox.draw(5, 6, 11, 8 + w) == philox.uniform_from_word(words[w])
        assert philox.draw_scalar(5, 6, 11, 8 + w) == philox.uniform_from_word(words[w])


# ---------------------------------------------------------------- bath ------
def test_kms_detailed_balance():
    """Sec. II, eq. KMS: gamma(-w) = exp(-beta w) gamma(w)."""
    T = W.kelvin_to_rad_per_ns(0.012)
    w = np.concatenate([np.logspace(-9, 2.2, 300)])
    gp = model.gamma_ohmic(w, 1e-4, 8 * np.pi, T)
    gm = model.gamma_ohmic(-w, 1e-4, 8 * np.pi, T)
    np.testing.assert_allclose(gm, np.exp(-w / T) * gp, rtol=1e-13, atol=0)
    assert np.all(gp > 0) and np.all(gm >= 0)


def test_gamma_zero_is_the_limit():
    T = 1.3
    g0 = model.gamma_ohmic(0.0, 2e-4, 5.0, T)
    for eps in (1e-6, -1e-6, 1e-9, -1e-9):
        g = model.gamma_ohmic(eps, 2e-4, 5.0, T)
        assert abs(g / g0 - 1.0) < 2 * abs(eps) / T
    # large frequency: Bose factor -> 1, so gamma -> 2 pi eta w exp(-w / wc)
    w = 80.0
    np.testing.assert_allclose(model.gamma_ohmic(w, 2e-4, 5.0, T),
                               2 * np.pi * 2e-4 * w * np.exp(-w / 5.0), rtol=1e-12)


def test_temperature_units_match_paper_pairs():
    """Sec. V quotes 12 mK as 1.57 and 20 mK as 2.6 / 2.62 in hbar = 1 units."""
    assert abs(W.kelvin_to_rad_per_ns(0.012) - 1.57) < 0.005
    assert abs(W.kelvin_to_rad_per_ns(0.020) - 2.62) < 0.005


# ---------------------------------------------------------------- model -----
def test_ising_diagonal_by_bitstring_enumeration():
    inst = W.ring_instance(4, 1001)
    e = model.hz_diag(inst.h, inst.J)
    for x in range(16):
        sig = [1 - 2 * ((x >> i) & 1) for i in range(4)]
        ref = sum(inst.h[i] * sig[i] for i in range(4))
        ref += sum(inst.J[i, j] * sig[i] * sig[j] for i in range(4) for j in range(i + 1, 4))
        assert abs(e[x] - ref) < 1e-14
    np.testing.assert_allclose(np.diag(model.hz_dense(inst.h, inst.J)), e, atol=1e-14)


def test_transverse_field_flips_one_bit():
    H = model.hx_dense(3)
    for x in range(8):
        for y in range(8):
            want = -1.0 if bin(x ^ y).count("1") == 1 else 0.0
            assert H[x, y] == want


def test_one_qubit_spectrum_closed_form():
    inst = W.Instance(name="q", n_qubits=1, h=np.array([0.7]), J=np.zeros((1, 1)), t_f=10.0,
                      A_ctrl=np.array([2.0, 0.0]), B_ctrl=np.array([0.0, 3.0]))
    for s in (0.0, 0.3, 0.8, 1.0):
        a, b = model.schedule(inst.A_ctrl, inst.B_ctrl, s)
        E = np.linalg.eigvalsh(model.hamiltonian_dense(inst, s))
        r = math.hypot(a, b * 0.7)
        np.testing.assert_allclose(E, [-r, r], atol=1e-14)


def test_field_sign_reading_is_a_symmetry():
    """h -> -h is the conjugation by prod_i sx_i, so spectra and P_GS agree."""
    inst = W.ring_instance(3, 7, t_f=50.0, n_grid=41)
    flip = inst.with_(h=-inst.h)
    for s in (0.2, 0.6, 1.0):
        np.testing.assert_allclose(np.linalg.eigvalsh(model.hamiltonian_dense(inst, s)),
                                   np.linalg.eigvalsh(model.hamiltonian_dense(flip, s)), atol=1e-12)
    P1 = ame.split_step(spectrum.table_stream(inst), inst)
    P2 = ame.split_step(spectrum.table_stream(flip), flip)
    np.testing.assert_allclose(P1, P2, atol=1e-11)


# ---------------------------------------------------------------- spectrum --
def test_canonical_basis_at_s1_is_computational():
    inst = W.pm1_all_to_all(5, 3)
    E, V, gs = spectrum.eigen(inst, 1.0, 32, 1e-8)
    assert np.allclose(np.abs(V).max(axis=0), 1.0)
    idx = np.abs(V).argmax(axis=0)
    # ascending energy, ties in ascending basis index
    e = model.hz_diag(inst.h, inst.J)
    order = sorted(range(32), key=lambda x: (e[x], x))
    assert list(idx) == order
    assert np.all(V[idx, np.arange(32)] > 0)


def test_eigen_residual_and_orthonormality():
    inst = W.pm1_all_to_all(6, 11)
    H = model.hamiltonian_dense(inst, 0.37)
    E, V, _ = spectrum.eigen(inst, 0.37, 64, 1e-8)
    assert np.abs(H @ V - V * E).max() < 1e-11
    assert np.abs(V.T @ V - np.eye(64)).max() < 1e-12


def test_sum_of_squared_matrix_elements_is_one():
    """Full spectrum: sum_a <a|sz|b>^2 = <b|sz^2|b> = 1."""
    inst = W.ring_instance(4, 5)
    tabs = spectrum.all_tables(inst, n_grid=11)
    for T in tabs:
        np.testing.assert_allclose((T.z ** 2).sum(axis=1), 1.0, atol=1e-12)


def test_relaxation_rate_closed_form():
    """Sec. V eq. inctunnrate / App. F: lambda_{1->0} = sum_a gamma(w10) |<0|sz_a|1>|^2."""
    inst = W.ring_instance(4, 1001)
    for s in (0.3, 0.55, 0.9):
        H = model.hamiltonian_dense(inst, s)
        E, V = np.linalg.eigh(H)
        w10 = E[1] - E[0]
        lam = sum(model.gamma_ohmic(w10, inst.eta, inst.omega_c, inst.T) *
                  (V[:, 0] @ model.pauli_on(model.SZ, a, 4) @ V[:, 1]) ** 2 for a in range(4))
        Ec, Vc, _ = spectrum.eigen(inst, s, 16, 1e-8)
        _, R, _, _, _, _ = spectrum.grid_tables(inst, Ec, Vc, 1.0)
        np.testing.assert_allclose(R[:, 1, 0].sum(), lam, rtol=1e-12)


def test_rate_matrix_detailed_balance_and_gibbs_null_vector():
    inst = W.ring_instance(4, 1001)
    T = spectrum.all_tables(inst, n_grid=5)[2]
    Wm = ame.rate_matrix(T)
    pi = np.exp(-(T.E - T.E[0]) / inst.T)
    pi /= pi.sum()
    F = Wm * pi[None, :]
    off = ~np.eye(len(pi), dtype=bool)
    np.testing.assert_allclose(F[off], F.T[off], rtol=1e-10, atol=1e-18)
    assert np.abs(Wm.sum(axis=0)).max() < 1e-15
    assert np.abs(Wm @ pi).max() < 1e-15


# ---------------------------------------------------------------- AME --------
@pytest.mark.parametrize("lamb", [False, True])
def test_split_step_map_equals_explicit_liouvillian(lamb):
    """Decoupled population/coherence update = expm of the Lindbladian built from eq. Lindblad2
    (with lamb: plus -i[H_LS, rho], H_LS = sum S(w) A^dag A built from the operators)."""
    inst = W.ring_instance(2, 3, t_f=40.0, lamb_shift=lamb)
    for T in spectrum.all_tables(inst, n_grid=6)[1:4]:
        dt = 3.7
        rng = np.random.default_rng(T.g)
        X = rng.normal(size=(4, 4)) + 1j * rng.normal(size=(4, 4))
        rho = X @ X.conj().T
        rho /= np.trace(rho)
        got = ame.step_map(rho, T, inst, dt)
        want = (sla.expm(ame.liouvillian(T, inst) * dt) @ rho.reshape(-1, order="F")).reshape(4, 4, order="F")
        np.testing.assert_allclose(got, want, atol=1e-13)


def test_split_step_trace_hermitian_psd():
    inst = W.config_small()
    P, rho = ame.split_step(spectrum.table_stream(inst), inst, keep_rho=True)
    assert abs(np.trace(rho) - 1.0) < 1e-12
    assert np.abs(rho - rho.conj().T).max() < 1e-14
    assert np.linalg.eigvalsh(rho).min() > -1e-12
    assert np.all((P >= -1e-12) & (P <= 1 + 1e-12))


def test_two_level_relaxation_closed_form():
    """Fixed H = -A sx: P1(t) = Peq (1 - exp(-kappa t)), kappa = g(2A)+g(-2A), Peq = 1/(1+e^{2 beta A})."""
    A = 0.3
    inst = W.two_level_fixed(A=A, t_f=400.0, n_grid=81, eta=2e-3)
    P0 = ame.split_step(spectrum.table_stream(inst), inst)
    t = np.linspace(0, inst.t_f, inst.n_grid)
    gp = model.gamma_ohmic(2 * A, inst.eta, inst.omega_c, inst.T)
    gm = model.gamma_ohmic(-2 * A, inst.eta, inst.omega_c, inst.T)
    kappa, peq = gp + gm, 1.0 / (1.0 + np.exp(2 * A / inst.T))
    np.testing.assert_allclose(1.0 - P0, peq * (1.0 - np.exp(-kappa * t)), atol=1e-12)


def test_frozen_hamiltonian_relaxes_to_gibbs():
    inst = W.ring_instance(3, 21, t_f=4.0e5, n_grid=41, eta=2e-3,
                           A_ctrl=np.array([1.0, 1.0]), B_ctrl=np.array([1.5, 1.5]))
    tabs = spectrum.all_tables(inst)
    P, rho = ame.split_step(tabs, inst, keep_rho=True)
    E = tabs[-1].E
    pi = np.exp(-(E - E[0]) / inst.T)
    pi /= pi.sum()
    np.testing.assert_allclose(np.real(np.diag(rho)), pi, atol=1e-9)
    assert np.abs(rho - np.diag(np.diag(rho))).max() < 1e-9


def test_split_step_converges_to_continuous_ame():
    """Right-end-point split step is first order in dt: the mid-anneal error halves when M doubles."""
    inst = W.ring_instance(2, 4, t_f=30.0, eta=5e-3)
    B = ame.continuous(inst, np.array([0.5, 1.0]))
    mid, end = [], []
    for M in (241, 481, 961):
        P = ame.split_step(spectrum.table_stream(inst, n_grid=M), inst, n_grid=M)
        mid.append(abs(P[(M - 1) // 2] - B[0]))
        end.append(abs(P[M - 1] - B[1]))
    assert 1.8 < mid[0] / mid[1] < 2.3 and 1.8 < mid[1] / mid[2] < 2.3
    assert end[2] < end[1] < end[0] and mid[2] < 3e-5


def test_continuous_ame_frozen_matches_liouvillian():
    inst = W.ring_instance(2, 9, t_f=25.0, eta=5e-3, A_ctrl=np.array([0.8, 0.8]),
                           B_ctrl=np.array([1.1, 1.1]))
    Pc = ame.continuous(inst, np.array([1.0]), rtol=1e-11, atol=1e-13)
    P = ame.split_step(spectrum.table_stream(inst, n_grid=3), inst, n_grid=3)
    assert abs(Pc[0] - P[-1]) < 1e-8


def test_closed_system_matches_lab_frame_schrodinger():
    """eta = 0 on a diabatic anneal (P_GS ~ 0.74): no jumps, norm conserved, and the
    eigenbasis stepping converges to lab-frame Schrodinger evolution."""
    inst = W.ring_instance(3, 8, t_f=1.0, eta=0.0)
    lab = ame.closed_system_lab(inst, np.array([0.5, 1.0]))
    errs = []
    for M in (201, 801):
        tabs = spectrum.all_tables(inst, n_grid=M)
        res = trajectories.run(tabs, inst, 3, n_grid=M)
        assert res.kind_totals.sum() == 0
        assert np.abs(np.linalg.norm(res.final_state, axis=0) - 1.0).max() < 1e-12
        P = res.pgs_sum / 3
        errs.append(np.abs(P[[(M - 1) // 2, M - 1]] - lab).max())
    assert lab[1] < 0.8 and errs[1] < 1e-6 and errs[1] < errs[0] / 3.0


# ---------------------------------------------------------------- trajectories
def test_crossing_time_matches_brentq():
    rng = np.random.default_rng(0)
    for _ in range(200):
        n = rng.integers(2, 40)
        w = rng.random(n)
        w /= w.sum()
        Gam = rng.random(n) * rng.choice([1e-3, 1.0, 30.0])
        tmax = 5.0
        end = (w * np.exp(-Gam * tmax)).sum()
        r = end + (1 - end) * rng.random()
        tau = trajectories.crossing_time(w, Gam, r, tmax, tmax)
        ref = so.brentq(lambda t: (w * np.exp(-Gam * t)).sum() - r, 0.0, tmax, xtol=1e-16, rtol=1e-15)
        # conditioning of the root: an O(eps) relative error of the norm moves tau by eps g/|g'|
        gref = (w * np.exp(-Gam * ref)).sum()
        slope = (Gam * w * np.exp(-Gam * ref)).sum()
        assert abs(tau - ref) <= 1e-14 * tmax + 8e-16 * gref / slope


def test_pick_is_the_inverse_cdf():
    w = np.array([0.0, 2.0, 0.0, 1.0, 1.0])
    assert trajectories.pick(w, 0.0) == 1
    assert trajectories.pick(w, 0.49) == 1
    assert trajectories.pick(w, 0.51) == 3
    assert trajectories.pick(w, 0.76) == 4
    assert trajectories.pick(w, 1.0 - 1e-17) == 4


def test_waiting_time_is_exponential():
    """App. C: from an eigenstate with frozen H the first jump time is Exp(Gamma_b)."""
    inst = W.ring_instance(3, 21, t_f=15.0, n_grid=21, eta=5e-3,
                           A_ctrl=np.array([1.0, 1.0]), B_ctrl=np.array([1.5, 1.5]))
    tabs = spectrum.all_tables(inst)
    res = trajectories.run(tabs, inst, 2000)
    first = np.array([j[0][0] if j else np.inf for j in res.jumps])
    rate = tabs[0].Gamma[0]
    # censor at t_f: compare the survival function on the observed window
    cdf = lambda t: 1.0 - np.exp(-rate * np.minimum(t, inst.t_f))
    obs = first[np.isfinite(first)]
    frac_censored = np.mean(~np.isfinite(first))
    assert abs(frac_censored - np.exp(-rate * inst.t_f)) < 4 * math.sqrt(0.25 / 2000)
    ks = st.kstest(obs, lambda t: cdf(t) / cdf(inst.t_f))
    assert ks.pvalue > 1e-3


def test_frozen_trajectories_are_a_classical_chain():
    """App. E: eigenstate trajectories change only by jumps, a Markov chain with rates W."""
    inst = W.ring_instance(3, 21, t_f=40.0, n_grid=31, eta=5e-3,
                           A_ctrl=np.array([1.0, 1.0]), B_ctrl=np.array([1.5, 1.5]))
    tabs = spectrum.all_tables(inst)
    K = 1500
    res = trajectories.run(tabs, inst, K)
    T = tabs[0]
    Wm = ame.rate_matrix(T)
    n = len(T.E)
    g0 = model.gamma_ohmic(0.0, inst.eta, inst.omega_c, inst.T)
    deph = g0 * (T.zdiag ** 2).sum(axis=0)
    # Gillespie simulation of the same chain with an unrelated RNG
    rng = np.random.default_rng(12345)
    cnt_trans, cnt_deph = [], []
    for _ in range(K):
        b, t, ntr, nde = 0, 0.0, 0, 0
        while True:
            out = -Wm[b, b]
            tot = out + deph[b]
            t += rng.exponential(1.0 / tot)
            if t > inst.t_f:
                break
            if rng.random() < deph[b] / tot:
                nde += 1
            else:
                p = Wm[:, b].copy()
                p[b] = 0
                b = rng.choice(n, p=p / p.sum())
                ntr += 1
        cnt_trans.append(ntr)
        cnt_deph.append(nde)
    got_tr = np.array([sum(1 for j in js if j[3] != j[4]) for js in res.jumps])
    got_de = np.array([sum(1 for j in js if j[3] == j[4]) for js in res.jumps])
    for a, b in ((got_tr, np.array(cnt_trans)), (got_de, np.array(cnt_deph))):
        se = math.sqrt(a.var() / K + b.var() / K)
        assert abs(a.mean() - b.mean()) < 4 * se + 1e-9
    # populations stay pure eigenstates between jumps: P_GS is 0 or 1 per trajectory
    assert np.all(np.abs(res.pgs_sum - res.pgs_sumsq) < 1e-9 * K)


def test_trajectory_average_matches_split_step_ame():
    """Averaging trajectories recovers the master equation (Sec. IV, App. B): 4-qubit workload."""
    inst = W.config_small()
    tabs = spectrum.all_tables(inst)
    P = ame.split_step(tabs, inst)
    K = 1000
    res = trajectories.run(tabs, inst, K, record=False)
    m, se = trajectories.mean_and_stderr(res.pgs_sum, res.pgs_sumsq, K)
    sigma = np.maximum(se, np.sqrt(np.clip(P * (1 - P), 0, None) / K))
    assert np.all(np.abs(m - P) <= 3 * sigma + 1e-4)


def test_trajectory_average_matches_ame_nonadiabatic():
    """Fast, strongly coupled anneal: jumps act on superpositions (source choice and
    the omega = 0 operator matter), the average still equals the split-step AME."""
    inst = W.ring_instance(3, 8, t_f=1.5, eta=0.1, n_grid=101)
    tabs = spectrum.all_tables(inst)
    P = ame.split_step(tabs, inst)
    K = 3000
    res = trajectories.run(tabs, inst, K, record=False)
    m, se = trajectories.mean_and_stderr(res.pgs_sum, res.pgs_sumsq, K)
    sigma = np.maximum(se, np.sqrt(np.clip(P * (1 - P), 0, None) / K))
    assert P.min() < 0.9 and res.kind_totals.sum() > K
    assert np.all(np.abs(m - P) <= 3 * sigma + 1e-4)


def test_jump_counts_match_ame_rates_after_quench():
    """Sec. III: E[dN_i] = <A_i^dag A_i> dt.  A diabatic ramp into a frozen Hamiltonian at low
    temperature leaves superpositions of levels whose decay rates differ by 10x or more, so the
    source level must be drawn with weight q_b Gamma_b (App. B, eq. Pi(t)).  Jump counts by
    kind and the ground-state population both match the exact AME expectations."""
    A = np.array([3.0] + [0.8] * 10)
    B = np.array([0.0] + [1.2] * 10)
    inst = W.ring_instance(3, 8, t_f=20.0, eta=0.1, n_grid=201, T=0.05, A_ctrl=A, B_ctrl=B)
    tabs = spectrum.all_tables(inst)
    P = ame.split_step(tabs, inst)
    expect = ame.expected_jumps(tabs, inst)
    K = 3000
    res = trajectories.run(tabs, inst, K)
    m, se = trajectories.mean_and_stderr(res.pgs_sum, res.pgs_sumsq, K)
    sigma = np.maximum(se, np.sqrt(np.clip(P * (1 - P), 0, None) / K))
    assert np.all(np.abs(m - P) <= 3 * sigma + 1e-4)
    counts = np.zeros((K, 3))
    for j, js in enumerate(res.jumps):
        for rec in js:
            counts[j, rec[5]] += 1
    assert expect[0] > 0.1 and tabs[-1].Gamma.max() > 10 * tabs[-1].Gamma.min()
    for kind in range(3):
        se_k = max(counts[:, kind].std() / math.sqrt(K), math.sqrt(expect[kind] / K))
        assert abs(counts[:, kind].mean() - expect[kind]) < 4 * se_k


def test_standard_error_formula():
    """Sec. VI eq. stderror evaluated from running sums equals the two-pass definition."""
    x = np.random.default_rng(3).random(501)
    R = len(x)
    M = x.mean()
    ref = np.sqrt(((x - M) ** 2).sum() / (R * (R - 1)))
    m, se = trajectories.mean_and_stderr(x.sum(), (x * x).sum(), R)
    assert abs(m - M) < 1e-15 and abs(se - ref) < 1e-13


def test_a2a8_seed_is_first_with_unique_final_ground_state():
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "a2a8_seed_scan.json")) as f:
        scan = json.load(f)
    assert W.A2A8_SEED == scan["chosen"]
    inst = W.config_a2a8(10)
    e = np.sort(model.hz_diag(inst.h, inst.J))
    assert e[1] - e[0] > 0.5


def test_sparse_eigensolver_finds_every_sector_and_multiplicity():
    """The Lanczos path used above 4096 states against dense eigh on a 10-qubit two-cluster
    gadget (qubit-permutation symmetry, degenerate levels at every s): same lowest 40
    energies with multiplicities, and the same retained subspace."""
    inst = W.gadget_instance(5, n_levels=24, n_grid=50)
    for s in (0.3, 1.0):
        Ed, Vd, gd = spectrum.eigen(inst, s, 40, 1e-8, method="dense")
        Es, Vs, gsz = spectrum.eigen(inst, s, 40, 1e-8, method="sparse")
        np.testing.assert_allclose(Es, Ed, atol=1e-9 * np.abs(Ed).max())
        assert gd == gsz
        # compare subspaces spanned by complete clusters within the 24 lowest levels
        cut = 24
        while cut > 0 and abs(Ed[cut] - Ed[cut - 1]) < 1e-6:
            cut -= 1
        Pd = Vd[:, :cut] @ Vd[:, :cut].T
        Ps = Vs[:, :cut] @ Vs[:, :cut].T
        assert np.abs(Pd - Ps).max() < 1e-7


def test_polar_completion_is_orthogonal_and_agrees_on_kept_directions():
    """Polar factor with lost directions: for M = U diag(s) W^T with one singular value
    below the loss threshold, the completed factor is orthogonal, maps every kept right
    singular vector w_a to u_a exactly as the polar factor does, and maps the lost one
    into the orthogonal complement of the kept u_a; with nothing lost it is U W^T."""
    rng = np.random.default_rng(5)
    n = 6
    U, _ = np.linalg.qr(rng.standard_normal((n, n)))
    Wm, _ = np.linalg.qr(rng.standard_normal((n, n)))
    s = np.array([1.0, 0.9, 0.7, 0.5, 0.2, 1e-9])
    M = U @ np.diag(s) @ Wm.T
    P, S = spectrum.polar(M)
    np.testing.assert_allclose(P.T @ P, np.eye(n), atol=1e-12)
    for a in range(n - 1):
        np.testing.assert_allclose(P @ Wm[:, a], U[:, a], atol=1e-9)
    lost = P @ Wm[:, n - 1]
    assert np.abs(U[:, : n - 1].T @ lost).max() < 1e-9
    assert abs(np.linalg.norm(lost) - 1.0) < 1e-12
    s2 = np.array([1.0, 0.9, 0.7, 0.5, 0.2, 0.1])
    P2, _ = spectrum.polar(U @ np.diag(s2) @ Wm.T)
    np.testing.assert_allclose(P2, U @ Wm.T, atol=1e-12)
    # the completion depends only on the lost and free subspaces, not on the signs the
    # SVD happens to give their vectors: -M has the same subspaces, so the same completion
    P3, _ = spectrum.polar(-M)
    np.testing.assert_allclose(P3 @ Wm[:, n - 1], lost, atol=1e-9)


def test_gradient_oracle_two_level_closed_form():
    """Central differences of the final ground-state population against the closed form
    of a frozen two-level relaxation: P = 1 - Peq (1 - e^{-kappa t}), kappa = g(2A) + g(-2A)
    proportional to eta, Peq = 1 / (1 + e^{2A/T}).  d/deta, the sum over the A controls
    (a uniform shift of A), and d/dB = 0 (no field or coupling terms)."""
    from oracle import gradient
    A, t = 0.3, 150.0
    inst = W.two_level_fixed(A=A, t_f=t, n_grid=41, eta=2e-3)
    g = gradient.fd_gradient(inst, h=1e-5)

    def closed(A_, eta_):
        gp = model.gamma_ohmic(2 * A_, eta_, inst.omega_c, inst.T)
        gm = model.gamma_ohmic(-2 * A_, eta_, inst.omega_c, inst.T)
        peq = 1.0 / (1.0 + np.exp(2 * A_ / inst.T))
        return 1.0 - peq * (1.0 - np.exp(-(gp + gm) * t))

    gp = model.gamma_ohmic(2 * A, inst.eta, inst.omega_c, inst.T)
    gm = model.gamma_ohmic(-2 * A, inst.eta, inst.omega_c, inst.T)
    kappa, peq = gp + gm, 1.0 / (1.0 + np.exp(2 * A / inst.T))
    d_eta = -peq * t * np.exp(-kappa * t) * kappa / inst.eta        # kappa is linear in eta
    assert abs(g["deta"] - d_eta) <= 1e-6 * abs(d_eta)
    hA = 1e-6
    d_A = (closed(A + hA, inst.eta) - closed(A - hA, inst.eta)) / (2 * hA)
    assert abs(g["dA"].sum() - d_A) <= 1e-5 * abs(d_A)
    np.testing.assert_allclose(g["dB"], 0.0, atol=1e-12)


def _gradient_instance():
    """3-qubit ring, fast strongly coupled anneal (jumps act on superpositions), three
    control points per schedule."""
    A, B = W.linear_schedule(3)
    return W.ring_instance(3, 8, t_f=1.5, eta=0.1, n_grid=101, A_ctrl=A, B_ctrl=B)


def test_path_replay_reproduces_the_trajectory():
    """Rebuilding each recorded path from its jump times and channels (Sec. III eq. jump,
    App. B) lands on the trajectory's own final state, up to normalisation and a global
    phase, and gives back its final ground-cluster population."""
    from oracle import gradient
    inst = _gradient_instance()
    tabs = spectrum.all_tables(inst)
    res = trajectories.run(tabs, inst, 300, record=True)
    logW, logN, C = gradient.replay_log_weight(tabs, inst, res.jumps)
    cf = res.final_state
    ov = np.abs(np.sum(np.conj(cf) * C, axis=0)) / (np.linalg.norm(cf, axis=0) * np.linalg.norm(C, axis=0))
    np.testing.assert_allclose(ov, 1.0, atol=1e-12)
    gs = tabs[-1].gs
    p = (np.abs(cf[:gs]) ** 2).sum(axis=0) / (np.abs(cf) ** 2).sum(axis=0)
    np.testing.assert_allclose(np.exp(logW - logN), p, atol=1e-13)
    assert res.kind_totals.sum() > 300


def test_trajectory_gradient_estimates_are_unbiased():
    """The mean of the per-trajectory estimates equals the central difference of the
    split-step AME (the exact mean of the process) for every control point and eta,
    within three standard errors."""
    from oracle import gradient
    inst = _gradient_instance()
    K = 2000
    r = gradient.trajectory_gradients(inst, K)
    fd = gradient.fd_gradient(inst)
    ref = np.concatenate([fd["dA"], fd["dB"], [fd["deta"]]])
    m = r["g"].mean(axis=0)
    se = r["g"].std(axis=0, ddof=1) / np.sqrt(K)
    assert np.all(np.abs(m - ref) <= 3.0 * se + 1e-4), (m, ref, se)
    # the estimates are informative: the largest components are resolved well beyond noise
    assert np.sum(np.abs(ref) > 5.0 * se) >= 3
    # the path-density score has mean zero (the total probability does not depend on theta)
    s = r["score"]
    assert np.all(np.abs(s.mean(axis=0)) <= 3.0 * s.std(axis=0, ddof=1) / np.sqrt(K))
    assert np.all(s.std(axis=0) > 0)


def test_lamb_shift_function_zero_temperature_closed_form():
    """The principal-value integral of the Ohmic gamma against the T = 0 closed form
    eta (-wc + w e^{-w/wc} Ei(w/wc)) at a temperature far below every |w| tested."""
    wc = 8 * np.pi
    for w in (-80.0, -20.0, -3.0, -0.5, 0.5, 3.0, 20.0, 80.0):
        got = model.lamb_S(w, 1e-4, wc, 1e-3)
        want = float(model.lamb_S_zero_temperature(w, 1e-4, wc))
        assert abs(got - want) <= 1e-6 * abs(want), (w, got, want)


def test_lamb_shift_function_at_zero_frequency():
    """S(0) = -(1/2pi) int gamma(w)/w dw = -eta wc at every temperature: the Bose factors
    of +w and -w add to one."""
    for T in (0.05, 1.571044, 7.0):
        assert abs(model.lamb_S(0.0, 2e-4, 5.0, T) + 2e-4 * 5.0) <= 1e-12


def test_lamb_shift_leaves_frozen_populations_alone():
    """H_LS commutes with H_S (it is diagonal in the eigenbasis): for a frozen Hamiltonian
    started in its ground state the split-step AME state does not change at all."""
    inst = W.ring_instance(2, 3, t_f=40.0, n_grid=6, A_ctrl=np.array([1.0, 1.0]), B_ctrl=np.array([0.7, 0.7]),
                           eta=1e-2)
    P0, r0 = ame.split_step(spectrum.all_tables(inst), inst, keep_rho=True)
    P1, r1 = ame.split_step(spectrum.all_tables(inst.with_(lamb_shift=True)), inst.with_(lamb_shift=True),
                            keep_rho=True)
    np.testing.assert_allclose(np.diag(r1).real, np.diag(r0).real, atol=1e-14)
    np.testing.assert_allclose(P1, P0, atol=1e-14)


@pytest.mark.parametrize("rho", [0.0, 0.6, -0.35])
def test_correlated_baths_split_step_equals_double_sum(rho):
    """Correlated baths gamma_ab(w) = C_ab gamma(w): the split-step map built from the
    Cholesky channels equals expm of eq. ME2-L written as the double sum over qubits with
    the per-qubit operators (no factorisation of C); rho = 0 is the independent case."""
    C = np.array([[1.0, rho], [rho, 1.0]])
    inst = W.ring_instance(2, 3, t_f=40.0, bath_corr=C, eta=3e-3)
    for T in spectrum.all_tables(inst, n_grid=6, keep_V=True)[1:4]:
        zq = [T.V.T @ (model.sz_diag(q, 2)[:, None] * T.V) for q in range(2)]
        dt = 3.7
        rng = np.random.default_rng(T.g)
        X = rng.normal(size=(4, 4)) + 1j * rng.normal(size=(4, 4))
        r0 = X @ X.conj().T
        r0 /= np.trace(r0)
        got = ame.step_map(r0, T, inst, dt)
        Ls = ame.liouvillian_correlated(T, inst, zq)
        want = (sla.expm(Ls * dt) @ r0.reshape(-1, order="F")).reshape(4, 4, order="F")
        np.testing.assert_allclose(got, want, atol=1e-13)
    if rho == 0.0:
        base = spectrum.all_tables(inst.with_(bath_corr=None), n_grid=6)
        for T, B in zip(spectrum.all_tables(inst, n_grid=6), base):
            np.testing.assert_array_equal(T.R, B.R)


def test_psd_factor_reproduces_semidefinite_matrices():
    """C = F F^T for positive definite and rank-deficient C; a rank-r C gives r channels,
    and a positive definite C gives the Cholesky factor."""
    rng = np.random.default_rng(3)
    X = rng.normal(size=(5, 5))
    for C, r in ((X @ X.T + 0.1 * np.eye(5), 5), (0.7 * np.ones((5, 5)), 1), (X[:, :2] @ X[:, :2].T, 2)):
        F = model.psd_factor(C)
        assert F.shape == (5, r)
        np.testing.assert_allclose(F @ F.T, C, atol=1e-12 * np.abs(C).max())
    C = X @ X.T + 0.1 * np.eye(5)
    np.testing.assert_allclose(model.psd_factor(C), np.linalg.cholesky(C), rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("rho,xi", [(0.5, 0.5), (1.2, -0.3)])
def test_frequency_dependent_bath_split_step_equals_double_sum(rho, xi):
    """gamma_ab(w) = sum_m C_m[a, b] gamma(w; omega_c,m) with non-commuting C_m (local baths
    correlated as xi^|a-b| plus a rank-one shared bath with a lower cutoff): gamma(w) has
    w-dependent eigenvectors, and the split-step map built from the per-term channels
    equals expm of eq. ME2-L written as the double sum over qubits with gamma_ab(w) taken
    from its definition."""
    terms = W.two_term_bath(3, rho=rho, xi=xi)
    inst = W.ring_instance(3, 5, t_f=40.0, eta=3e-3, bath_terms=terms)
    G1, G2 = model.gamma_matrix(inst, 1.0), model.gamma_matrix(inst, 20.0)
    assert np.abs(G1 @ G2 - G2 @ G1).max() > 1e-2 * np.abs(G1).max() * np.abs(G2).max()
    tabs = spectrum.all_tables(inst, n_grid=6, keep_V=True)
    assert tabs[1].R.shape[0] == 4              # 3 local channels + 1 shared
    for T in tabs[1:4]:
        zq = [T.V.T @ (model.sz_diag(q, 3)[:, None] * T.V) for q in range(3)]
        dt = 3.7
        rng = np.random.default_rng(T.g)
        X = rng.normal(size=(8, 8)) + 1j * rng.normal(size=(8, 8))
        r0 = X @ X.conj().T
        r0 /= np.trace(r0)
        got = ame.step_map(r0, T, inst, dt)
        Ls = ame.liouvillian_correlated(T, inst, zq)
        want = (sla.expm(Ls * dt) @ r0.reshape(-1, order="F")).reshape(8, 8, order="F")
        np.testing.assert_allclose(got, want, atol=1e-13)


def test_lamb_shift_of_bath_terms_equals_double_sum():
    """Lamb shift with frequency-dependent correlations: the shift of each level from the
    per-term channels (each S with its term's cutoff) equals the double sum over qubits
    sum_ab S_ab(w) <a|sz_a|b><a|sz_b|b> with S_ab(w) = sum_m C_m[a, b] S(w; omega_c,m),
    built from per-qubit operators (no factorisation); S(0) = -eta omega_c,m per term."""
    terms = W.two_term_bath(2, rho=0.8)
    inst = W.ring_instance(2, 3, t_f=40.0, eta=3e-3, bath_terms=terms, lamb_shift=True)
    T = spectrum.all_tables(inst, n_grid=4, keep_V=True)[2]
    zq = [T.V.T @ (model.sz_diag(q, 2)[:, None] * T.V) for q in range(2)]
    n = len(T.E)

    def S_ab(w):
        return sum(np.asarray(C) * model.lamb_S(w, inst.eta, wc, inst.T) for C, wc in terms)

    want = np.zeros(n)
    for b in range(n):
        for a in range(n):
            G = S_ab(0.0 if a == b else float(T.E[b] - T.E[a]))
            v = np.array([zq[q][a, b] for q in range(2)])
            want[b] += v @ G @ v
    np.testing.assert_allclose(T.shift, want, rtol=1e-10, atol=1e-14)
    for C, wc in terms:
        np.testing.assert_allclose(model.lamb_S(0.0, inst.eta, wc, inst.T), -inst.eta * wc, rtol=1e-9)


def test_single_bath_term_equals_constant_correlation():
    """One term (C, omega_c of the bath) is the constant-correlation model."""
    C = np.array([[1.0, 0.4, 0.1], [0.4, 1.0, 0.4], [0.1, 0.4, 1.0]])
    inst = W.ring_instance(3, 5, t_f=40.0, eta=3e-3)
    a = spectrum.all_tables(inst.with_(bath_corr=C), n_grid=5)
    b = spectrum.all_tables(inst.with_(bath_terms=((C, inst.omega_c),)), n_grid=5)
    for Ta, Tb in zip(a[1:], b[1:]):
        np.testing.assert_allclose(Tb.R, Ta.R, rtol=1e-12, atol=1e-18)
        np.testing.assert_allclose(Tb.Gamma, Ta.Gamma, rtol=1e-12)


def test_trajectory_average_matches_ame_frequency_dependent_bath():
    """Trajectories with the per-term channels average to the split-step AME."""
    inst = W.ring_instance(3, 8, t_f=1.5, eta=0.1, n_grid=61, bath_terms=W.two_term_bath(3, rho=0.8))
    tabs = spectrum.all_tables(inst)
    P = ame.split_step(tabs, inst)
    K = 2000
    res = trajectories.run(tabs, inst, K, record=False)
    m, se = trajectories.mean_and_stderr(res.pgs_sum, res.pgs_sumsq, K)
    sigma = np.maximum(se, np.sqrt(np.clip(P * (1 - P), 0, None) / K))
    assert P.min() < 0.9 and res.kind_totals.sum() > K
    assert np.all(np.abs(m - P) <= 3 * sigma + 1e-4)


@pytest.mark.parametrize("cz,cx", [(0.0, 1.0), (0.6, 0.8)])
def test_two_level_sx_coupling_closed_form(cz, cx):
    """Fixed H = -A sx coupled through cz sz + cx sx: the sx part commutes with H, so it
    only dephases (omega = 0 operator sqrt(gamma(0)) cx diag(1, -1) in the eigenbasis,
    coherence decay 2 cx^2 gamma(0)), and the sz part relaxes the populations at
    kappa = cz^2 (gamma(2A) + gamma(-2A)) towards Peq = 1/(1+e^{2 beta A})."""
    A = 0.3
    inst = W.two_level_fixed(A=A, t_f=400.0, n_grid=81, eta=2e-3, coupling=([[cz]], [[cx]], None))
    P0 = ame.split_step(spectrum.table_stream(inst), inst)
    t = np.linspace(0, inst.t_f, inst.n_grid)
    gp = model.gamma_ohmic(2 * A, inst.eta, inst.omega_c, inst.T)
    gm = model.gamma_ohmic(-2 * A, inst.eta, inst.omega_c, inst.T)
    g0 = float(model.gamma_ohmic(0.0, inst.eta, inst.omega_c, inst.T))
    kappa, peq = cz ** 2 * (gp + gm), 1.0 / (1.0 + np.exp(2 * A / inst.T))
    np.testing.assert_allclose(1.0 - P0, peq * (1.0 - np.exp(-kappa * t)), atol=1e-12)
    T = spectrum.all_tables(inst)[3]
    r0 = np.array([[0.7, 0.3 - 0.2j], [0.3 + 0.2j, 0.3]])
    dt = 5.0
    got = ame.step_map(r0, T, inst, dt)
    if cz == 0.0:   # populations frozen, coherence: phase and exp(-2 cx^2 gamma(0) dt)
        np.testing.assert_allclose(np.diag(got).real, np.diag(r0).real, atol=1e-15)
        want = r0[0, 1] * np.exp(-1j * (T.E[0] - T.E[1]) * dt) * np.exp(-2.0 * cx ** 2 * g0 * dt)
        np.testing.assert_allclose(got[0, 1], want, rtol=1e-13)


def test_mixed_coupling_split_step_equals_lindblad_form():
    """Channels with operators sum_a (cz sz_a + cx sx_a): the split-step map built from the
    tables (sx applied as a row permutation) equals expm of the Lindblad form whose
    operators come from dense Kronecker-product Pauli matrices in the eigenbasis."""
    cz = np.array([[0.7, 0.0], [0.0, 0.0], [-0.4, 1.0]])
    cx = np.array([[0.0, 0.5], [1.0, 0.0], [0.3, 0.0]])
    wc = np.array([8.0 * math.pi, 4.0, 8.0 * math.pi])
    inst = W.ring_instance(2, 3, t_f=40.0, eta=3e-3, coupling=(cz, cx, wc))
    tabs = spectrum.all_tables(inst, n_grid=6, keep_V=True)
    assert tabs[1].R.shape[0] == 3
    for T in tabs[1:4]:
        ops = [sum(cz[k, a] * model.pauli_on(model.SZ, a, 2) + cx[k, a] * model.pauli_on(model.SX, a, 2)
                   for a in range(2)) for k in range(3)]
        zk = np.stack([T.V.T @ O @ T.V for O in ops])
        T2 = dataclasses.replace(T, z=zk)
        dt = 3.7
        rng = np.random.default_rng(T.g)
        X = rng.normal(size=(4, 4)) + 1j * rng.normal(size=(4, 4))
        r0 = X @ X.conj().T
        r0 /= np.trace(r0)
        got = ame.step_map(r0, T, inst, dt)
        Ls = ame.liouvillian(T2, inst)
        want = (sla.expm(Ls * dt) @ r0.reshape(-1, order="F")).reshape(4, 4, order="F")
        np.testing.assert_allclose(got, want, atol=1e-13)


def test_step_bound_and_bound_grid_closed_form():
    """One qubit, H = -A(s) sx with A = a0 (1 + s) and a vanishing bath: |H_eff| = A,
    |dH/dt| = a0 / t_f, so the App. B bound is min(t_f (1 + s), 1 / A) = 1 / (a0 (1 + s));
    equidistributing its inverse gives s_g + s_g^2 / 2 = 3 g / (2 (M - 1)),
    s_g = -1 + sqrt(1 + 3 g / (M - 1))."""
    a0, M = 1.0, 11
    inst = W.two_level_fixed(A=a0, t_f=100.0, n_grid=M, eta=1e-10).with_(A_ctrl=np.array([a0, 2 * a0]))
    sp = np.linspace(0.0, 1.0, 7)
    np.testing.assert_allclose(spectrum.step_bound(inst, sp), 1.0 / (a0 * (1.0 + sp)), rtol=1e-12)
    g = spectrum.bound_grid(inst, M, n_probe=2001)
    np.testing.assert_allclose(g, -1.0 + np.sqrt(1.0 + 3.0 * np.arange(M) / (M - 1)), atol=1e-7)


def test_bound_grid_of_a_frozen_hamiltonian_is_equidistant():
    inst = W.ring_instance(3, 21, t_f=50.0, n_grid=9, eta=2e-3, A_ctrl=np.array([1.0, 1.0]),
                           B_ctrl=np.array([1.5, 1.5]))
    np.testing.assert_allclose(spectrum.bound_grid(inst, 9, n_probe=101), np.linspace(0.0, 1.0, 9), atol=1e-12)


def test_explicit_equidistant_grid_matches_the_default():
    inst = W.ring_instance(3, 8, t_f=1.5, eta=0.1, n_grid=21)
    a = spectrum.all_tables(inst)
    b = spectrum.all_tables(inst.with_(s_grid=np.linspace(0.0, 1.0, 21)))
    for Ta, Tb in zip(a, b):
        np.testing.assert_allclose(Tb.R, Ta.R, rtol=1e-11, atol=1e-13 * np.abs(Ta.R).max())
        np.testing.assert_allclose(Tb.d, Ta.d, rtol=1e-11)
        assert abs(Tb.t0 - Ta.t0) <= 1e-14 and abs(Tb.dt - Ta.dt) <= 1e-14


def test_trajectory_average_matches_ame_on_the_bound_grid():
    """Exact-mean parity does not depend on the grid: trajectories on the App. B grid
    (steps of different lengths) average to the split-step AME on that grid."""
    inst = W.ring_instance(3, 8, t_f=1.5, eta=0.1, n_grid=61)
    sg = spectrum.bound_grid(inst, 61, n_probe=121)
    steps = np.diff(sg)
    assert steps.max() > 1.5 * steps.min()
    inst = inst.with_(s_grid=sg)
    tabs = spectrum.all_tables(inst)
    P = ame.split_step(tabs, inst)
    K = 2000
    res = trajectories.run(tabs, inst, K, record=False)
    m, se = trajectories.mean_and_stderr(res.pgs_sum, res.pgs_sumsq, K)
    sigma = np.maximum(se, np.sqrt(np.clip(P * (1 - P), 0, None) / K))
    assert np.all(np.abs(m - P) <= 3 * sigma + 1e-4)


def test_split_step_is_second_order_on_a_non_uniform_grid():
    """On points of unequal spacing the split step still approaches the continuous AME
    (the lab-frame route, independent of the eigenbasis tables) at second order: the
    factor of each grid point covers half of each neighbouring step, so every step is
    split symmetrically around its basis change.  Halving the spacing of a grid that is
    four times denser mid-anneal must cut the error by about 4 (by about 2 if each point's
    factor covered only the step before it)."""
    inst = W.ring_instance(3, 8, t_f=1.5, eta=0.1)
    ref = ame.continuous(inst, [1.0])[-1]
    errs = []
    for M in (41, 81, 161):
        sp = np.linspace(0.0, 1.0, 401)
        rho = 1.0 + 3.0 * np.exp(-((sp - 0.5) / 0.15) ** 2)
        F = np.concatenate([[0.0], np.cumsum(0.5 * (rho[1:] + rho[:-1]) * np.diff(sp))])
        sg = np.interp(np.linspace(0.0, F[-1], M), F, sp)
        sg[0], sg[-1] = 0.0, 1.0
        grid = inst.with_(n_grid=M, s_grid=sg)
        tabs = spectrum.all_tables(grid)
        assert abs(sum(T.dt for T in tabs) - inst.t_f) < 1e-12 * inst.t_f
        errs.append(abs(ame.split_step(tabs, grid)[-1] - ref))
    assert errs[0] / errs[1] > 3.0 and errs[1] / errs[2] > 3.0, errs


def test_fixed_step_two_level_follows_the_discrete_chain():
    """Fixed-step unraveling (App. B): a frozen two-level system stays in eigenstates, and
    per sub-step h it jumps 0 -> 1 with probability h W10 and 1 -> 0 with h W01, so its
    mean follows the discrete chain p <- p (1 - h W10) + (1 - p) h W01, not the AME's
    exponential relaxation (which the waiting-time procedure reproduces)."""
    inst = W.two_level_fixed(A=0.3, t_f=20.0, n_grid=11, eta=1e-2)
    tabs = spectrum.all_tables(inst)
    S, K = 2, 20000
    res = trajectories.run_fixed_step(tabs, inst, K, S, record=False)
    T = tabs[0]
    W10, W01 = T.R[:, 0, 1].sum(), T.R[:, 1, 0].sum()
    h = inst.t_f / (inst.n_grid - 1) / S
    p, chain = 1.0, [1.0]
    for _ in range(1, inst.n_grid):
        for _ in range(S):
            p = p * (1 - h * W10) + (1 - p) * h * W01
        chain.append(p)
    chain = np.array(chain)
    m, se = trajectories.mean_and_stderr(res.pgs_sum, res.pgs_sumsq, K)
    assert np.all(np.abs(m - chain)[1:] <= 3 * se[1:])
    P = ame.split_step(tabs, inst)
    assert np.max(np.abs(m - P)[1:] / se[1:]) > 4


def test_fixed_step_closed_system_is_the_no_jump_evolution():
    """eta = 0: no jumps, and the fixed-step state equals the waiting-time run's."""
    inst = W.ring_instance(3, 77, t_f=30.0, eta=0.0, n_grid=60)
    tabs = spectrum.all_tables(inst)
    a = trajectories.run_fixed_step(tabs, inst, 3, 5)
    b = trajectories.run(tabs, inst, 3)
    assert a.kind_totals.sum() == 0
    np.testing.assert_allclose(a.final_state, b.final_state, atol=1e-12)


def test_stored_discretisation_values_agree_with_the_stored_ame():
    """The discretisation record's workload-grid values are the same split-step AME as the
    stored references of the bench (two runs of the oracle, bit for bit), and finer grids
    move the 4-qubit value towards the continuous AME."""
    import json
    import os
    here = os.path.join(os.path.dirname(__file__), "golden")
    d = {c["instance"]: c for c in json.load(open(os.path.join(here, "discretisation.json")))["cases"]}
    a2a8 = json.load(open(os.path.join(here, "a2a8_ame_pgs.json")))
    small = json.load(open(os.path.join(here, "small_ame_pgs.json")))
    assert d[a2a8["instance"]]["pgs"][str(a2a8["n_grid"])] == a2a8["pgs"][-1]
    assert d[small["instance"]]["pgs"][str(small["n_grid"])] == small["pgs"][-1]
    r = d[small["instance"]]
    errs = [abs(r["pgs"][k] - r["continuous"]) for k in sorted(r["pgs"], key=int)]
    assert errs[0] > errs[1] > errs[2]


def test_stored_batched_reference_is_the_oracles():
    """The stored AME reference of the batched workload (tests/golden/batched_ame_pgs.json,
    written by make_golden.py --batched) for its smallest instance (6 qubits, 16 levels,
    1000 grid points) is what the oracle's split-step AME gives now."""
    import json
    import os
    import workloads
    ref = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "batched_ame_pgs.json")))
    row = next(r for r in ref["instances"] if r["name"].startswith("batch2-"))
    inst = workloads.config_batched()[row["index"]]
    assert inst.name == row["name"] and inst.n_grid == row["n_grid"]
    P = ame.split_step(spectrum.table_stream(inst), inst)
    np.testing.assert_allclose(P[np.array(row["grid_points"])], row["pgs"], rtol=1e-10, atol=1e-12)
