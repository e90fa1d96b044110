"""Pins of the CPU oracle against facts that do not come from the oracle itself:
closed forms, reductions to textbook systems, invariants, brute force on tiny inputs and
published generator outputs.  Each test names the part of the oracle a plausible mistake
(dropped term, wrong sign, swapped bit order, wrong midpoint) would break.
"""
import math
import os

import numpy as np
import pytest
import scipy.linalg

from oracle import evolve, model, observables
from paper_2510_09813_amd import workloads as wl

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
C6 = wl.C6_RB


def single_atom_closed_form(omega, delta, phi, t):
    """Rabi oscillation of one driven two-level atom from |0>:
    c0 = e^{i d t/2} [cos(W t/2) - i (d/W) sin(W t/2)],
    c1 = -i e^{i d t/2} (O/W) e^{-i phi} sin(W t/2),  W = sqrt(O^2 + d^2)."""
    w = math.hypot(omega, delta)
    ph = np.exp(0.5j * delta * t)
    c0 = ph * (math.cos(0.5 * w * t) - 1j * (delta / w) * math.sin(0.5 * w * t))
    c1 = -1j * ph * (omega / w) * np.exp(-1j * phi) * math.sin(0.5 * w * t)
    return np.array([c0, c1])


def run(xyz, omega, delta, phi, t_ns, dt_ns, method, c6=C6, psi0=None, **kw):
    return evolve.evolve(xyz, c6, omega, delta, phi, t_ns, dt_ns, psi0=psi0, method=method, **kw)


# ------------------------------------------------------------------ closed forms
@pytest.mark.parametrize("method", ["dense", "lanczos"])
def test_single_atom_rabi_closed_form(method):
    """Pins: sign of delta, sign of phi, the 1/2 of Omega/2, time units, the stepper."""
    om, de, ph, t_ns = 2 * np.pi * 1.3, 2 * np.pi * 0.7, 0.4, 1000
    psi = run(wl.chain(1, 5.0), wl.constant(om, t_ns), wl.constant(de, t_ns),
              wl.constant(ph, t_ns), t_ns, 10, method)
    ref = single_atom_closed_form(om, de, ph, t_ns * 1e-3)
    np.testing.assert_allclose(psi, ref, atol=1e-11)
    # population formula Omega^2/(Omega^2+delta^2) sin^2(sqrt(Omega^2+delta^2) t/2)
    w = math.hypot(om, de)
    p1 = om ** 2 / w ** 2 * math.sin(0.5 * w * t_ns * 1e-3) ** 2
    assert abs(abs(psi[1]) ** 2 - p1) < 1e-11


@pytest.mark.parametrize("method", ["dense", "lanczos"])
def test_product_state_pins_bit_order(method):
    """Non-interacting atoms (C = 0) with distinct per-site drives evolve into the tensor
    product of single-atom states with atom 0 as the leading factor."""
    n, t_ns = 3, 500
    oms = 2 * np.pi * np.array([0.6, 1.1, 1.9])
    des = 2 * np.pi * np.array([0.3, -0.8, 0.0])
    phs = np.array([0.0, 0.7, -1.2])
    om = np.stack([wl.constant(v, t_ns) for v in oms])
    de = np.stack([wl.constant(v, t_ns) for v in des])
    ph = np.stack([wl.constant(v, t_ns) for v in phs])
    psi = run(wl.chain(n, 5.0), om, de, ph, t_ns, 5, method, c6=0.0)
    ref = np.array([1.0 + 0j])
    singles = [single_atom_closed_form(oms[i], des[i], phs[i], t_ns * 1e-3) for i in range(n)]
    for s in singles:
        ref = np.kron(ref, s)
    np.testing.assert_allclose(psi, ref, atol=1e-11)
    occ = observables.occupations(psi)
    np.testing.assert_allclose(occ, [abs(s[1]) ** 2 for s in singles], atol=1e-12)


def test_two_atom_blockade_symmetric_subspace():
    """Two atoms 2 um apart: the dynamics stays in span{|00>, |W>, |11>} with
    H = [[0, O/sqrt2, 0], [O/sqrt2, -d, O/sqrt2], [0, O/sqrt2, U - 2d]] (hand-derived), and in
    full blockade P(one excitation) = sin^2(sqrt2 O t / 2)."""
    r, om, de, t_ns = 2.0, 2 * np.pi, 2 * np.pi * 0.25, 800
    xyz = wl.chain(2, r)
    u = C6 / r ** 6
    psi = run(xyz, wl.constant(om, t_ns), wl.constant(de, t_ns), None, t_ns, 10, "dense")
    g = om / math.sqrt(2)
    h3 = np.array([[0, g, 0], [g, -de, g], [0, g, u - 2 * de]], dtype=complex)
    a = scipy.linalg.expm(-1j * h3 * t_ns * 1e-3) @ np.array([1, 0, 0], dtype=complex)
    ref = np.array([a[0], a[1] / math.sqrt(2), a[1] / math.sqrt(2), a[2]])
    np.testing.assert_allclose(psi, ref, atol=1e-10)
    # full-blockade collective Rabi frequency at resonance
    psi0 = run(xyz, wl.constant(om, t_ns), wl.constant(0.0, t_ns), None, t_ns, 10, "lanczos")
    for t_chk in [t_ns]:
        pw = math.sin(math.sqrt(2) * om * t_chk * 1e-3 / 2) ** 2
        assert abs(abs(psi0[1]) ** 2 + abs(psi0[2]) ** 2 - pw) < 1e-6
        occ = observables.occupations(psi0)
        np.testing.assert_allclose(occ, [pw / 2, pw / 2], atol=1e-6)


def test_three_atom_blockade_sqrt3():
    """Equilateral triangle of side 2 um in full blockade: one shared excitation oscillates
    at sqrt(3) Omega."""
    om, t_ns = 2 * np.pi, 300
    s = 2.0
    xyz = np.array([[0, 0, 0], [s, 0, 0], [s / 2, s * math.sqrt(3) / 2, 0]])
    psi = run(xyz, wl.constant(om, t_ns), wl.constant(0.0, t_ns), None, t_ns, 10, "lanczos")
    p_one = sum(abs(psi[b]) ** 2 for b in (1, 2, 4))
    assert abs(p_one - math.sin(math.sqrt(3) * om * t_ns * 1e-3 / 2) ** 2) < 1e-6


# ------------------------------------------------------------------ formulations
def test_three_formulations_of_h_agree():
    """Dense Kronecker H, tensor-slicing H|psi> and single rows from matrix elements."""
    rng = np.random.default_rng(3)
    n = 5
    xyz = wl.random_register(n, 12.0, 3.0, rng)
    u = model.interaction_matrix(xyz, C6)
    om, de, ph = rng.uniform(0, 10, n), rng.uniform(-10, 10, n), rng.uniform(-3, 3, n)
    psi = wl.random_state(n, rng)
    dense = model.dense_hamiltonian(u, om, de, ph) @ psi
    sliced = model.apply_hamiltonian(psi, u, om, de, ph)
    rows = np.array([model.hamiltonian_row(b, psi, u, om, de, ph) for b in range(1 << n)])
    np.testing.assert_allclose(sliced, dense, atol=1e-9)
    np.testing.assert_allclose(rows, dense, atol=1e-9)
    h = model.dense_hamiltonian(u, om, de, ph)
    assert np.allclose(h, h.conj().T)


def test_interaction_matrix_and_diagonal():
    xyz = np.array([[0, 0, 0], [3.0, 4.0, 0.0], [0, 0, 2.0]])
    u = model.interaction_matrix(xyz, 7.0)
    assert u[0, 1] == pytest.approx(7.0 / 5.0 ** 6, rel=1e-15)
    assert u[2, 0] == pytest.approx(7.0 / 2.0 ** 6, rel=1e-15)
    assert np.allclose(u, u.T) and np.all(np.diag(u) == 0)
    # all-excited state: every pair counted exactly once
    assert model.interaction_energy(0b111, u) == pytest.approx(u[0, 1] + u[0, 2] + u[1, 2])
    # atom 0 is the most significant bit: b = 0b110 excites atoms 0 and 1
    assert model.interaction_energy(0b110, u) == pytest.approx(u[0, 1])
    with pytest.raises(ValueError):
        model.interaction_matrix(np.zeros((2, 3)), 1.0)


def test_midpoint_rule():
    """Sec. III midpoint: dt = 10 uses sample 10k+5; dt = 5 the mean of 5k+2 and 5k+3;
    on a linear ramp the value equals the ramp at (k + 1/2) dt."""
    t_ns = 100
    ramp = np.arange(t_ns + 1, dtype=float) * 0.5 + 1.0
    for k in range(10):
        assert model.midpoint_sample(ramp, 10, k) == ramp[10 * k + 5]
    for k in range(20):
        assert model.midpoint_sample(ramp, 5, k) == 0.5 * (ramp[5 * k + 2] + ramp[5 * k + 3])
        assert model.midpoint_sample(ramp, 5, k) == pytest.approx(1.0 + 0.5 * (k + 0.5) * 5)
    assert model.midpoint_sample(ramp, 1, 99) == 0.5 * (ramp[99] + ramp[100])


# ------------------------------------------------------------------ invariants
def _sweep(n, seed, t_ns=1000, per_site=False):
    rng = np.random.default_rng(seed)
    xyz = wl.random_register(n, 14.0, 5.0, rng)
    om, de, _ = wl.sweep_pulses(t_ns // 8, t_ns - 2 * (t_ns // 8), 2 * np.pi * 2, 2 * np.pi * 3)
    ph = None
    if per_site:
        sc = rng.uniform(0.5, 1.5, n)
        om = np.outer(sc, om)
        de = np.outer(rng.uniform(0.5, 1.5, n), de)
        ph = np.outer(rng.uniform(-1, 1, n), np.ones(t_ns + 1))
    return xyz, om, de, ph


def test_dense_vs_lanczos_time_dependent():
    """The two propagators are independent; per-site drives with phases, odd dt."""
    xyz, om, de, ph = _sweep(6, 11, t_ns=600, per_site=True)
    a = run(xyz, om, de, ph, 600, 5, "dense")
    b, st = run(xyz, om, de, ph, 600, 5, "lanczos", tol=1e-13, return_stats=True)
    assert np.linalg.norm(a - b) < 1e-10
    assert st["iters"] > 0


def test_norm_and_energy_conservation():
    xyz, om, de, ph = _sweep(7, 5, t_ns=1000)
    psi = run(xyz, om, de, ph, 1000, 10, "lanczos")
    assert abs(np.linalg.norm(psi) - 1.0) < 1e-12
    # constant pulse: <H> is conserved
    u = model.interaction_matrix(xyz, C6)
    t_ns = 500
    om_c, de_c = wl.constant(2 * np.pi * 1.5, t_ns), wl.constant(2 * np.pi * 0.5, t_ns)
    pars = model.step_parameters(7, om_c, de_c, None, 10, 0)
    apply_h = lambda x: model.apply_hamiltonian(x, u, *pars)
    rng = np.random.default_rng(1)
    psi0 = wl.random_state(7, rng)
    e0 = observables.energy(psi0, apply_h)
    psi1 = run(xyz, om_c, de_c, None, t_ns, 10, "lanczos", psi0=psi0)
    assert abs(observables.energy(psi1, apply_h) - e0) < 1e-9 * max(1.0, abs(e0))


def test_step_splitting_constant_h():
    """K steps of dt equal one exponential over K dt for a constant H."""
    xyz = wl.chain(5, 6.0)
    t_ns = 400
    om, de = wl.constant(2 * np.pi, t_ns), wl.constant(2 * np.pi * 0.3, t_ns)
    psi = run(xyz, om, de, None, t_ns, 10, "lanczos")
    u = model.interaction_matrix(xyz, C6)
    h = model.dense_hamiltonian(u, *model.step_parameters(5, om, de, None, 10, 0))
    e0 = np.zeros(32, dtype=complex)
    e0[0] = 1
    ref = scipy.linalg.expm(-1j * h * t_ns * 1e-3) @ e0
    np.testing.assert_allclose(psi, ref, atol=1e-10)


def test_time_reversal():
    """Reversed sample arrays with Omega, delta and C negated apply exp(+i H_k dt) for
    k = K-1..0 and return the initial state."""
    xyz, om, de, ph = _sweep(6, 9, t_ns=700, per_site=True)
    rng = np.random.default_rng(2)
    psi0 = wl.random_state(6, rng)
    fwd = run(xyz, om, de, ph, 700, 7, "lanczos", psi0=psi0)
    back = run(xyz, -om[..., ::-1], -de[..., ::-1], ph[..., ::-1], 700, 7, "lanczos",
               c6=-C6, psi0=fwd)
    assert np.linalg.norm(back - psi0) < 1e-10


def test_dt_squared_convergence():
    """Sec. III: the midpoint scheme is second order in dt on a smooth pulse."""
    t_ns = 1200
    xyz = wl.chain(4, 7.0)
    tt = np.arange(t_ns + 1) / t_ns
    om = 2 * np.pi * 2.0 * np.sin(np.pi * tt) ** 2
    de = 2 * np.pi * 3.0 * (2 * tt - 1)
    ref = run(xyz, om, de, None, t_ns, 1, "dense")
    errs = [np.linalg.norm(run(xyz, om, de, None, t_ns, dt, "dense") - ref) for dt in (40, 20, 10)]
    for a, b in zip(errs, errs[1:]):
        assert 3.0 < a / b < 5.0


def test_mirror_symmetry_chain10():
    """Global drive on a uniform chain: <n_i> = <n_{N-1-i}>, and sum_i <n_i> = <popcount>."""
    w = wl.chain10()
    psi = evolve.evolve_workload(w, method="dense")
    occ = observables.occupations(psi)
    np.testing.assert_allclose(occ, occ[::-1], atol=1e-12)
    p = observables.probabilities(psi)
    pop = np.array([bin(b).count("1") for b in range(p.size)])
    assert abs(occ.sum() - (p * pop).sum() / p.sum()) < 1e-12


def test_lanczos_substeps_when_kmax_small():
    """With a tiny Krylov space the step is halved with the same H_k; the result is
    unchanged."""
    xyz = wl.chain(5, 7.0)
    om, de, _ = wl.sweep_pulses(50, 100, 2 * np.pi * 2, 2 * np.pi * 3)
    a = run(xyz, om, de, None, 200, 20, "dense")
    b, st = run(xyz, om, de, None, 200, 20, "lanczos", kmax=6, tol=1e-12, return_stats=True)
    assert st["substeps"] > 0
    assert np.linalg.norm(a - b) < 1e-10


def test_invariant_subspace_happy_breakdown():
    """Omega = 0: |0...0> is an eigenvector, the Krylov space has dimension 1."""
    t_ns = 100
    psi, st = run(wl.chain(4, 5.0), wl.constant(0.0, t_ns), wl.constant(3.0, t_ns), None, t_ns,
                  10, "lanczos", return_stats=True)
    assert st["iters"] == 10
    assert abs(psi[0] - 1.0) < 1e-14


# ------------------------------------------------------------------ observables
def test_splitmix64_published_outputs():
    with open(os.path.join(GOLDEN, "splitmix64.txt")) as f:
        rows = [l.split() for l in f if l.strip() and not l.startswith("#")]
    for seed, idx, val in rows:
        assert observables.splitmix64(int(seed), int(idx) + 1)[-1] == int(val)
    u = observables.uniforms(7, 1000)
    assert np.all((u >= 0) & (u < 1))


def test_sampler_brute_force_definition():
    rng = np.random.default_rng(5)
    psi = wl.random_state(4, rng)
    psi[3] = 0  # a zero-probability state must never be drawn
    p = observables.probabilities(psi)
    got = observables.sample(psi, 11, 500)
    u = observables.uniforms(11, 500)
    for s in range(500):
        target = u[s] * sum(p)
        acc, b = 0.0, None
        for i, pi in enumerate(p):  # smallest b with CDF(b) > target
            acc += pi
            if acc > target:
                b = i
                break
        assert got[s] == b
    assert 3 not in set(got.tolist())


def test_sampler_frequencies():
    rng = np.random.default_rng(8)
    psi = wl.random_state(3, rng)
    p = observables.probabilities(psi)
    shots = 40000
    counts = np.bincount(observables.sample(psi, 0, shots).astype(np.int64), minlength=8)
    chi2 = np.sum((counts - shots * p) ** 2 / (shots * p))
    assert chi2 < 30.0  # 7 degrees of freedom; p-value ~ 1e-4


def test_fidelity_loss():
    rng = np.random.default_rng(4)
    a = wl.random_state(5, rng)
    assert observables.fidelity_loss(a, np.exp(0.7j) * a) < 1e-30 + 1e-15
    b = wl.random_state(5, rng)
    b = b - np.vdot(a, b) * a
    assert abs(observables.fidelity_loss(a, b) - 1.0) < 1e-14
    eps = 1e-7
    c = (a + eps * b / np.linalg.norm(b))
    assert observables.fidelity_loss(a, c) == pytest.approx(eps ** 2, rel=1e-6)


def test_energy_expectation():
    """<H> of a basis state is its diagonal entry (pair energies minus detunings); for one
    atom in a|0> + b|1>, <H> = -delta |b|^2 + Omega Re(conj(b) a e^{-i phi})."""
    rng = np.random.default_rng(12)
    n = 5
    xyz = wl.random_register(n, 12.0, 3.0, rng)
    u = model.interaction_matrix(xyz, C6)
    om, de, ph = rng.uniform(0, 10, n), rng.uniform(-10, 10, n), rng.uniform(-3, 3, n)
    apply_h = lambda x: model.apply_hamiltonian(x, u, om, de, ph)
    for b in (0, 1, 0b10110, 0b11111):
        e = np.zeros(1 << n, dtype=complex)
        e[b] = 1.0
        lv = model.atom_levels(b, n)
        want = sum(u[i, j] for i in range(n) for j in range(i) if lv[i] and lv[j]) - sum(
            de[i] for i in range(n) if lv[i])
        assert observables.energy(e, apply_h) == pytest.approx(want, rel=1e-14, abs=1e-12)
    a, b = 0.6 * np.exp(0.3j), 0.8 * np.exp(-1.1j)
    o1, d1, p1 = 3.0, 1.7, 0.9
    want = -d1 * abs(b) ** 2 + o1 * (np.conj(b) * a * np.exp(-1j * p1)).real
    got = observables.energy(np.array([a, b]), lambda x: model.apply_hamiltonian(
        x, np.zeros((1, 1)), [o1], [d1], [p1]))
    assert got == pytest.approx(want, rel=1e-14)


def test_correlations_pins():
    """<n_i n_j>: basis states (0/1 products), a product state (<n_i n_j> = <n_i><n_j> off
    the diagonal, <n_i> on it) and the two-atom blockade state (|01> + |10>)/sqrt(2), whose
    pair correlator vanishes."""
    n = 4
    for b in (0, 5, 15, 9):
        psi = np.zeros(1 << n, complex)
        psi[b] = 1
        lv = np.array(model.atom_levels(b, n), float)
        np.testing.assert_array_equal(observables.correlations(psi), np.outer(lv, lv))
    rng = np.random.default_rng(3)
    singles = [rng.standard_normal(2) + 1j * rng.standard_normal(2) for _ in range(n)]
    psi = singles[0]
    for s_ in singles[1:]:
        psi = np.kron(psi, s_)
    q = np.array([abs(s_[1]) ** 2 / (abs(s_[0]) ** 2 + abs(s_[1]) ** 2) for s_ in singles])
    want = np.outer(q, q)
    np.fill_diagonal(want, q)
    np.testing.assert_allclose(observables.correlations(psi), want, atol=1e-14)
    w = np.array([0, 1, 1, 0]) / np.sqrt(2)
    np.testing.assert_allclose(observables.correlations(w), [[0.5, 0.0], [0.0, 0.5]], atol=1e-15)


def test_square20_golden_symmetries():
    """The stored oracle result of the 4x5 lattice sweep (tests/golden/make_square20.py):
    global pulses on a lattice with two mirror axes give occupations invariant under both
    reflections; the norm is conserved; the stored amplitudes reproduce the occupations."""
    import os
    g = np.load(os.path.join(os.path.dirname(__file__), "golden", "square20_final.npz"))
    occ = g["occ"].reshape(4, 5)
    np.testing.assert_allclose(occ, occ[::-1, :], atol=1e-10)
    np.testing.assert_allclose(occ, occ[:, ::-1], atol=1e-10)
    assert abs(float(g["norm"]) - 1.0) < 1e-12
    psi = np.zeros(1 << 20, complex)
    psi[g["idx"].astype(np.int64)] = g["amp"]
    assert float(g["dropped_mass"]) < 1e-12
    np.testing.assert_allclose(observables.occupations(psi), g["occ"], atol=2e-12)
