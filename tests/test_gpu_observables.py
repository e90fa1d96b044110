"""Observables beyond <n_i> and samples (Sec. IV: expectation values of emulator outputs):
<n_i n_j> correlators and <H> of device states against the oracle, and occupations at
intermediate times recorded by the pass that forms each state, against the oracle's
evolution at the same steps."""
import numpy as np
import pytest

from oracle import evolve, model, observables
from paper_2510_09813_amd import rsv
from paper_2510_09813_amd import workloads as wl
from tests.gpu_util import to_dev

pytestmark = pytest.mark.gpu
OCC = {"c128": 1e-8, "c64": 1e-5}


@pytest.fixture(scope="module")
def ctx():
    import torch
    torch.cuda.set_device(0)
    c = rsv.rsv_ctx_create(0)
    yield c
    rsv.rsv_ctx_destroy(c)


@pytest.mark.parametrize("prec", ["c128", "c64"])
@pytest.mark.parametrize("n", [1, 2, 5, 9, 12, 13, 17, 22])
def test_correlations_of_device_states(ctx, n, prec):
    """Tile boundaries at 12 bits, ragged chunks below, zero blocks; at 22 atoms ten index
    bits above the 4096-amplitude chunks."""
    rng = np.random.default_rng(100 + n)
    psi = wl.random_state(n, rng) * (rng.uniform(0, 1, 1 << n) ** 2)
    psi[rng.integers(0, 1 << n, max(1, (1 << n) // 8))] = 0
    if prec == "c64":
        psi = psi.astype(np.complex64).astype(np.complex128)
    got = rsv.rsv_correlations_device(ctx, n, to_dev(psi, prec), prec)
    want = observables.correlations(psi)
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-12)
    np.testing.assert_array_equal(got, got.T)
    np.testing.assert_allclose(np.diag(got), rsv.rsv_occupations_device(ctx, n, to_dev(psi, prec), prec),
                               atol=1e-13)


@pytest.mark.parametrize("prec", ["c128", "c64"])
@pytest.mark.parametrize("n,per_site", [(3, False), (6, True), (11, False), (16, True), (21, False),
                                        (22, False), (23, True)])
def test_energy_of_device_states(ctx, n, per_site, prec):
    """<H_k> of a random state through the H|psi> passes, against the oracle's H applied
    to it; at 22 (complex64) and 23 atoms the low pass also flips top bits from
    neighbouring tiles."""
    rng = np.random.default_rng(200 + n)
    xyz = wl.random_register(n, 25.0, 4.5, rng)
    om = rng.uniform(0, 15, (n, 41) if per_site else 41)
    de = rng.uniform(-20, 20, (n, 41) if per_site else 41)
    ph = rng.uniform(-2, 2, (n, 41)) if per_site else None
    reg = rsv.rsv_register_create(ctx, xyz, wl.C6_RB, prec)
    psi = wl.random_state(n, rng)
    if prec == "c64":
        psi = psi.astype(np.complex64).astype(np.complex128)
    step, dt = 2, 10
    got = rsv.rsv_energy_device(reg, rsv.PulseArrays(om, de, ph), step, dt, to_dev(psi, prec))
    rsv.rsv_register_destroy(reg)
    u = model.interaction_matrix(xyz, wl.C6_RB)
    pars = model.step_parameters(n, om, de, ph, dt, step)
    want = observables.energy(psi, lambda x: model.apply_hamiltonian(x, u, *pars))
    # rounding scale: <psi| |H| |psi> with every term taken in magnitude
    absh = model.apply_hamiltonian(np.abs(psi), np.abs(u), np.abs(pars[0]), -np.abs(pars[1]),
                                   np.zeros(n))
    scale = float(np.vdot(np.abs(psi), absh).real)
    eps = 2.0 ** -52 if prec == "c128" else 2.0 ** -23
    assert abs(got - want) <= 4 * (n + 3) * eps * scale, (got, want, scale)


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_observed_evolution_chain10(ctx, prec):
    """<n_i> after every 10th step of the 10-atom chain against the dense oracle's states at
    those steps; recording them leaves the evolved state unchanged bit for bit."""
    import torch
    w = wl.chain10()
    reg = rsv.rsv_register_create(ctx, w.xyz, w.c6, prec)
    pulses = rsv.PulseArrays(w.omega, w.delta)
    tol = w.tol if prec == "c128" else 1e-7
    dt = torch.complex128 if prec == "c128" else torch.complex64
    a = torch.zeros(1 << w.n_atoms, dtype=dt, device="cuda:0")
    a[0] = 1
    b = a.clone()
    st, occ = rsv.rsv_evolve_device_observed(reg, pulses, rsv.evolve_opts(w.dt_ns, tol, w.kmax), a, 10)
    rsv.rsv_evolve_device(reg, pulses, rsv.evolve_opts(w.dt_ns, tol, w.kmax), b)
    torch.cuda.synchronize()
    rsv.rsv_register_destroy(reg)
    assert torch.equal(a, b)
    assert occ.shape == (10, w.n_atoms) and st.steps == 100
    psi = None
    for r in range(10):
        psi = evolve.evolve_workload(w, method="dense", psi0=psi, steps=10, first_step=10 * r)
        np.testing.assert_allclose(occ[r], observables.occupations(psi), rtol=0, atol=OCC[prec])
    np.testing.assert_allclose(occ[-1], rsv.rsv_occupations_device(ctx, w.n_atoms, a, prec),
                               atol=1e-12)


@pytest.mark.parametrize("prec,n", [("c64", 24), ("c128", 22), ("c64", 14)])
def test_observed_evolution_large(ctx, prec, n):
    """Sizes whose fused sums use 2048 workgroups and 3..5 loop bits (22, 24 atoms) or a
    smaller grid (14): every recorded <n_i> against the occupation kernel on the state
    evolved to the same step."""
    import torch
    w = wl.random27(n_atoms=n, precision=prec)
    reg = rsv.rsv_register_create(ctx, w.xyz, w.c6, prec)
    pulses = rsv.PulseArrays(w.omega, w.delta)
    dt = torch.complex128 if prec == "c128" else torch.complex64
    a = torch.zeros(1 << n, dtype=dt, device="cuda:0")
    a[0] = 1
    b = a.clone()
    first, steps = 40, 3
    st, occ = rsv.rsv_evolve_device_observed(reg, pulses, rsv.evolve_opts(w.dt_ns, w.tol, w.kmax, 12, first, steps), a, 1)
    for r in range(steps):
        rsv.rsv_evolve_device(reg, pulses, rsv.evolve_opts(w.dt_ns, w.tol, w.kmax, 12, first + r, 1), b)
        torch.cuda.synchronize()
        np.testing.assert_allclose(occ[r], rsv.rsv_occupations_device(ctx, n, b, prec), atol=1e-12)
    rsv.rsv_register_destroy(reg)
    assert torch.equal(a, b)


def test_observable_arguments_rejected(ctx):
    import torch
    w = wl.chain10()
    reg = rsv.rsv_register_create(ctx, w.xyz, w.c6, "c128")
    a = torch.zeros(1 << w.n_atoms, dtype=torch.complex128, device="cuda:0")
    a[0] = 1
    with pytest.raises(ValueError):
        rsv.rsv_evolve_device_observed(reg, rsv.PulseArrays(w.omega, w.delta),
                                       rsv.evolve_opts(w.dt_ns), a, 0)
    with pytest.raises(rsv.RsvError):
        rsv.rsv_energy_device(reg, rsv.PulseArrays(w.omega, w.delta), 10 ** 6, w.dt_ns, a)
    with pytest.raises(rsv.RsvError):
        rsv.rsv_correlations_device(ctx, w.n_atoms, torch.zeros_like(a), "c128")  # zero norm
    rsv.rsv_register_destroy(reg)
