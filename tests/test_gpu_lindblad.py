"""The Lindblad path (Sec. III.A, open systems): the Liouvillian kernel against the oracle's
dense superoperator element by element, the Arnoldi evolution against the oracle's dense
exponentials, no dissipation against the pure-state path, and closed forms at sizes the
dense oracle cannot reach."""
import numpy as np
import pytest

from oracle import lindblad, model
from paper_2510_09813_amd import rsv
from paper_2510_09813_amd import workloads as wl
from tests.gpu_util import rel_err

pytestmark = pytest.mark.gpu
DT = {"c128": "complex128", "c64": "complex64"}
TOL = {"c128": 1e-12, "c64": 1e-5}


@pytest.fixture(scope="module")
def ctx():
    import torch
    torch.cuda.set_device(0)
    c = rsv.rsv_ctx_create(0)
    yield c
    rsv.rsv_ctx_destroy(c)


def dev(rho, prec):
    import torch
    return torch.from_numpy(np.ascontiguousarray(rho).reshape(-1).astype(DT[prec])).to("cuda:0")


def host(t, n):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy().astype(np.complex128).reshape(1 << n, 1 << n)


def random_rho(n, rng):
    a = rng.standard_normal((1 << n, 1 << n)) + 1j * rng.standard_normal((1 << n, 1 << n))
    r = a @ a.conj().T
    return r / np.trace(r)


def pulses(n, t_ns, rng, per_site=True):
    om = wl.pwl([0, t_ns // 2, t_ns], [0, 12, 4], t_ns)
    de = wl.pwl([0, t_ns], [-9, 7], t_ns)
    if not per_site:
        return om, de, None
    return (np.outer(rng.uniform(0.5, 1.5, n), om), np.outer(rng.uniform(0.5, 1.5, n), de),
            np.outer(rng.uniform(-1, 1, n), np.linspace(0, 1, t_ns + 1)))


@pytest.mark.parametrize("prec", ["c128", "c64"])
@pytest.mark.parametrize("n", [1, 2, 3, 5])
def test_liouvillian_against_dense_superoperator(ctx, n, prec):
    import torch
    rng = np.random.default_rng(n)
    xyz = wl.random_register(n, 14.0, 4.0, rng)
    om, de, ph = pulses(n, 100, rng)
    rates = (0.7, 0.45)
    rho = random_rho(n, rng)
    if prec == "c64":
        rho = rho.astype(np.complex64).astype(np.complex128)
    reg = rsv.rsv_register_create(ctx, xyz, wl.C6_RB, prec)
    x = dev(rho, prec)
    y = torch.empty_like(x)
    rsv.rsv_lindblad_apply(reg, rsv.PulseArrays(om, de, ph), 3, 10, rates, x, y)
    rsv.rsv_register_destroy(reg)
    u = model.interaction_matrix(xyz, wl.C6_RB)
    h = model.dense_hamiltonian(u, *model.step_parameters(n, om, de, ph, 10, 3))
    lv = lindblad.liouvillian(h, lindblad.jump_operators(n, *rates))
    ref = (lv @ rho.reshape(-1)).reshape(rho.shape)
    assert rel_err(host(y, n), ref) <= TOL[prec] * (10 if n > 3 else 1), n


@pytest.mark.parametrize("prec", ["c128", "c64"])
@pytest.mark.parametrize("n", [6, 7, 9, 12])
def test_liouvillian_against_matrix_form(ctx, n, prec):
    """6..12 atoms (the gather form up to the largest size it serves): element by element
    against the oracle's matrix-product form, with both channels on and a per-site drive
    with phases."""
    import torch
    rng = np.random.default_rng(40 + n)
    xyz = wl.random_register(n, 18.0, 4.0, rng)
    om, de, ph = pulses(n, 100, rng)
    rates = (0.9, 0.35)
    rho = random_rho(n, rng)
    if prec == "c64":
        rho = rho.astype(np.complex64).astype(np.complex128)
    reg = rsv.rsv_register_create(ctx, xyz, wl.C6_RB, prec)
    x = dev(rho, prec)
    y = torch.empty_like(x)
    rsv.rsv_lindblad_apply(reg, rsv.PulseArrays(om, de, ph), 4, 10, rates, x, y)
    got = host(y, n)
    rsv.rsv_register_destroy(reg)
    u = model.interaction_matrix(xyz, wl.C6_RB)
    h = model.dense_hamiltonian(u, *model.step_parameters(n, om, de, ph, 10, 4))
    ref = lindblad.apply_liouvillian(rho, h, lindblad.jump_operators(n, *rates))
    assert rel_err(got, ref) <= TOL[prec] * 10, n


@pytest.mark.parametrize("prec", ["c128", "c64"])
@pytest.mark.parametrize("n", [13, 14])
def test_tiled_liouvillian_sampled(ctx, n, prec):
    """13 and 14 atoms (the largest density matrix, 4 GiB in complex128): the Liouvillian on
    LDS tiles of 4096 elements (column bits in LDS, row bits and the top column bits from
    neighbouring tiles), 400 sampled elements (tile corners, diagonal and random) against
    the oracle's element-by-element form; any matrix will do, L is linear."""
    import torch
    rng = np.random.default_rng(117 + n)
    xyz = wl.random_register(n, 20.0, 4.0, rng)
    om, de, ph = pulses(n, 100, rng)
    rates = (0.9, 0.35)
    g = torch.Generator(device="cuda:0").manual_seed(13)
    x = torch.randn(1 << (2 * n), dtype=getattr(torch, DT[prec]), device="cuda:0", generator=g)
    y = torch.empty_like(x)
    reg = rsv.rsv_register_create(ctx, xyz, wl.C6_RB, prec)
    rsv.rsv_lindblad_apply(reg, rsv.PulseArrays(om, de, ph), 4, 10, rates, x, y)
    torch.cuda.synchronize()
    rsv.rsv_register_destroy(reg)
    rho = x.cpu().numpy().astype(np.complex128).reshape(1 << n, 1 << n)
    out = y.cpu().numpy().astype(np.complex128).reshape(1 << n, 1 << n)
    d = 1 << n
    pts = [(0, 0), (d - 1, d - 1), (0, d - 1), (d - 1, 0), (1, 4095), (4096 // d, 4095 % d)]
    pts += [(int(i), int(i)) for i in rng.integers(0, d, 30)]
    pts += [(int(a), int(b)) for a, b in rng.integers(0, d, (364, 2))]
    u = model.interaction_matrix(xyz, wl.C6_RB)
    pars = model.step_parameters(n, om, de, ph, 10, 4)
    for r, c in pts:
        want = lindblad.liouvillian_element(r, c, rho, u, *pars, *rates)
        scale = np.abs(rho[r, :]).max() + np.abs(rho[:, c]).max()
        assert abs(out[r, c] - want) <= TOL[prec] * 1e3 * scale, (r, c, out[r, c], want)


@pytest.mark.parametrize("prec", ["c128", "c64"])
@pytest.mark.parametrize("n,per_site,rates", [(2, True, (0.7, 0.45)), (4, False, (1.5, 0.0)),
                                              (4, True, (0.0, 2.0)), (5, False, (0.3, 0.3))])
def test_evolution_against_dense_oracle(ctx, n, per_site, rates, prec):
    rng = np.random.default_rng(10 + n)
    t_ns = 300
    xyz = wl.random_register(n, 14.0, 4.5, rng)
    om, de, ph = pulses(n, t_ns, rng, per_site)
    psi0 = wl.random_state(n, rng)
    rho0 = np.outer(psi0, psi0.conj())
    reg = rsv.rsv_register_create(ctx, xyz, wl.C6_RB, prec)
    x = dev(rho0, prec)
    tol = 1e-11 if prec == "c128" else 1e-7
    st = rsv.rsv_lindblad_evolve_device(reg, rsv.PulseArrays(om, de, ph),
                                        rsv.evolve_opts(10, tol, 40, 12), rates, x)
    got = host(x, n)
    rsv.rsv_register_destroy(reg)
    ref = lindblad.evolve(xyz, wl.C6_RB, om, de, ph, t_ns, 10, rho0, *rates)
    err = np.linalg.norm(got - ref)
    assert err <= (1e-9 if prec == "c128" else 2e-5), err
    assert st.steps == t_ns // 10 and st.krylov_iters >= st.steps
    occ, tr = rsv.rsv_lindblad_occupations(ctx, n, x, prec)
    np.testing.assert_allclose(occ, lindblad.occupations(ref), atol=1e-9 if prec == "c128" else 2e-5)
    assert abs(tr - 1) <= (1e-10 if prec == "c128" else 1e-5)


def test_no_dissipation_equals_pure_state_path(ctx):
    """gamma = 0 at 9 atoms (a 2^18-amplitude density matrix): rho(T) = |psi(T)><psi(T)| with
    psi from the Lanczos pure-state path."""
    import torch
    n, t_ns = 9, 200
    w = wl.serving_job(np.random.default_rng(9), n_min=n, n_max=n, precision="c128")
    w.t_ns, w.omega, w.delta = t_ns, w.omega[:t_ns + 1], w.delta[:t_ns + 1]
    psi0 = wl.random_state(n, np.random.default_rng(3))
    reg = rsv.rsv_register_create(ctx, w.xyz, w.c6, "c128")
    pl = rsv.PulseArrays(w.omega, w.delta)
    x = dev(np.outer(psi0, psi0.conj()), "c128")
    rsv.rsv_lindblad_evolve_device(reg, pl, rsv.evolve_opts(10, 1e-11, 40, 12), (0.0, 0.0), x)
    p = torch.from_numpy(psi0).to("cuda:0")
    rsv.rsv_evolve_device(reg, pl, rsv.evolve_opts(10, 1e-12, 40, 12), p)
    psi = p.cpu().numpy()
    got = host(x, n)
    rsv.rsv_register_destroy(reg)
    assert np.linalg.norm(got - np.outer(psi, psi.conj())) <= 1e-9


def test_independent_atoms_reach_bloch_steady_state(ctx):
    """Eight non-interacting atoms (C = 0), constant drive and detuning with relaxation:
    every atom follows the single-atom oracle evolution and approaches the optical Bloch
    steady state; the trace stays 1."""
    n, t_ns = 8, 6000
    om_, d, g = 5.0, 1.5, 3.0
    reg = rsv.rsv_register_create(ctx, wl.chain(n, 5.0), 0.0, "c128")
    rho0 = np.zeros((1 << n, 1 << n), complex)
    rho0[0, 0] = 1
    x = dev(rho0, "c128")
    st = rsv.rsv_lindblad_evolve_device(reg, rsv.PulseArrays(np.full(t_ns + 1, om_), np.full(t_ns + 1, d)),
                                        rsv.evolve_opts(200, 1e-10, 50, 12), (g, 0.0), x)
    occ, tr = rsv.rsv_lindblad_occupations(ctx, n, x, "c128")
    rsv.rsv_register_destroy(reg)
    one = lindblad.evolve(np.zeros((1, 3)), wl.C6_RB, np.full(t_ns + 1, om_), np.full(t_ns + 1, d),
                          None, t_ns, 200, np.diag([1.0, 0.0]).astype(complex), g, 0.0)
    np.testing.assert_allclose(occ, lindblad.occupations(one)[0], atol=1e-8)
    ss = (om_ ** 2 / 4) / (d ** 2 + om_ ** 2 / 2 + g ** 2 / 4)
    np.testing.assert_allclose(occ, ss, atol=1e-3)
    assert abs(tr - 1) < 1e-9 and st.steps == t_ns // 200


def test_lindblad_rejections(ctx):
    import torch
    reg = rsv.rsv_register_create(ctx, wl.chain(15, 5.0), wl.C6_RB, "c64")
    om = np.ones(11)
    # 15 atoms: beyond the density-matrix limit
    assert rsv.lib().rsv_lindblad_evolve_device(reg, None, None, None, None, None, None) == rsv.RSV_EINVAL
    rsv.rsv_register_destroy(reg)
    reg = rsv.rsv_register_create(ctx, wl.chain(2, 5.0), wl.C6_RB, "c128")
    x = dev(np.eye(4) / 4, "c128")
    with pytest.raises(rsv.RsvError):
        rsv.rsv_lindblad_evolve_device(reg, rsv.PulseArrays(om, om), rsv.evolve_opts(10), (-1.0, 0.0), x)
    with pytest.raises(ValueError):
        rsv.rsv_lindblad_evolve_device(reg, rsv.PulseArrays(om, om), rsv.evolve_opts(10), (0.1, 0.0),
                                       torch.zeros(8, dtype=torch.complex128, device="cuda:0"))
    rsv.rsv_register_destroy(reg)
