"""Pulse gradients on the GPU (Sec. IV: derivatives of expectation values with respect to the
pulse) against the oracle's dense adjoint with scipy's Frechet derivatives, sample by sample,
and the single-atom closed form."""
import numpy as np
import pytest

from oracle import gradient
from paper_2510_09813_amd import rsv
from paper_2510_09813_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    torch.cuda.set_device(0)
    c = rsv.rsv_ctx_create(0)
    yield c
    rsv.rsv_ctx_destroy(c)


def gpu_grad(ctx, xyz, c6, om, de, ph, dt, w, prec, psi0=None, tol=None):
    reg = rsv.rsv_register_create(ctx, xyz, c6, prec)
    try:
        tol = tol or (1e-11 if prec == "c128" else 1e-7)
        return rsv.rsv_gradient_occupations(reg, rsv.PulseArrays(om, de, ph),
                                            rsv.evolve_opts(dt, tol, 40, 12), w, psi0)
    finally:
        rsv.rsv_register_destroy(reg)


def test_single_atom_closed_form(ctx):
    om, de, t_ns = 7.0, 3.0, 600
    T = t_ns * 1e-3
    c, g_om, g_de, st = gpu_grad(ctx, np.zeros((1, 3)), wl.C6_RB, np.full(t_ns + 1, om),
                                 np.full(t_ns + 1, de), None, 10, [1.0], "c128")
    W = np.hypot(om, de)
    s, co = np.sin(W * T / 2), np.cos(W * T / 2)
    assert abs(c - om ** 2 / W ** 2 * s ** 2) < 1e-10
    assert abs(g_om.sum() - (2 * om * de ** 2 / W ** 4 * s ** 2 + om ** 3 * T * s * co / W ** 3)) < 1e-9
    assert abs(g_de.sum() - om ** 2 * de * (-2 * s ** 2 / W ** 4 + T * s * co / W ** 3)) < 1e-9
    assert st.steps == 60


@pytest.mark.parametrize("prec", ["c128", "c64"])
@pytest.mark.parametrize("n,dt,phase", [(2, 10, False), (4, 5, True), (7, 10, True), (9, 10, False)])
def test_against_oracle(ctx, n, dt, phase, prec):
    rng = np.random.default_rng(30 + n)
    t_ns = 200
    xyz = wl.random_register(n, 16.0, 5.0, rng)
    om = wl.pwl([0, 80, 200], [0, 13, 4], t_ns)
    de = wl.pwl([0, 200], [-9, 11], t_ns)
    ph = np.linspace(-0.4, 0.8, t_ns + 1) if phase else None
    w = rng.uniform(-1, 1, n)
    psi0 = wl.random_state(n, rng)
    c, g_om, g_de, st = gpu_grad(ctx, xyz, wl.C6_RB, om, de, ph, dt, w, prec, psi0)
    rc, r_om, r_de = gradient.gradient(xyz, wl.C6_RB, om, de, ph, t_ns, dt, w, psi0=psi0)
    scale = max(np.abs(r_om).max(), np.abs(r_de).max())
    tol = 1e-8 if prec == "c128" else 2e-4
    assert abs(c - rc) <= (1e-10 if prec == "c128" else 1e-5)
    assert np.abs(g_om - r_om).max() <= tol * scale, np.abs(g_om - r_om).max() / scale
    assert np.abs(g_de - r_de).max() <= tol * scale, np.abs(g_de - r_de).max() / scale
    assert st.krylov_iters > 3 * st.steps


def test_gradient_rejections(ctx):
    reg = rsv.rsv_register_create(ctx, wl.chain(3, 5.0), wl.C6_RB, "c128")
    om = np.ones((3, 21))
    with pytest.raises(ValueError):  # per-site pulses
        rsv.rsv_gradient_occupations(reg, rsv.PulseArrays(om, om), rsv.evolve_opts(10), [1, 1, 1])
    with pytest.raises(ValueError):
        rsv.rsv_gradient_occupations(reg, rsv.PulseArrays(om[0], om[0]), rsv.evolve_opts(10), [1, 1])
    with pytest.raises(rsv.RsvError):
        rsv.rsv_gradient_occupations(reg, rsv.PulseArrays(om[0], om[0]), rsv.evolve_opts(10),
                                     [1, np.nan, 1])
    rsv.rsv_register_destroy(reg)
