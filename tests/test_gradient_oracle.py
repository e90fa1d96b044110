"""Pins of the oracle's pulse gradients (oracle/gradient.py), CPU only: the closed-form
derivatives of the single-atom Rabi population, central finite differences of the pinned
dense evolution, and zero where no step reads a sample."""
import numpy as np
import pytest

from oracle import gradient
from paper_2510_09813_amd import workloads as wl


@pytest.mark.parametrize("om,de", [(2 * np.pi, 0.0), (7.0, 3.0), (4.0, -6.0)])
def test_single_atom_closed_form(om, de):
    """Constant pulses: shifting every sample shifts every step, so the summed sample
    derivatives are the derivatives of P_1 = Omega^2/W^2 sin^2(W T/2), W^2 = Omega^2 + delta^2."""
    t_ns, dt = 600, 10
    T = t_ns * 1e-3
    c, g_om, g_de = gradient.gradient(np.zeros((1, 3)), wl.C6_RB, np.full(t_ns + 1, om),
                                      np.full(t_ns + 1, de), None, t_ns, dt, [1.0])
    W = np.hypot(om, de)
    s, co = np.sin(W * T / 2), np.cos(W * T / 2)
    assert abs(c - om ** 2 / W ** 2 * s ** 2) < 1e-12
    d_om = 2 * om * de ** 2 / W ** 4 * s ** 2 + om ** 3 * T * s * co / W ** 3
    d_de = om ** 2 * de * (-2 * s ** 2 / W ** 4 + T * s * co / W ** 3)
    assert abs(g_om.sum() - d_om) < 1e-11
    assert abs(g_de.sum() - d_de) < 1e-11


def test_against_finite_differences():
    rng = np.random.default_rng(2)
    n, t_ns, dt = 3, 120, 10
    xyz = wl.random_register(n, 12.0, 5.0, rng)
    om = wl.pwl([0, 60, 120], [0, 14, 5], t_ns)
    de = wl.pwl([0, 120], [-10, 8], t_ns)
    ph = np.linspace(0.2, 0.9, t_ns + 1)
    w = [0.5, 1.0, -0.7]
    c, g_om, g_de = gradient.gradient(xyz, wl.C6_RB, om, de, ph, t_ns, dt, w)
    assert abs(c - gradient.value(xyz, wl.C6_RB, om, de, ph, t_ns, dt, w)) < 1e-12
    h = 1e-5
    for j in (5, 15, 35, 65, 115):  # samples on the midpoints of dt = 10 ns steps
        for arr, g in ((om, g_om), (de, g_de)):
            a, b = arr.copy(), arr.copy()
            a[j] += h
            b[j] -= h
            if arr is om:
                fd = (gradient.value(xyz, wl.C6_RB, a, de, ph, t_ns, dt, w)
                      - gradient.value(xyz, wl.C6_RB, b, de, ph, t_ns, dt, w)) / (2 * h)
            else:
                fd = (gradient.value(xyz, wl.C6_RB, om, a, ph, t_ns, dt, w)
                      - gradient.value(xyz, wl.C6_RB, om, b, ph, t_ns, dt, w)) / (2 * h)
            assert abs(g[j] - fd) < 1e-7 * max(1.0, abs(fd)), (j, g[j], fd)
    # with dt = 10 ns only the samples at 10 k + 5 enter a step
    unused = np.setdiff1d(np.arange(t_ns + 1), 10 * np.arange(12) + 5)
    assert np.all(g_om[unused] == 0) and np.all(g_de[unused] == 0)
