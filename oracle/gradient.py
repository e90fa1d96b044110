"""Derivatives of an emulator output with respect to the pulse samples (Sec. IV: the emulator
is differentiable) -- TEST INFRASTRUCTURE ONLY.

C = <psi_K| O |psi_K>, O = sum_i w_i n_i, psi_K the eq. (6) evolution under global pulses
(Sec. III midpoint rule).  Written directly from the chain rule on the product of step
propagators U_k = exp(-i H_k dt) (dense, small N):
    dC/dtheta_k = 2 Re <lambda_{k+1}| dU_k/dtheta_k |psi_k>,
    lambda_{k+1} = U_{k+1}^+ ... U_{K-1}^+ O psi_K,
with dU_k/dtheta the Frechet derivative of the matrix exponential at -i H_k dt in the
direction -i (dH/dtheta) dt (scipy's expm_frechet), for theta = the step's Omega
(dH/dOmega = sum_i (cos phi sigma^x_i - sin phi sigma^y_i) / 2) and delta (dH/ddelta =
-sum_i n_i).  Step k's value is the mean of the samples at floor(m) and ceil(m),
m = (k + 1/2) dt, so each of the two receives half of the step's derivative.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.linalg import expm, expm_frechet

from . import model


def gradient(xyz, c6, omega, delta, phi, t_ns: int, dt_ns: int, weights, psi0=None,
             steps=None, first_step: int = 0):
    """(C, dC/dOmega_j, dC/ddelta_j) for the 1-D (global) sample arrays."""
    n = int(np.asarray(xyz).shape[0])
    u = model.interaction_matrix(xyz, c6)
    omega = np.asarray(omega, dtype=np.float64)
    delta = np.asarray(delta, dtype=np.float64)
    obs = sum(w * np.real(np.diag(model._embed(model.N_OP, i, n))) for i, w in enumerate(weights))
    total = t_ns // dt_ns
    count = total - first_step if steps is None else min(steps, total - first_step)
    tau = dt_ns * 1e-3
    psi = np.zeros(1 << n, dtype=np.complex128)
    if psi0 is None:
        psi[0] = 1.0
    else:
        psi[:] = psi0
    states, props, hams = [], [], []
    for k in range(first_step, first_step + count):
        pars = model.step_parameters(n, omega, delta, phi, dt_ns, k)
        h = model.dense_hamiltonian(u, *pars)
        uk = expm(-1j * tau * h)
        states.append(psi)
        props.append(uk)
        hams.append((h, pars[2]))
        psi = uk @ psi
    lam = obs * psi
    value = float(np.vdot(psi, lam).real)
    g_om, g_de = np.zeros(omega.size), np.zeros(delta.size)
    v_de = -sum(model._embed(model.N_OP, i, n) for i in range(n))
    for idx in range(count - 1, -1, -1):
        k = first_step + idx
        h, ph = hams[idx]
        v_om = sum(0.5 * model._embed(math.cos(ph[i]) * model.SIGMA_X - math.sin(ph[i]) * model.SIGMA_Y, i, n)
                   for i in range(n))
        m = (k + 0.5) * dt_ns
        for v, g in ((v_om, g_om), (v_de, g_de)):
            frechet = expm_frechet(-1j * tau * h, -1j * tau * v, compute_expm=False)
            d = 2.0 * float(np.vdot(lam, frechet @ states[idx]).real)
            g[int(math.floor(m))] += 0.5 * d
            g[int(math.ceil(m))] += 0.5 * d
        lam = props[idx].conj().T @ lam
    return value, g_om, g_de


def value(xyz, c6, omega, delta, phi, t_ns, dt_ns, weights, psi0=None):
    """C alone, by the pinned dense evolution (for finite differences)."""
    from . import evolve
    psi = evolve.evolve(xyz, c6, omega, delta, phi, t_ns, dt_ns, psi0=psi0, method="dense")
    n = int(np.asarray(xyz).shape[0])
    p = np.abs(psi) ** 2
    return float(sum(w * np.take(p.reshape((2,) * n), 1, axis=i).sum() for i, w in enumerate(weights)))
