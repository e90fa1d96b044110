"""Open-system dynamics by the Lindblad master equation (Sec. III.A) -- TEST INFRASTRUCTURE
ONLY.

The paper evolves the full master equation with a Krylov method but does not print it; the
standard Lindblad form is written out here from its definition:
    d rho/dt = -i [H, rho] + sum_k (L_k rho L_k^+ - 1/2 {L_k^+ L_k, rho}),
with H the Hamiltonian of eq. (3) (plus the drive phase) and, per atom i, the jump operators
    relaxation of the Rydberg level   L = sqrt(gamma_r) |0><1|_i,
    dephasing                         L = sqrt(2 gamma_phi) n_i   (coherences decay at gamma_phi).
The Liouvillian is assembled as a dense 4^N x 4^N matrix acting on rho flattened row-major
(vec(A rho B) = (A kron B^T) vec(rho)), and each step applies scipy's matrix exponential of
dt L_k (the pulse held at its midpoint value, Sec. III).  Small N only (N <= 5).
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import expm

from . import model

SIGMA_MINUS = np.array([[0.0, 1.0], [0.0, 0.0]], dtype=np.complex128)  # |0><1|


def jump_operators(n: int, gamma_r: float, gamma_phi: float):
    ops = []
    for i in range(n):
        if gamma_r > 0:
            ops.append(np.sqrt(gamma_r) * model._embed(SIGMA_MINUS, i, n))
        if gamma_phi > 0:
            ops.append(np.sqrt(2.0 * gamma_phi) * model._embed(model.N_OP, i, n))
    return ops


def liouvillian(h: np.ndarray, ops) -> np.ndarray:
    """Dense superoperator of d rho/dt on row-major vec(rho)."""
    d = h.shape[0]
    eye = np.eye(d)
    lv = -1j * (np.kron(h, eye) - np.kron(eye, h.T))
    for op in ops:
        ld = op.conj().T @ op
        lv += np.kron(op, op.conj()) - 0.5 * np.kron(ld, eye) - 0.5 * np.kron(eye, ld.T)
    return lv


def apply_liouvillian(rho, h, ops) -> np.ndarray:
    """d rho/dt from its definition with matrix products (no superoperator): for checking
    the operator at sizes whose 4^N x 4^N matrix would not fit."""
    rho = np.asarray(rho, dtype=np.complex128)
    out = -1j * (h @ rho - rho @ h)
    for op in ops:
        ld = op.conj().T @ op
        out += op @ rho @ op.conj().T - 0.5 * (ld @ rho + rho @ ld)
    return out


def liouvillian_element(r: int, c: int, rho, u, omega, delta, phi, gamma_r: float,
                        gamma_phi: float) -> complex:
    """(d rho/dt)_rc from matrix elements, for large N: (H rho)_rc is row r of H applied to
    column c of rho, (rho H)_rc = conj((H conj(rho_r.))_c) with rho_r. row r (H Hermitian),
    and per atom i (level bits ri, ci of r and c) the relaxation adds gamma_r rho_{r+, c+}
    (both levels raised to 1) when ri = ci = 0 and removes gamma_r (ri + ci)/2 rho_rc, the
    dephasing removes gamma_phi rho_rc when ri != ci."""
    n = len(omega)
    rho = np.asarray(rho)
    h_rho = model.hamiltonian_row(r, rho[:, c], u, omega, delta, phi)
    rho_h = np.conj(model.hamiltonian_row(c, np.conj(rho[r, :]), u, omega, delta, phi))
    out = -1j * (h_rho - rho_h)
    lr, lc = model.atom_levels(r, n), model.atom_levels(c, n)
    for i in range(n):
        bit = 1 << (n - 1 - i)
        if lr[i] == 0 and lc[i] == 0:
            out += gamma_r * rho[r | bit, c | bit]
        out -= 0.5 * gamma_r * (lr[i] + lc[i]) * rho[r, c]
        if lr[i] != lc[i]:
            out -= gamma_phi * rho[r, c]
    return complex(out)


def evolve(xyz, c6, omega, delta, phi, t_ns: int, dt_ns: int, rho0, gamma_r: float,
           gamma_phi: float, steps=None, first_step: int = 0) -> np.ndarray:
    """rho after steps first_step .. first_step + steps - 1 of rho_{k+1} = exp(dt L_k) rho_k."""
    n = int(np.asarray(xyz).shape[0])
    u = model.interaction_matrix(xyz, c6)
    ops = jump_operators(n, gamma_r, gamma_phi)
    total = t_ns // dt_ns
    count = total - first_step if steps is None else min(steps, total - first_step)
    rho = np.array(rho0, dtype=np.complex128).reshape(-1)
    tau = dt_ns * 1e-3
    key, prop = None, None
    for k in range(first_step, first_step + count):
        om, de, ph = model.step_parameters(n, omega, delta, phi, dt_ns, k)
        kk = (om.tobytes(), de.tobytes(), ph.tobytes())
        if kk != key:
            prop = expm(tau * liouvillian(model.dense_hamiltonian(u, om, de, ph), ops))
            key = kk
        rho = prop @ rho
    d = 1 << n
    return rho.reshape(d, d)


def occupations(rho) -> np.ndarray:
    """<n_i> = Tr(rho n_i) / Tr(rho)."""
    rho = np.asarray(rho)
    n = int(round(np.log2(rho.shape[0])))
    p = np.real(np.diag(rho))
    t = p.reshape((2,) * n)
    return np.array([np.take(t, 1, axis=i).sum() for i in range(n)]) / p.sum()
