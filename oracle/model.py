"""The Rydberg Hamiltonian of eq. (3) (Sec. II.A) and the pulse discretisation of Sec. III.

Conventions (each is a reading of the paper, see the design notes):
* |1> is the Rydberg state and n = |1><1| (Sec. II.A).
* Atom i (0-based) is the i-th tensor factor of c_{i_1...i_N} in row-major order (Sec. II.B),
  so atom 0 is the most significant bit of the flat index.
* The drive of atom i is Omega_i/2 (cos phi_i sigma^x - sin phi_i sigma^y) with
  sigma^y = [[0, -i], [i, 0]]; for phi = 0 this is the Omega_i/2 sigma^x term of eq. (3).
* Each pair i > j is counted once in the interaction sum, U_ij = C / |r_i - r_j|^6.
"""
from __future__ import annotations

import math

import numpy as np

SIGMA_X = np.array([[0.0, 1.0], [1.0, 0.0]], dtype=np.complex128)
SIGMA_Y = np.array([[0.0, -1.0j], [1.0j, 0.0]], dtype=np.complex128)
N_OP = np.array([[0.0, 0.0], [0.0, 1.0]], dtype=np.complex128)


def interaction_matrix(xyz, c6: float) -> np.ndarray:
    """U[i, j] = C / |r_i - r_j|^6 for i != j, zero diagonal (eq. 3, third term).
    Coincident atoms are rejected."""
    xyz = np.asarray(xyz, dtype=np.float64)
    n = xyz.shape[0]
    u = np.zeros((n, n))
    for i in range(n):
        for j in range(i):
            r = math.sqrt(float(np.sum((xyz[i] - xyz[j]) ** 2)))
            if r == 0.0:
                raise ValueError(f"atoms {i} and {j} coincide")
            u[i, j] = u[j, i] = c6 / r ** 6
    return u


def midpoint_sample(samples: np.ndarray, dt_ns: int, k: int) -> np.ndarray:
    """Sec. III: the pulse is held constant over step k at its midpoint value.  With
    m = (k + 1/2) dt (in ns, samples on the 1 ns grid), the value is the mean of the samples at
    floor(m) and ceil(m).  Works on the last axis, so [T+1] and [N, T+1] arrays both work."""
    m = (k + 0.5) * dt_ns
    lo, hi = int(math.floor(m)), int(math.ceil(m))
    return 0.5 * (samples[..., lo] + samples[..., hi])


def step_parameters(n_atoms: int, omega, delta, phi, dt_ns: int, k: int):
    """Per-site (Omega_i, delta_i, phi_i) of the constant Hamiltonian H_k of step k."""
    def per_site(x):
        if x is None:
            return np.zeros(n_atoms)
        v = midpoint_sample(np.asarray(x, dtype=np.float64), dt_ns, k)
        return np.broadcast_to(v, (n_atoms,)).astype(np.float64).copy()
    return per_site(omega), per_site(delta), per_site(phi)


def _embed(op: np.ndarray, i: int, n: int) -> np.ndarray:
    """op acting on atom i of n, identity elsewhere; atom 0 is the leftmost factor."""
    return np.kron(np.kron(np.eye(1 << i), op), np.eye(1 << (n - 1 - i)))


def _occupation_vector(i: int, n: int) -> np.ndarray:
    """Diagonal of the embedded n_i, from the Kronecker product of diagonals."""
    return np.kron(np.kron(np.ones(1 << i), np.array([0.0, 1.0])), np.ones(1 << (n - 1 - i)))


def dense_hamiltonian(u: np.ndarray, omega, delta, phi) -> np.ndarray:
    """H of eq. (3) (plus the drive phase) as a dense 2^N x 2^N complex matrix, assembled
    term by term from Kronecker products."""
    n = len(omega)
    diag = np.zeros(1 << n)
    for i in range(n):
        diag -= delta[i] * _occupation_vector(i, n)
        for j in range(i):
            diag += u[i, j] * _occupation_vector(i, n) * _occupation_vector(j, n)
    h = np.diag(diag).astype(np.complex128)
    for i in range(n):
        drive = math.cos(phi[i]) * SIGMA_X - math.sin(phi[i]) * SIGMA_Y
        h += 0.5 * omega[i] * _embed(drive, i, n)
    return h


def diagonal_tensor(u: np.ndarray, delta) -> np.ndarray:
    """Diagonal of H as an N-dimensional (2,...,2) tensor: sum_{i>j} U_ij n_i n_j - sum_i delta_i n_i.

    The result depends only on (U, delta); the most recent ones are kept (see
    ``_DIAG_CACHE``), so the many H|psi> of one time step build it once.  The cached array
    is the one this function computes, so caching changes no arithmetic."""
    key = (np.asarray(u, dtype=np.float64).tobytes(), np.asarray(delta, dtype=np.float64).tobytes())
    hit = _DIAG_CACHE.get(key)
    if hit is not None:
        return hit
    d = _diagonal_tensor(u, delta)
    d.setflags(write=False)
    _DIAG_CACHE.clear()  # one entry: at 27 atoms it is 1 GiB
    _DIAG_CACHE[key] = d
    return d


_DIAG_CACHE: dict = {}


def _diagonal_tensor(u: np.ndarray, delta) -> np.ndarray:
    n = len(delta)
    occ = [np.arange(2.0).reshape([2 if a == i else 1 for a in range(n)]) for i in range(n)]
    d = np.zeros((2,) * n)
    for i in range(n):
        d = d - delta[i] * occ[i]
        for j in range(i):
            d = d + u[i, j] * occ[i] * occ[j]
    return d


def apply_hamiltonian(psi: np.ndarray, u: np.ndarray, omega, delta, phi) -> np.ndarray:
    """H|psi> in two steps (Sec. III.A): the diagonal, then for each atom the amplitudes with
    that atom's level swapped, scaled by the drive matrix element.  psi is the tensor
    c_{i_1...i_N} in row-major order, so for atom i the flat vector viewed as
    (2^i, 2, 2^(N-1-i)) has the atom's level on its middle axis: entry [:, 0, :] holds the
    amplitudes with atom i in |0>, entry [:, 1, :] those with atom i in |1>."""
    n = len(omega)
    x = np.asarray(psi, dtype=np.complex128).reshape(-1)
    out = diagonal_tensor(u, delta).reshape(-1) * x
    term = np.empty(x.size // 2, dtype=np.complex128)
    for i in range(n):
        up = 0.5 * omega[i] * np.exp(-1j * phi[i])    # <1|h_i|0>
        down = 0.5 * omega[i] * np.exp(1j * phi[i])   # <0|h_i|1>
        shape = (1 << i, 2, 1 << (n - 1 - i))
        t, o, tm = x.reshape(shape), out.reshape(shape), term.reshape(shape[0], shape[2])
        np.multiply(up, t[:, 0, :], out=tm)
        o[:, 1, :] += tm
        np.multiply(down, t[:, 1, :], out=tm)
        o[:, 0, :] += tm
    return out


def atom_levels(b: int, n: int):
    """Levels (0/1) of atoms 0..n-1 in basis index b (atom 0 = most significant bit)."""
    return [(b >> (n - 1 - i)) & 1 for i in range(n)]


def interaction_energy(b: int, u: np.ndarray) -> float:
    """sum_{i>j} U_ij n_i n_j evaluated on basis state b, pair by pair."""
    n = u.shape[0]
    lv = atom_levels(b, n)
    e = 0.0
    for i in range(n):
        for j in range(i):
            if lv[i] and lv[j]:
                e += u[i, j]
    return e


def hamiltonian_row(b: int, psi: np.ndarray, u: np.ndarray, omega, delta, phi) -> complex:
    """(H psi)_b from the matrix elements of row b: the diagonal entry times psi_b plus one
    off-diagonal entry per atom, coupling b to b with that atom's level swapped."""
    n = len(omega)
    lv = atom_levels(b, n)
    val = (interaction_energy(b, u) - sum(delta[i] * lv[i] for i in range(n))) * psi[b]
    for i in range(n):
        partner = b ^ (1 << (n - 1 - i))
        if lv[i] == 1:
            coef = 0.5 * omega[i] * np.exp(-1j * phi[i])
        else:
            coef = 0.5 * omega[i] * np.exp(1j * phi[i])
        val += coef * psi[partner]
    return complex(val)
