"""Seeded synthetic inputs for the Rydberg state-vector emulator.

This module only *generates inputs*: atom registers, pulse samples on the 1 ns grid,
initial states and the serving job stream.  It evaluates no part of the method (no
Hamiltonian, no midpoint rule, no propagation); both the HIP path and the CPU oracle
consume the arrays it returns.

Units: positions in micrometres, time in nanoseconds on the sample grid, Rabi frequency
and detuning in rad/us, phase in rad, interaction constant C6 in rad*us^-1*um^6.

The pulse shapes stand in for the building blocks a pulse-programming front end would
sample (linear ramps and plateaus, sampled at t_n = n ns, Sec. III); the registers follow
the lattice geometries used for the workloads (chain, square, triangular, random with a
minimum distance).  The paper evaluates on no public dataset, so everything is synthetic.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np

TWO_PI = 2.0 * np.pi
C6_RB = 5.42e6  # rad/us * um^6, the hardware constant C of eq. (3) used by every workload


# --------------------------------------------------------------------------- registers
def chain(n: int, spacing: float) -> np.ndarray:
    """1D chain along x: atom i at (i*spacing, 0, 0)."""
    xyz = np.zeros((n, 3))
    xyz[:, 0] = spacing * np.arange(n)
    return xyz


def square_lattice(rows: int, cols: int, spacing: float) -> np.ndarray:
    """rows x cols square lattice, atoms listed row-major."""
    xyz = np.zeros((rows * cols, 3))
    for r in range(rows):
        for c in range(cols):
            xyz[r * cols + c, :2] = (c * spacing, r * spacing)
    return xyz


def triangular_lattice(rows: int, cols: int, spacing: float) -> np.ndarray:
    """rows x cols triangular lattice: odd rows shifted by spacing/2, row pitch
    spacing*sqrt(3)/2, atoms listed row-major."""
    xyz = np.zeros((rows * cols, 3))
    pitch = spacing * np.sqrt(3.0) / 2.0
    for r in range(rows):
        for c in range(cols):
            xyz[r * cols + c, :2] = (c * spacing + (0.5 * spacing if r % 2 else 0.0), r * pitch)
    return xyz


def random_register(n: int, box: float, dmin: float, rng: np.random.Generator,
                    max_tries: int = 100000) -> np.ndarray:
    """n points uniform in [0, box]^2, placed one at a time: a candidate closer than dmin to
    an already placed atom is redrawn (sequential rejection).  Restarts from scratch if
    max_tries draws do not suffice."""
    while True:
        pts: List[np.ndarray] = []
        tries = 0
        while len(pts) < n and tries < max_tries:
            p = rng.uniform(0.0, box, size=2)
            tries += 1
            if all(np.hypot(*(p - q)) >= dmin for q in pts):
                pts.append(p)
        if len(pts) == n:
            xyz = np.zeros((n, 3))
            xyz[:, :2] = np.array(pts)
            return xyz


# --------------------------------------------------------------------------- pulses
def pwl(knots_ns, values, t_ns: int) -> np.ndarray:
    """Piecewise-linear waveform through (knots_ns[k], values[k]) sampled at the integer
    times 0, 1, ..., t_ns (t_ns + 1 samples, both ends included)."""
    t = np.arange(t_ns + 1, dtype=np.float64)
    return np.interp(t, np.asarray(knots_ns, dtype=np.float64), np.asarray(values, dtype=np.float64))


def constant(value: float, t_ns: int) -> np.ndarray:
    return np.full(t_ns + 1, float(value))


def random_state(n_atoms: int, rng: np.random.Generator) -> np.ndarray:
    """Normalised complex Gaussian vector of length 2**n_atoms (complex128)."""
    dim = 1 << n_atoms
    v = rng.standard_normal(dim) + 1j * rng.standard_normal(dim)
    return (v / np.linalg.norm(v)).astype(np.complex128)


# --------------------------------------------------------------------------- workloads
@dataclasses.dataclass
class Workload:
    """One emulation job: register, sampled pulses and integrator options.

    omega/delta/phi are either shape [t_ns+1] (global drive) or [n_atoms, t_ns+1]
    (per-site drive).  phi may be None (zero phase)."""
    name: str
    xyz: np.ndarray
    c6: float
    omega: np.ndarray
    delta: np.ndarray
    phi: Optional[np.ndarray]
    t_ns: int
    dt_ns: int
    tol: float = 1e-10
    kmax: int = 30
    precision: str = "c128"
    n_shots: int = 0
    seed: int = 0

    @property
    def n_atoms(self) -> int:
        return int(self.xyz.shape[0])

    @property
    def n_steps(self) -> int:
        return self.t_ns // self.dt_ns


def sweep_pulses(t_ramp: int, t_plateau: int, omega_max: float, delta_max: float):
    """Adiabatic sweep: Omega 0 -> omega_max (ramp) -> plateau -> 0 (ramp); delta linear
    from -delta_max to +delta_max over the whole duration; phase zero."""
    t_ns = 2 * t_ramp + t_plateau
    omega = pwl([0, t_ramp, t_ramp + t_plateau, t_ns], [0.0, omega_max, omega_max, 0.0], t_ns)
    delta = pwl([0, t_ns], [-delta_max, delta_max], t_ns)
    return omega, delta, t_ns


def chain10() -> Workload:
    """10-atom chain, 5 um spacing, constant Omega = 2pi rad/us, delta = 0, 1 us at dt = 10 ns,
    1000 shots with seed 0."""
    t_ns = 1000
    return Workload("chain10", chain(10, 5.0), C6_RB, constant(TWO_PI, t_ns), constant(0.0, t_ns),
                    None, t_ns, 10, tol=1e-10, kmax=30, precision="c128", n_shots=1000, seed=0)


def square20() -> Workload:
    """4x5 square lattice, 6 um; 0.5 us ramps around a 3 us plateau at 2pi*2 rad/us, detuning
    swept -2pi*4 -> +2pi*4 rad/us over 4 us, dt = 10 ns."""
    omega, delta, t_ns = sweep_pulses(500, 3000, TWO_PI * 2.0, TWO_PI * 4.0)
    return Workload("square20", square_lattice(4, 5, 6.0), C6_RB, omega, delta, None, t_ns, 10)


def random27(seed: int = 0, n_atoms: int = 27, precision: str = "c128") -> Workload:
    """Random register in a 30x30 um box (5 um minimum distance); the sweep shape of
    square20 with Omega_max and delta_max drawn from U[2pi, 2pi*3] after the positions."""
    rng = np.random.default_rng(seed)
    xyz = random_register(n_atoms, 30.0, 5.0, rng)
    omax = rng.uniform(TWO_PI, TWO_PI * 3.0)
    dmax = rng.uniform(TWO_PI, TWO_PI * 3.0)
    omega, delta, t_ns = sweep_pulses(500, 3000, omax, dmax)
    tol = 1e-10 if precision == "c128" else 1e-7
    return Workload(f"random{n_atoms}", xyz, C6_RB, omega, delta, None, t_ns, 10, tol=tol,
                    kmax=48, precision=precision)


def triangular30(n_atoms: int = 30, precision: str = "c64") -> Workload:
    """5x6 triangular lattice, 5.5 um (first n_atoms atoms); quench at Omega = 2pi*2,
    delta = 2pi rad/us for 2 us, dt = 5 ns, Krylov dimension <= 20."""
    t_ns = 2000
    xyz = triangular_lattice(5, 6, 5.5)[:n_atoms]
    tol = 1e-10 if precision == "c128" else 1e-7
    return Workload(f"triangular{n_atoms}", xyz, C6_RB, constant(TWO_PI * 2.0, t_ns),
                    constant(TWO_PI, t_ns), None, t_ns, 5, tol=tol, kmax=20, precision=precision)


def serving_job(rng: np.random.Generator, n_min: int = 12, n_max: int = 24,
                dt_ns: int = 10, precision: str = "c64") -> Workload:
    """One job of the mixed-size serving stream: N ~ U{n_min..n_max}, random register as in
    random27, random piecewise-linear pulses with 4-8 segments (Omega knots in [0, 2pi*3],
    delta knots in [-2pi*5, 2pi*5]), duration 0.5-4 us rounded to 10 ns."""
    n = int(rng.integers(n_min, n_max + 1))
    xyz = random_register(n, 30.0, 5.0, rng)
    t_ns = int(10 * round(rng.uniform(0.5, 4.0) * 100))
    n_seg = int(rng.integers(4, 9))
    interior = np.sort(rng.choice(np.arange(1, t_ns), size=n_seg - 1, replace=False))
    knots = np.concatenate([[0], interior, [t_ns]])
    om = rng.uniform(0.0, TWO_PI * 3.0, size=n_seg + 1)
    de = rng.uniform(-TWO_PI * 5.0, TWO_PI * 5.0, size=n_seg + 1)
    tol = 1e-10 if precision == "c128" else 1e-7
    return Workload(f"job{n}", xyz, C6_RB, pwl(knots, om, t_ns), pwl(knots, de, t_ns), None,
                    t_ns, dt_ns, tol=tol, kmax=30, precision=precision)


def serving_stream(n_jobs: int, seed: int = 0, **kw) -> List[Workload]:
    """n_jobs independent jobs; each job draws from its own child of SeedSequence(seed)."""
    children = np.random.SeedSequence(seed).spawn(n_jobs)
    return [serving_job(np.random.default_rng(c), **kw) for c in children]


def poisson_arrivals(n_jobs: int, rate_per_s: float, seed: int = 1) -> np.ndarray:
    """Arrival times (s) of a Poisson process with the given rate."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate_per_s, size=n_jobs))
