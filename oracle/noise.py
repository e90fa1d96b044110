"""Shot-to-shot parameter noise (Sec. III.A: open-system effects modelled by varying the
Hamiltonian's parameters from shot to shot) -- TEST INFRASTRUCTURE ONLY.

The paper names the mechanism but not its distributions; the reading used here: every
ensemble member (shot) s draws independent standard normal variates g and perturbs
  * the drive amplitude by one factor shared by all atoms: Omega_i(t) -> (1 + s_Omega g) Omega_i(t)
    (shot-to-shot laser intensity),
  * each atom's detuning by a constant offset: delta_i(t) -> delta_i(t) + s_delta g
    (Doppler shift of a thermal atom),
  * each atom's position on each axis: r_i -> r_i + s_r (g, g, g)
    (position spread of the trap),
and is then evolved exactly as a noiseless job (eq. 6).

Variates: member s uses 4N + 1 of them, numbered j = 0 (amplitude), 1 + i (detuning of atom
i), 1 + N + 3 i + a (axis a of atom i).  Variate number c = s (4N + 1) + j is one Box-Muller
transform (Box & Muller 1958) of two uniforms taken from the SplitMix64 stream seeded with
the noise seed (Steele, Lea & Flood 2014), outputs 2c and 2c + 1:
    u1 = ((x_2c >> 11) + 1) 2^-53  in (0, 1],   u2 = (x_{2c+1} >> 11) 2^-53  in [0, 1),
    g  = sqrt(-2 ln u1) cos(2 pi u2).
The k-th output of the stream is the finaliser applied to seed + (k + 1) * 0x9E3779B97F4A7C15
(mod 2^64): the generator is counter based, so any member is drawn without the others.
"""
from __future__ import annotations

import math

import numpy as np

MASK64 = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15


def splitmix64_at(seed: int, k: int) -> int:
    """k-th output (k = 0, 1, ...) of SplitMix64 seeded with seed."""
    z = (seed + (k + 1) * GAMMA) & MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def gaussian(seed: int, c: int) -> float:
    """Standard normal variate number c of the noise stream."""
    u1 = ((splitmix64_at(seed, 2 * c) >> 11) + 1) * 2.0 ** -53
    u2 = (splitmix64_at(seed, 2 * c + 1) >> 11) * 2.0 ** -53
    return math.sqrt(-2.0 * math.log(u1)) * math.cos(2.0 * math.pi * u2)


def member(seed: int, s: int, n_atoms: int, sigma_omega: float, sigma_delta: float,
           sigma_pos: float, xyz):
    """Perturbation of ensemble member s: (omega factor, delta offsets [N], positions [N, 3])."""
    per = 4 * n_atoms + 1
    g = [gaussian(seed, s * per + j) for j in range(per)]
    factor = 1.0 + sigma_omega * g[0]
    offsets = np.array([sigma_delta * g[1 + i] for i in range(n_atoms)])
    disp = np.array([[sigma_pos * g[1 + n_atoms + 3 * i + a] for a in range(3)]
                     for i in range(n_atoms)])
    return factor, offsets, np.asarray(xyz, dtype=np.float64) + disp


def member_pulses(omega, delta, factor, offsets):
    """Per-site sample arrays [N, T+1] of a member: scaled drive, offset detuning."""
    n = offsets.size
    om = np.broadcast_to(np.asarray(omega, dtype=np.float64), (n, np.asarray(omega).shape[-1]))
    de = np.broadcast_to(np.asarray(delta, dtype=np.float64), (n, np.asarray(delta).shape[-1]))
    return factor * om, de + offsets[:, None]
