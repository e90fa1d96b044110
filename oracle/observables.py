"""Outputs of an emulation: occupations <n_i>, bitstring samples, fidelity and energy.

The sampler consumes a SplitMix64 stream (Steele, Lea & Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014), written here from its published definition:
the state advances by the odd constant 0x9E3779B97F4A7C15 and each output is the state
passed through the variant-13 finaliser (xor-shift 30, multiply, xor-shift 27, multiply,
xor-shift 31).  Shot s uses the s-th output x_s (s = 0, 1, ...) of the stream seeded with
``seed``, as the uniform u_s = (x_s >> 11) * 2^-53, and returns the smallest basis index b
whose cumulative probability exceeds u_s times the total; if rounding leaves no such b, the
largest b with nonzero probability.
"""
from __future__ import annotations

import numpy as np

MASK64 = (1 << 64) - 1
GOLDEN_GAMMA = 0x9E3779B97F4A7C15


def splitmix64(seed: int, count: int):
    """First ``count`` outputs of SplitMix64 seeded with ``seed`` (Python ints)."""
    state = seed & MASK64
    out = []
    for _ in range(count):
        state = (state + GOLDEN_GAMMA) & MASK64
        z = state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
        out.append(z ^ (z >> 31))
    return out


def uniforms(seed: int, count: int) -> np.ndarray:
    return np.array([(x >> 11) * 2.0 ** -53 for x in splitmix64(seed, count)], dtype=np.float64)


def probabilities(psi) -> np.ndarray:
    psi = np.asarray(psi, dtype=np.complex128)
    return psi.real ** 2 + psi.imag ** 2


def occupations(psi) -> np.ndarray:
    """<n_i> = sum_b |psi_b|^2 [level of atom i in b] / sum_b |psi_b|^2 (atom 0 = leading axis)."""
    p = probabilities(psi)
    n = int(round(np.log2(p.size)))
    t = p.reshape((2,) * n)
    total = p.sum()
    out = np.empty(n)
    for i in range(n):
        out[i] = np.take(t, 1, axis=i).sum() / total
    return out


def correlations(psi) -> np.ndarray:
    """<n_i n_j> = sum_b |psi_b|^2 [atom i excited][atom j excited] / sum_b |psi_b|^2, as an
    N x N matrix (diagonal: <n_i>)."""
    p = probabilities(psi)
    n = int(round(np.log2(p.size)))
    t = p.reshape((2,) * n)
    total = p.sum()
    out = np.empty((n, n))
    for i in range(n):
        ti = np.take(t, [1], axis=i)
        for j in range(n):
            out[i, j] = np.take(ti, [1], axis=j).sum() / total if j != i else ti.sum() / total
    return out


def sample(psi, seed: int, shots: int) -> np.ndarray:
    """Basis indices (uint64) of ``shots`` samples of |psi_b|^2, in shot order."""
    p = probabilities(psi)
    cdf = np.cumsum(p)
    total = cdf[-1]
    u = uniforms(seed, shots)
    out = np.empty(shots, dtype=np.uint64)
    nonzero = np.nonzero(p)[0]
    last = int(nonzero[-1]) if nonzero.size else p.size - 1
    for s in range(shots):
        b = int(np.searchsorted(cdf, u[s] * total, side="right"))
        out[s] = b if b < p.size else last
    return out


def fidelity_loss(a, b) -> float:
    """1 - |<a|b>|^2 for the normalised vectors, evaluated as || b - <a|b> a ||^2."""
    a = np.asarray(a, dtype=np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    a = a / np.linalg.norm(a)
    b = b / np.linalg.norm(b)
    r = b - np.vdot(a, b) * a
    return float(np.vdot(r, r).real)


def energy(psi, apply_h) -> float:
    psi = np.asarray(psi, dtype=np.complex128)
    return float(np.vdot(psi, apply_h(psi)).real / np.vdot(psi, psi).real)
