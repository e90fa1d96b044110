"""Time stepping of eq. (6): psi_{k+1} = exp(-i H_k dt) psi_k (Sec. III).

Two independent propagators, both reached through ``evolve``:
* method "dense"   -- exp(-i tau H_k) psi from numpy's Hermitian eigendecomposition of the
                      dense H_k (the plain definition; small N only).
* method "lanczos" -- ``expm_lanczos``, the Krylov (Lanczos) approximation of Sec. III.A:
                      build an orthonormal basis of span{psi, H psi, H^2 psi, ...} with the
                      three-term recurrence, re-orthogonalised against every earlier vector
                      (classical Gram-Schmidt, applied twice: all inner products against the
                      same vector, w <- w - V (V^H w)), then exp(-i tau T) e_1 from the
                      eigendecomposition of the small tridiagonal T.  Converged when the
                      a-posteriori estimate beta_m |[exp(-i tau T_m) e_1]_m| is at most tol.

Non-convergence within kmax vectors halves the step with the same H_k (exact, because
exp(-i H tau) = exp(-i H tau/2)^2), to a depth of 8.
"""
from __future__ import annotations

import numpy as np

from . import model


class NotConverged(RuntimeError):
    pass


def expm_lanczos(apply_h, psi: np.ndarray, tau: float, tol: float, kmax: int):
    """exp(-i tau H) psi.  Returns (result, converged, krylov_dim)."""
    nrm = np.linalg.norm(psi)
    if nrm == 0.0:
        return psi.copy(), True, 0
    basis = np.empty((kmax + 1, psi.size), dtype=np.complex128)  # row l = v_l
    basis[0] = psi / nrm
    alpha, beta = [], []
    for j in range(kmax):
        v = basis[j]
        w = apply_h(v)
        a = float(np.vdot(v, w).real)
        w = w - a * v
        if j > 0:
            w = w - beta[-1] * basis[j - 1]
        vs = basis[:j + 1]
        for _ in range(2):  # classical Gram-Schmidt, twice: c_l = <v_l, w> = conj(v_l . conj(w))
            w = w - vs.T @ np.conj(vs @ np.conj(w))
        b = float(np.linalg.norm(w))
        alpha.append(a)
        m = j + 1
        t = np.diag(alpha) + np.diag(beta, 1) + np.diag(beta, -1)
        lam, q = np.linalg.eigh(t)
        y = q @ (np.exp(-1j * lam * tau) * q[0, :])
        err = b * abs(y[m - 1]) * nrm
        if err <= tol or b == 0.0:
            return nrm * (basis[:m].T @ y), True, m
        beta.append(b)
        basis[j + 1] = w / b
    return None, False, kmax


def _propagate(apply_h, psi, tau, tol, kmax, depth, stats):
    res, ok, m = expm_lanczos(apply_h, psi, tau, tol, kmax)
    stats["iters"] += m
    if ok:
        return res
    if depth >= 8:
        raise NotConverged(f"Lanczos did not converge within {kmax} vectors")
    stats["substeps"] += 1
    half = _propagate(apply_h, psi, 0.5 * tau, tol, kmax, depth + 1, stats)
    return _propagate(apply_h, half, 0.5 * tau, tol, kmax, depth + 1, stats)


def _check_grid(n_samples: int, t_ns: int, dt_ns: int):
    if dt_ns <= 0 or t_ns < 0 or t_ns % dt_ns != 0:
        raise ValueError("duration must be a non-negative multiple of dt")
    if n_samples < t_ns + 1:
        raise ValueError("need samples at t = 0..T ns")


def _samples_len(x):
    return np.asarray(x).shape[-1]


def evolve(xyz, c6, omega, delta, phi, t_ns: int, dt_ns: int, psi0=None, method="lanczos",
           tol: float = 1e-13, kmax: int = 60, steps=None, first_step: int = 0,
           return_stats=False):
    """Evolve psi0 (default |0...0>) through steps 0..K-1 of eq. (6), K = t_ns / dt_ns.

    method = "dense" uses exp by eigendecomposition of each H_k (re-used while the
    midpoint parameters do not change); "lanczos" uses the Krylov exponential with full
    re-orthogonalisation.  The run covers steps first_step .. first_step + steps - 1 (all
    remaining steps when ``steps`` is None), starting from psi0 at step first_step."""
    n = int(np.asarray(xyz).shape[0])
    _check_grid(_samples_len(omega), t_ns, dt_ns)
    u = model.interaction_matrix(xyz, c6)
    psi = np.zeros(1 << n, dtype=np.complex128)
    if psi0 is None:
        psi[0] = 1.0
    else:
        psi[:] = np.asarray(psi0, dtype=np.complex128)
    total = t_ns // dt_ns
    n_steps = total - first_step if steps is None else min(steps, total - first_step)
    tau = dt_ns * 1e-3
    stats = {"iters": 0, "substeps": 0, "steps": n_steps}
    cache_key, cache = None, None
    for k in range(first_step, first_step + n_steps):
        om, de, ph = model.step_parameters(n, omega, delta, phi, dt_ns, k)
        if method == "dense":
            key = (om.tobytes(), de.tobytes(), ph.tobytes())
            if key != cache_key:
                h = model.dense_hamiltonian(u, om, de, ph)
                cache = np.linalg.eigh(h)
                cache_key = key
            w, v = cache
            psi = v @ (np.exp(-1j * w * tau) * (v.conj().T @ psi))
        elif method == "lanczos":
            apply_h = (lambda x, om=om, de=de, ph=ph: model.apply_hamiltonian(x, u, om, de, ph))
            psi = _propagate(apply_h, psi, tau, tol, kmax, 0, stats)
        else:
            raise ValueError(method)
    return (psi, stats) if return_stats else psi


def evolve_workload(w, method="lanczos", psi0=None, steps=None, first_step=0, **kw):
    """Convenience wrapper taking a ``workloads.Workload``-like object."""
    return evolve(w.xyz, w.c6, w.omega, w.delta, w.phi, w.t_ns, w.dt_ns, psi0=psi0,
                  method=method, steps=steps, first_step=first_step, **kw)
