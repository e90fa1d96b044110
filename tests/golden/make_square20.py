"""Writes tests/golden/square20_final.npz: the 4x5 square-lattice adiabatic sweep (20 atoms,
6 um; Omega 0 -> 2pi*2 -> 0 rad/us with 0.5 us ramps around a 3 us plateau, delta swept
-2pi*4 -> +2pi*4 rad/us over 4 us, dt = 10 ns: all 400 steps of eq. 6 from |0...0>) computed
by the oracle's Krylov propagator (full re-orthogonalisation, tolerance 1e-13).

Only oracle/ and the seed-free input generator are called.  Stored:
  occ        <n_i> of the final state (float64, 20 values)
  norm       |psi_K|
  idx, amp   the amplitudes with |psi_b|^2 >= 1e-16 (uint32 indices, complex128 values);
             the dropped ones hold 9.2e-13 of the probability (stored as dropped_mass), so the
             infidelity computed against the stored vector is exact to ~1e-12, far below the
             1e-10 bar of the tests
  iters, substeps   the oracle's Krylov statistics (-1 when written from a cached state)

python tests/golden/make_square20.py [--cache PATH]   (about an hour on 8 host cores)
"""
import argparse
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import evolve, observables  # noqa: E402
from paper_2510_09813_amd import workloads as wl  # noqa: E402

CUT = 1e-16


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--cache", help="optional .npy path for the full final state")
    args = ap.parse_args()
    w = wl.square20()
    if args.cache and os.path.exists(args.cache):
        psi = np.load(args.cache)
        stats = {"iters": -1, "substeps": -1}
    else:
        psi = np.zeros(1 << w.n_atoms, dtype=np.complex128)
        psi[0] = 1.0
        stats = {"iters": 0, "substeps": 0}
        t0 = time.time()
        for first in range(0, w.n_steps, 20):  # progress every 20 steps
            psi, st = evolve.evolve_workload(w, psi0=psi, steps=20, first_step=first, tol=1e-13,
                                             return_stats=True)
            stats["iters"] += st["iters"]
            stats["substeps"] += st["substeps"]
            print(f"steps {first}..{first + 19} done, {time.time() - t0:.0f} s", flush=True)
        if args.cache:
            np.save(args.cache, psi)
    p = np.abs(psi) ** 2
    keep = np.flatnonzero(p >= CUT).astype(np.uint32)
    np.savez_compressed(os.path.join(HERE, "square20_final.npz"),
                        occ=observables.occupations(psi), norm=np.linalg.norm(psi),
                        idx=keep, amp=psi[keep], iters=stats["iters"],
                        substeps=stats["substeps"], dropped_mass=p.sum() - p[keep].sum())
    print(f"kept {keep.size} of {psi.size} amplitudes, dropped mass {p.sum() - p[keep].sum():.3e}")


if __name__ == "__main__":
    main()
