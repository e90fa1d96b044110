"""CPU oracle for Rydberg state-vector time evolution -- TEST INFRASTRUCTURE ONLY.

A plain, slow, obviously correct numpy (complex128 / float64) implementation of what the
emulator computes, written from the paper's statement of the method:

* ``model``       -- eq. (3) of Sec. II.A: the interaction matrix, the dense Hamiltonian from
                     Kronecker products, H|psi> by tensor-axis slicing, single rows of H|psi>;
                     the midpoint rule of Sec. III for the piecewise-constant pulse.
* ``evolve``      -- eq. (6): psi_{k+1} = exp(-i H_k dt) psi_k, by dense eigendecomposition
                     (small N) or by a Lanczos Krylov exponential with full
                     re-orthogonalisation (Sec. III.A).
* ``observables`` -- occupations <n_i>, bitstring sampling with a SplitMix64 stream,
                     fidelity and energy.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py``
may import this package.  The HIP library never calls into it and shares no code with it;
the only shared module is the seeded input generator (``paper_2510_09813_amd.workloads``),
which holds no arithmetic of the method.

Parity status: every public function is pinned by ``tests/test_oracle_pins.py`` against
closed forms (single-atom Rabi oscillation, blockaded two- and three-atom collective Rabi
frequencies, non-interacting product states), invariants (norm, energy, time reversal,
step splitting, mirror symmetry), brute force on tiny inputs and the published reference
outputs of SplitMix64.  No function is "parity unpinned".
"""
from . import model, evolve, observables  # noqa: F401
