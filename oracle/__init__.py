"""CPU oracle for Rydberg state-vector time evolution -- TEST INFRASTRUCTURE ONLY.

A plain, slow, obviously correct numpy (complex128 / float64) implementation of what the
emulator computes, written from the paper's statement of the method:

* ``model``       -- eq. (3) of Sec. II.A: the interaction matrix, the dense Hamiltonian from
                     Kronecker products, H|psi> by tensor-axis slicing, single rows of H|psi>;
                     the midpoint rule of Sec. III for the piecewise-constant pulse.
* ``evolve``      -- eq. (6): psi_{k+1} = exp(-i H_k dt) psi_k, by dense eigendecomposition
                     (small N) or by a Lanczos Krylov exponential with full
                     re-orthogonalisation (Sec. III.A).
* ``observables`` -- occupations <n_i>, correlators <n_i n_j>, bitstring sampling with a
                     SplitMix64 stream, fidelity and energy.
* ``lindblad``    -- the Lindblad master equation of Sec. III.A (open systems): the dense
                     Liouvillian with per-atom relaxation and dephasing, stepped by scipy's
                     matrix exponential.
* ``noise``       -- shot-to-shot parameter noise of Sec. III.A: each ensemble member's
                     perturbed drive amplitude, detunings and positions, drawn by a counter-
                     based SplitMix64 stream and the Box-Muller transform.
* ``gradient``    -- Sec. IV (the emulator is differentiable): derivatives of a weighted sum
                     of final occupations with respect to the Omega and delta samples, by the
                     adjoint method on the dense propagators of eq. (6).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py``
may import this package.  The HIP library never calls into it and shares no code with it;
the only shared module is the seeded input generator (``paper_2510_09813_amd.workloads``),
which holds no arithmetic of the method.

Parity status (what pins each public function in ``tests/test_oracle_pins.py``,
``tests/test_noise.py``, ``tests/test_lindblad_oracle.py`` and
``tests/test_gradient_oracle.py``):
* model.interaction_matrix, interaction_energy -- hand-computed pair energies and the
  all-excited state;
* model.midpoint_sample, step_parameters -- the midpoint indices of Sec. III on a ramp and
  dt^2 convergence of the midpoint scheme;
* model.dense_hamiltonian, diagonal_tensor, apply_hamiltonian, hamiltonian_row,
  atom_levels -- the single-atom Rabi closed form (amplitudes and phases), non-interacting
  product states with distinct drives (bit order), the hand-derived blockade Hamiltonian
  of two atoms and the sqrt(2), sqrt(3) collective frequencies, and agreement of the three
  formulations;
* evolve.evolve (dense and Lanczos), expm_lanczos -- the same closed forms, dense against
  Lanczos, norm and energy conservation, step splitting against scipy's expm, time
  reversal, sub-steps, the invariant subspace;
* observables.splitmix64, uniforms -- the generator's published reference outputs;
  occupations -- product states; correlations -- basis states, product states and the
  two-atom blockade state; sample -- brute force of its definition and a chi-square test;
  fidelity_loss -- global phase, orthogonal and near-parallel vectors; energy -- basis
  states and the two-level expectation value written out by hand.
* noise.splitmix64_at -- the published SplitMix64 outputs; gaussian -- mean, variance and a
  Kolmogorov-Smirnov test against the standard normal, no correlation between streams or
  neighbours; member, member_pulses -- zero noise is the identity, perturbations scale
  linearly with the standard deviations, the variate numbering.
* lindblad.evolve, liouvillian, jump_operators, occupations -- no dissipation equals the
  pure-state oracle, relaxation and dephasing closed forms, the optical Bloch steady state,
  trace, Hermiticity and positivity; apply_liouvillian, liouvillian_element -- the
  superoperator they restate, element by element.
* gradient.gradient, value -- the closed-form derivatives of the single-atom Rabi
  population, central finite differences of the pinned dense evolution, zero where no step
  reads a sample.
Every public function has a pin; none is "parity unpinned".
"""
from . import model, evolve, gradient, lindblad, noise, observables  # noqa: F401
