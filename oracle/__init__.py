"""FP64 CPU oracle for symmetry-masked autoregressive NQS VMC (arXiv 2310.04166).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or link
this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
path; both read the same seeded inputs from ``synth``.

It computes every quantity of the hot path by the plainest route, and by a
route different from the GPU's wherever one exists.  Sections are named by the
paper's headings:

* ``hamiltonian``  matrix elements of the second-quantised Hamiltonian
                   ("System description", the H_SQ equation) by literal
                   creation/annihilation-operator application and by
                   Slater-Condon rules - not by Pauli strings.
* ``sector``       the symmetry sector, and physicality by the memoised
                   recursion of Algorithm 1 ("Physicality evaluation
                   algorithm") over qubits, with the particle-number and S_z
                   symmetries of Appendix A.
* ``model``        the amplitude networks (the ANQS product-rule equation;
                   Appendix B) with Mask-Unphysical conditionals ("Pruning
                   strategies").
* ``vmc``          local energy, counts-weighted energy estimator and VMC
                   gradient ("Variational Monte Carlo": the local-energy,
                   energy-estimator and gradient equations).
* ``sampler``      autoregressive statistics sampling with pruning
                   ("Autoregressive statistics sampling", "Pruning
                   strategies"), Philox4x32-10 and exact binomial draws.
* ``ed``           exact diagonalisation inside the sector.

Pins for every function live in ``tests/test_oracle_*.py``.
"""
