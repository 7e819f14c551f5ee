"""Plain FP64 CPU oracle for the alchemical-window hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link anything under ``oracle/``; only the tests, the smoke check and the
benchmark's CPU-baseline leg use it.  It shares no code with the HIP path:
brute-force O(N^2) pair sums, direct Ewald, an independently written FP64
smooth PME (numpy FFTs), bonded and Boresch terms, a Langevin-middle step with
iterative SHAKE constraints and a Philox noise stream written from its
published definition, the cross-lambda reduced potentials, a plain
self-consistent MBAR, Metropolis replica exchange between neighbouring
windows, the segmented free-energy assembly with the analytic restraint
term, and the Monte Carlo barostat's volume move.

Citations name the paper's sections:
  * "Double annihilation protocol" -- Beutler softcore form, Lorentz-Berthelot
    mixing, lambda_ij = min(lambda_i, lambda_j), alpha = 0.5, p = 1, ligand
    charges scaled linearly to zero;
  * "Restraints" -- Boresch distance/angle/dihedral set and its two energy
    forms;
  * "Simulation protocol" -- Langevin-middle integration (2 fs, friction
    0.5/ps), rigid TIP3P water, MBAR over the windows of a segment;
  * appendix B -- 1.0 nm PME real-space and vdW cutoffs.
Where the paper names a method without printing it (PME, SETTLE/SHAKE, MBAR,
Philox), the oracle follows the method's own publication.

Pinned by tests in ``tests/test_oracle_*.py`` (Madelung and Wigner constants,
alpha independence, lambda end points, finite differences, Newton's third
law, NVE drift, harmonic-oscillator statistics, analytic harmonic free
energies, BAR and EXP reductions, Philox known-answer vectors, the exact
stationary distribution of replica exchange over permutations, the analytic
restraint term against quadrature of the restrained partition function, the
ideal-gas isothermal-isobaric volume law and the gas constant at standard
conditions for the barostat).
"""
