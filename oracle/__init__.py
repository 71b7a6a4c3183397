"""Independent FP64 CPU oracle for the shift-and-invert Jacobi-Davidson hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product package imports, links or runs
anything under this directory; only the test-suite, the smoke check and the CPU
baseline leg of the benchmark do.  It shares no code, tables or helpers with the
HIP path: the one thing both sides have in common is the published SplitMix64
definition, which each side implements on its own.

What it computes (Schenk, Bollhoefer & Roemer, "On large scale diagonalization
techniques for the Anderson model of localization"):

* ``generator``  -- the box-distributed random diagonal of the Anderson model
  (section 3, eq. (eigenequation)), drawn from SplitMix64.
* ``lattice``    -- the Anderson Hamiltonian on the periodic L^3 lattice as a CSR
  matrix and its matrix-vector product (section 3, eq. (eigenequation)).
* ``jacobi``     -- dense cyclic Jacobi eigensolver (textbook method), the
  brute-force path for tiny lattices.
* ``ldlt``       -- exact sparse LDL^T of A - tau I by nested dissection with
  Bunch-Kaufman pivoting inside dense fronts; Sylvester inertia.
* ``lanczos``    -- shift-and-invert Lanczos with full reorthogonalisation
  (section 4.1; the recurrence of eq. (lanczos) applied to (A - sigma I)^{-1}).
* ``eig``        -- the result definition: the k eigenpairs nearest sigma, the
  clean-lattice closed form, the inertia certificate.

Every function is pinned by tests under ``tests/test_oracle_*.py`` against facts
the paper or mathematics fix (closed forms, invariants, brute force).
"""
