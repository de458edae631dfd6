"""Plain FP64 CPU oracle of the coarse-grid incremental pressure-projection
(CGP) time step.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
baseline leg of the benchmark may import this package.  It shares no code with
the HIP library (paper_1812_00185_amd) and imports nothing from it; both take
their inputs from the seeded generators in ``workloads``.

The oracle follows the paper step by step (Sect. 2.1, Eqs. 5-20; Sect. 2.2,
Eqs. 21-26; Sect. 2.3) with numpy / scipy.sparse as the only primitives:

  hierarchy.py   4:1 uniform refinement, injection R, linear prolongation P
  fem.py         P1 element matrices and global assembly (M, K, D, G, N)
  krylov.py      Jacobi-preconditioned CG and BiCGSTAB (the GPU's algorithms,
                 same stopping rule), written out plainly
  cgp.py         the six-step CGP time step
  mpnn.py        FP64 reference of the learned initial-guess network

Readings where the paper is silent are listed in each module's docstring.
"""
