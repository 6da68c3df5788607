"""CPU oracle for the LFA-tuned matrix-free elastic Helmholtz multigrid.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, float64 reference
written from the paper (Yovel & Treister, "LFA-tuned matrix-free multigrid
method for the elastic Helmholtz equation").  It exists to check the HIP
library: only the test-suite, the smoke check and the CPU-baseline leg of
the benchmark may import it.  The product path (the C-ABI library and its
Python binding) never calls into it and shares no code with it.

Contents (each module cites the passage it follows):
  grid       1D difference / averaging / transfer matrices, Kronecker helpers,
             DOF positions, absorbing-layer profile
  operator   the discrete mixed operator H^beta (eq. mixed-discretized),
             assembled as a sparse matrix (tiny grids) and applied
             matrix-free with the same 1D factors (any size)
  transfer   restriction R and prolongation P (Section 2.3 stencils)
  smoother   cell-wise Vanka relaxation, red-black and lexicographic,
             full and economic
  cycle      coarse hierarchy, two-grid / V-cycle (Algorithm 1), coarsest
             solves
  krylov     flexible GMRES(m) with right preconditioning
  kaczmarz   the paper's 3D coarsest-grid solver: Schur complement of the
             pressure, FGMRES preconditioned by hybrid (component-averaged,
             sub-region parallel) Kaczmarz sweeps
  adjoint    adjoint solve, misfit and parameter gradient
  symbols    closed-form Fourier symbols of the constant-coefficient blocks
  lfa        two-grid local Fourier analysis (Section 4): red-black full
             Vanka (the production smoother) and the paper's lexicographic
             economic Vanka
  lfa_tables the paper's LFA numbers (Table 1, Figures 3-4) and a 3D
             tuning table, printed by `python -m oracle.lfa_tables`

Parity status of every function is listed in the module headers; a function
without an independent pin says "parity unpinned".
"""
