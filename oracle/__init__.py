"""Plain, slow, FP64 CPU oracle for the FMM-BEM hot path.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
benchmark's CPU-baseline leg may import anything from this package; the
product path (the HIP library and its Python binding) never does.  It shares
no code with the HIP path: only the seeded input generators in ``synth`` serve
both.

Contents
  direct    -- the N-body sum the FMM approximates (plain definition), C and NumPy
  analytic  -- Born ion and Kirkwood sphere solvation energies (closed forms)
  tree      -- adaptive octree, Morton keys and the U/V/W/X interaction lists
  kifmm     -- the kernel-independent FMM, pass by pass, in FP64
  bem       -- dense P0 Galerkin boundary-element operators: direct, interior
               and exterior derivative formulations, reaction potential and
               solvation energy
  bem_p1    -- dense P1 (piecewise-linear) operators and the exterior
               derivative formulation on them, lumped-mass preconditioner
"""
