"""CPU oracle for the MDLG hot path.

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the
benchmark's CPU-baseline leg.  The product path (paper_2101_01160_amd) never
imports, links or calls anything here, and nothing here imports it.

Modules
  lattice       D2Q49 velocity set and its numbering
  md            ctypes front-end of md_oracle.c (LJ forces, velocity Verlet,
                coarse-graining: binned and literal Eq.(n_i))
  closed_forms  measured f_eq from counts, Gaussian and Poisson-WSG
                equilibria, lambda from the moments (mpmath, 50 digits)
  mlp           FP64 reference of the surrogate network (forward, backward, Adam)
"""
