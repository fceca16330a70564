"""CPU FP64 oracle for the ROM-based inexact FETI-DP method (test infrastructure).

This package is a plain, slow, direct transcription of the method into
NumPy/SciPy in float64.  It exists only to check the GPU library: it is
imported by the tests, by the smoke check and by the CPU-baseline leg of the
benchmark, and by nothing else.  It shares no code with the GPU library; the
only common module is `latticegen`, which generates problem data.

Modules (paper: Hirschler, Bouclier, Antolin, Buffa, "Reduced Order Modeling
based Inexact FETI-DP solver for lattice structures"):

  bspline    quadratic B-spline basis (Cox-de Boor) and Gauss rules   (Sec. 2.2.1 eq. 6)
  assembly   pulled-back material tensor and cell stiffness, loads   (eqs. 5, 52-54)
  dd         dof partition, jump operator B, weights D, primal map    (eqs. 12-18, 30)
  greedy     principal-cell selection and affine coordinates          (Alg. 4, eqs. 55-56)
  rom        principal bank, coefficient systems, ROM local operators (eqs. 22, 27-30, 39-43)
  operators  F̊, M̊_D^-1, Ů, Ůᵀ, K̊^-ROM, true saddle operator           (eqs. 16, 44-49, Algs. 1-3)
  krylov     PCG and flexible GMRES                                   (Sec. 2.3, 3.2.3)
  direct     conforming assembly + direct Cholesky (plain definition of the solution)
  fetidp     exact standard FETI-DP on small lattices                 (eqs. 20-31)
  gradient   compliance and its width gradient

Parity status of each function is stated in its module header.
"""
from .model import Model  # noqa: F401
