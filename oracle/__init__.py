"""FP64 CPU oracle for the HDG hot path -- TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously correct numpy/scipy code that computes what the GPU path
computes, written from the paper:
  condense.py  element Schur complements by one dense solve (Section 2.3, eq. 13-b/13-c)
               and local recovery (the equation after 13-c)
  assemble.py  face-block global matrix (Section 2.4, Section 4.2) and the
               uncondensed global system used as a brute-force check
  krylov.py    right-preconditioned FGMRES and left-preconditioned GMRES(m)
               (Section 3.1, Section 4.4), block-Jacobi (Sections 3.2, 4.5)
  poly.py      polynomial preconditioner: Arnoldi, harmonic Ritz values, Leja
               order, product-form apply (Sections 3.4, 4.7); Chebyshev smoother
  elements.py  element residuals and Jacobian blocks of scalar convection-diffusion
               models from the weak form (Sections 2.2, 4.1)
  elements_sys.py  the same for M-component models: linear elasticity and compressible
               Navier-Stokes (Section 2.1), flux derivatives by complex step
  newton.py    damped Newton with step halving on the residual norm (Section 4.4)
  dirk.py      stiffly accurate DIRK time stepping, one Newton solve per stage (Section 2.2)
  ilu_asm.py   additive Schwarz on multi-element subdomains with block ILU(0) local solves
               (Section 3.3's ASM with the incomplete factorisation the conclusions propose)

Only tests/, __graft_entry__.smoke() and bench.py's CPU-baseline leg may import
this package. It shares no code with the GPU library (paper_2512_13619_amd);
the two meet only at the seeded inputs produced by `workloads`.
"""
from . import condense, assemble, krylov, poly, elements, elements_sys, newton, dirk, ilu_asm  # noqa: F401
