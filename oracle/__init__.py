"""FP64 CPU oracle for the block-preconditioned FGMRES solve of the PFC system.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path imports, calls or
links this package: only the tests, the smoke check and the CPU-baseline leg
of the benchmark use it, to produce the values the HIP path is compared with.

It is written from the paper (Praetorius & Voigt, "Development and Analysis of
a Block-Preconditioner for the Phase-Field Crystal Equation"), plainly and in
float64, with numpy/scipy primitives (sparse matvec, dense LU, FFT, eig) as
the only library steps.  It shares no code, tables or helpers with the HIP
path; its inputs come from the seeded generators in `workloads`.

Modules
  simplex    exact integration of barycentric monomials on simplices, P1 geometry
  assembly   P1 mass M, stiffness K, psi^2-weighted mass and N(psi), load g(psi)
  pfc        the Rosenbrock stage matrix A^R, the operator F, stage right-hand
             sides, consistent initial values, the Ros3Pw step
  precond    the block preconditioner P_CH and its five-step apply
  krylov     Jacobi PCG, FGMRES(m) with modified Gram-Schmidt, full GMRES
  reference  dense LU and FFT-exact reference solves
  symbols    Fourier symbols, critical time step, asymptotic convergence factors

Pinning status of every function is listed in the module headers.
"""
