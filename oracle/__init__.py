"""CPU oracle for the folded-spectrum plane-wave eigensolve (test infrastructure).

This package is a plain, slow, FP64 reference of what the GPU library computes.
It is test infrastructure only: the test-suite, the smoke check and the
CPU-baseline leg of the benchmark may import it; the library never does, and
this package imports nothing from the library.  Arrays come in as plain numpy
inputs (cell, grid, atom centres, potential samples, KB strengths, start
vectors) and every derived quantity -- basis, kinetic energies, potential
Fourier coefficients, projectors, the Hamiltonian, eigenpairs, the folded CG --
is computed here from its definition.

Modules
  basis        plane-wave sphere and kinetic energies
  hamiltonian  dense H and matrix-free H psi (numpy FFT)
  eigen        nearest-to-E selection, residuals, Cholesky orthonormalisation
  precond      Teter-Payne-Allan and the paper's M(G) diagonal preconditioners
  fsm_cg       folded-spectrum preconditioned CG on A = (H - E)^2
  mlp          the per-shell preconditioner network: forward, backward, loss
  linsolve     spectral closed form and PCG for (H - E)^2 psi = (H - E) w
  chebfd       Chebyshev window filter p(H) and ChebFD steps
  kinterp      wave-function interpolation between two k-points

Every public function names the passage of the paper (or the textbook
definition) it follows.  Pins live in tests/test_oracle_*.py.
"""
