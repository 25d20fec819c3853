"""FP64 CPU oracle for the many-k plane-wave Hamiltonian (test infrastructure).

This package is a plain, slow, obviously correct restatement of what the
library computes, written from the paper (Gong & Dal Corso, CPC 2024,
arXiv 2412.01695).  It exists only to check the library: it may be
imported, called or executed only by the tests, by the smoke check and by
the CPU-baseline leg of the benchmark.  Nothing in the library's product
path depends on it, and it shares no code, tables or helpers with the HIP
path; the only module both sides use is the seeded input generator
``paper_2412_01695_amd.synth``, which holds none of the method's arithmetic.

Modules
  basis        plane-wave sphere per k (Sec. 2.2.1, sphere inequality)
  dft          separable 3D DFT exactly as written (Sec. 4, Eqs. zfft, yfft,
               xfft and fwFFT), evaluated as explicit sums (DFT matrices)
  hamiltonian  dense H_k and two independent H|psi> routes (Sec. 2.2); the
               overlap S_k and S|psi> by Eqs. delta_eq and finals
  solvers      dense (generalized) eigenpairs, the paper's Davidson steps
               (Sec. 2.1, with S), the paper's preconditioned CG (Sec. 2.4)
               and the closed-form solution of the DFPT linear system
               (Sec. 2.3, with S)
  response     the perturbation from the k to the k+q sphere (dense and
               through the mesh), the right-hand side at q != 0 and the
               induced density of Eq. drho

Parity status: every function here is pinned by the CPU tests in
tests/test_oracle_*.py against closed forms, invariants, brute force or
independent library routines (see each module's docstring).  The paper
prints no physical values (only timings), so no pin uses a number from it.
"""
