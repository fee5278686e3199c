"""CPU oracle for the red-black Shamir domain-wall path (TEST INFRASTRUCTURE).

This package is a plain, slow, FP64 NumPy statement of what the paper's
method computes.  It exists only to check the HIP implementation: the
tests, the package's ``smoke()`` self-check and the benchmark's CPU
baseline leg are the only code that may import it.  The product path never
calls into it and shares no code, table or layout with it.

Conventions (the paper leaves them open; see each module):

* natural layout ``psi[Ls][T][Z][Y][X][spin][colour]``, links
  ``U[T][Z][Y][X][mu][a][b]`` with mu = x, y, z, t; periodic 4D boundaries;
* chiral gamma basis with gamma5 = diag(1, 1, -1, -1);
* half-lattice (checkerboard) fields are full-lattice arrays that are zero
  on the other 4D parity, parity = (x + y + z + t) mod 2, even = 0.

Modules:

* ``lattice`` -- gamma matrices, D_hop, D_W, M5D, D_DW, the Schur blocks,
  M_pc, its adjoint and the normal operator, the red-black solve
  (Chiral Fermion Actions section; Results section, red-black CGNR).
* ``krylov``  -- CG, power method, Chebyshev filter and recursive series,
  Gram-Schmidt (Spectrum section; Chebyshev smoothers and Deflation basis
  setup sections).
* ``force``   -- the pseudofermion action and its link gradient
  (HMC usage in the Conclusions; derived, see the module).
* ``codec``   -- the FP16 + per-site scale storage emulation.
"""

from . import lattice, krylov, force, codec  # noqa: F401
