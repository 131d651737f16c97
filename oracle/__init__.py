"""FP64 CPU oracle for the fast spectral Boltzmann collision operator.

TEST INFRASTRUCTURE ONLY.  This package is the slow, plain reference that the
HIP path is checked against.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import it; the product path never does, and
this package imports nothing from the product package.

What it computes follows Appendix A of the paper (the Fourier-Galerkin spectral
method with the Carleman representation and the separable angular quadrature),
Section 2.1 (exact-shift transport, explicit Euler collision step, eq.
disc_relax), Section 2.2.1 (BGK relaxation), Section 3 (particle masses,
macroscopic moments, eq. DM_update) and Section 4.1 (the sequential FKS step).

Modules
  grid        velocity grid, Fourier modes, Fourier coefficients and synthesis
  tables      phi_R, psi_R, angular/radial quadrature, separable kernel terms
  collide     O-direct (the O(N^6) sum of eq. CF1) and O-fast (padded FFTs)
  conserve    moments and the FP64 conservation projection
  transport   generic-cell offsets, the exact periodic shift, eq. DM_update
  bgk         macroscopic variables (ToPrimitive), Maxwellians, the BGK operator
  integrators explicit Euler, Heun (RK2) and the exponential (stiff) step; FKS steps
  bkw         closed-form Bobylev-Krook-Wu solution for Maxwell molecules
  sigma_form  brute-force quadrature of the collision integral in sigma form
  mlp         FP64 MLP with hand-written backward pass (surrogate reference)
"""

from .grid import Grid, make_grid  # noqa: F401
from .tables import Plan, make_plan  # noqa: F401
