"""FP64 CPU oracle of the modified-Ehrenfest step.  TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import or call anything in this package.  The GPU library never calls it,
shares no code with it, and neither imports the other.

The oracle is a plain, slow, deliberately unblocked NumPy implementation in
float64/complex128 of what one step of the method computes, written from the
paper (Andrade et al., "Modified Ehrenfest formalism for efficient large-scale
ab initio molecular dynamics", arXiv:0812.2801):

* ``grid``      -- periodic real-space grid, 8th-order finite-difference
                   Laplacian (sec. 5, real-space finite differences).
* ``potentials``-- local ionic potential by structure factor (sec. 5.2,
                   eq. ionicpotential), Hartree by FFT, Slater exchange,
                   Ewald ion-ion energy and forces (the ion-ion term of
                   eq. E_KS).
* ``kb``        -- Gaussian s-channel Kleinman-Bylander projector.
* ``model``     -- the Hamiltonian of eq. new_EoM(a), its energy eq. E_KS
                   and forces -grad_R E_KS (eq. new_EoM(b)).
* ``dynamics``  -- fourth-order Taylor exponential and the AETRS propagator
                   (sec. 5.1, eq. aetrs), velocity Verlet for the ions, the
                   density eq. density.
* ``adjoint``   -- reverse-mode derivative of an AETRS trajectory.
* ``cp``        -- the Car-Parrinello comparison scheme (eq. L_CP, eq. EoM_CP)
                   with RATTLE / velocity Verlet for the orbitals.
* ``stability`` -- time-step limits of the Taylor exponential and of CP.
* ``finite``    -- the finite box (union of atom-centred spheres, zero
                   boundary condition) with free-space Hartree and ionic
                   potentials.
* ``toy``       -- the two-band toy model (eq. L_toy) by RK4: the modified
                   Ehrenfest, CP and gsBO motions, d_R, d_F, Delta t_max.

Conventions: arrays of grid functions have axes (z, y, x) with x fastest;
grid point (ix, iy, iz) sits at r = h*(ix, iy, iz); the inner product is the
grid quadrature h^3 sum conj(a) b.
"""
from .grid import Grid  # noqa: F401
from .model import Model  # noqa: F401
from . import dynamics, potentials, kb, adjoint, cp, toy, finite  # noqa: F401
