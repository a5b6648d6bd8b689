"""Seeded, synthetic inputs for the UGKS phase-space step.

This package builds only *inputs*: unstructured meshes stored as face lists
(cell volumes, centroids, face areas, unit normals, face centroids, boundary
tags), discrete velocity grids with quadrature weights, gas constants,
boundary-condition tables and initial conservative states.  It contains none
of the scheme's arithmetic (no Maxwellians, fluxes, gradients or updates), so
that the CPU oracle and the HIP library can both consume the same arrays while
sharing no code.

Nondimensionalisation (the paper fixes none): rho0 = 1, T0 = 1, length unit =
cavity / cube side or sphere radius, speed unit sqrt(2 R T0), hence R = 1/2 and
lambda0 = 1/(2 R T0) = 1.  Hard-sphere viscosity mu = mu_ref (T/T0)^0.5 with
mu_ref = (5 sqrt(pi) / 16) Kn.
"""

from .meshes import Mesh, quad_mesh, kuhn_tet_cube, cubed_sphere_shell, hex_box, cylinder_ogrid  # noqa: F401
from .velocity import (Velocity, midpoint_grid, gauss_hermite_grid, stretched_grid,  # noqa: F401
                       locally_refined_grid)
from .configs import (  # noqa: F401
    Gas, BC, Case, BC_INTERIOR, BC_WALL, BC_FARFIELD, BC_OUTFLOW,
    hard_sphere_mu_ref, cavity2d, couette2d, sod3d_tets, batch_cases,
    sphere_mach5, channel2d, make_case, uniform_W, maxwellian_box_case, cylinder2d,
)
