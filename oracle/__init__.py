"""FP64 CPU oracle for the VoxCap capacitance path -- TEST INFRASTRUCTURE ONLY.

Only tests/, the smoke check of the entry module and the CPU-baseline leg of the
bench may import this package.  The product library never calls it, and this
package imports nothing from the product (they share only the seeded scene
generators in `scenes/`).

What it computes is the plain definition of the paper's method (Sec. II.A):

* panels: every voxel face between a conductor and a non-conductor, and every
  face between two non-conductors of different permittivity (Sec. II.A, eq. 3);
* the Galerkin integrals of eq. (5) and eq. (6) evaluated by quadrature of the
  exact inner potential of a uniformly charged square (integrals.py);
* the dense system of eq. (4) with the jump term of eq. (7), solved by LU;
* the capacitance matrix of eq. (8) with the free-charge scaling of Sec. II.A;
* the adjoint derivative of C with respect to block permittivities;
* the Tucker format of eq. (13) by its definition (tucker.py);
* the Toeplitz octants of App. B, compressed over a largest grid and restored for a
  smaller one (toeplitz.py, Sec. II.C).

Dimensionless units: voxel edge 1 and 4*pi*eps0 = 1 (scaling of App. C).
"""
from . import panels, integrals, dense, tucker, toeplitz  # noqa: F401
from .panels import panelize, GeometryError  # noqa: F401
from .dense import (assemble, rhs, solve_capacitance, mvp, capacitance_gradient,  # noqa: F401
                    capacitance_from_rho, free_charge_weights, EPS0)
