"""FP64 CPU oracle for the VolumeDeform lattice solve (Innmann et al., 2016).

TEST INFRASTRUCTURE ONLY.  This package is the slow, plain reference that the
GPU library is checked against.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark may import it; the product path never calls
it and shares no code with it.

It follows the paper's statement of the problem:

* Sec. 4   -- the lattice, trilinear interpolation and the space deformation
             S(x) = sum_i alpha_i(x) t_i (global R, t fixed to the identity).
* Sec. 6   -- the energy, eqs. (1)-(4): point-to-plane, sparse point-to-point
             and the as-rigid-as-possible prior over the 6-neighbourhood.
* Sec. 7.1 -- the flip-flop: positions by the normal equations (solved exactly
             or by Jacobi-preconditioned CG), rotations by Procrustes/SVD.
* Sec. 7.2 -- the nested coarse-to-fine hierarchy with prolongation.

Every floating-point step is float64.  The Jacobian J is assembled explicitly
as a scipy sparse matrix, so A = J^T J and g = J^T r are library products of
the plain definitions.
"""

from .lattice import Grid, level_grids, trilinear, arap_edges  # noqa: F401
from .energy import (  # noqa: F401
    Constraints,
    prepare_constraints,
    assemble,
    residual_direct,
    energy_terms,
)
from .procrustes import cross_covariance, fit_rotations, rotation_step  # noqa: F401
from .solver import (  # noqa: F401
    jacobi_diag,
    pcg,
    position_step,
    inject,
    prolong,
    solve_frame,
    rest_state,
)
