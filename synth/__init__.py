"""Seeded synthetic inputs for the volumetric deformation solve.

This package only *generates* inputs: canonical surface samples, their observed
targets and normals, sparse point pairs and the lattice description.  It holds
none of the solver's arithmetic (no trilinear weights, residuals, normal
equations or rotation fitting), so both the CPU oracle and the GPU library can
consume its output without sharing any computation.
"""

from .scenes import (  # noqa: F401
    Scene,
    LatticeSpec,
    make_config0,
    make_config1,
    make_tiny,
    make_rigid_scene,
    make_sequence_frame,
    make_identity_scene,
    random_rotation,
)
