"""MI355X (gfx950) implementation of the VolumeDeform lattice solve.

The solver and the warm-start network live in the HIP library ``libvd.so``
(C-ABI: ``include/vd.h``, ``include/vd_net.h``, ``include/vd_track.h``);
this package is its Python binding.  Importing it loads the library and fails
loudly if it has not been built.
"""

from ._lib import (  # noqa: F401
    EXPORTED,
    LIB_PATH,
    Batch,
    Lattice,
    Net,
    associate,
    batch_precision,
    rigid_pose,
    rigid_pose_noalloc,
    VDError,
    fit_rotations,
    sort_pairs,
    exclusive_scan,
    lib,
    strerror,
    VD_OK, VD_EINVAL, VD_ERANGE, VD_ENOMEM, VD_EHIP, VD_ESTATE,
    VD_REPORT_PCG_GUARD, VD_REPORT_POLAR_FP64, VD_REPORT_POLAR_KEEP, VD_REPORT_WARM_REJECTED,
    VD_REPORT_BARRIER_TIMEOUT,
)
