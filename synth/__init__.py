"""Seeded synthetic inputs for the slimLS tomography workloads.

This package is shared by the FP64 oracle (``oracle/``) and the GPU path
(``paper_1912_07962_amd``).  It holds no arithmetic of the reconstruction
method itself: it draws random ellipse / ellipsoid phantoms, samples them at
pixel centres, evaluates their exact parallel-beam line integrals (closed
form), adds Gaussian noise at a stated relative level, and draws block
schedules.  The scan geometry it uses to place the rays is the data
acquisition convention, restated independently by each consumer.
"""
from .phantom import (  # noqa: F401
    Ellipse,
    random_ellipses,
    random_ellipsoids,
    ellipsoid_slice,
    rasterize,
    analytic_sinogram,
    add_noise,
    make_slice_problem,
    make_volume_problem,
    volume_slice,
    schedule,
    scan_geometry,
    n_rays_for,
)
from .phantom3d import (  # noqa: F401
    Ellipsoid3,
    random_directions,
    detector_basis,
    random_ellipsoids3,
    rasterize3,
    line_integrals,
    make_problem3,
)
from .configs import CONFIGS, get_config, warmstart_sample  # noqa: F401
