"""Seeded synthetic inputs for the motion-compensation hot path.

This package is shared by the GPU path's tests and benchmark and by the FP64
oracle. It only *creates inputs*: calibrated projection matrices of a circular
cone-beam scan, ellipsoid phantoms, their analytic line integrals under
per-view rigid motion, the FDK pre-filter (cosine, Parker, ramp) that turns
line integrals into the filtered projections the backprojection consumes,
and smooth random motion. None of the backprojection, its Jacobian, the
losses or the motion model used by the solver lives here.

All randomness is ``numpy.random.default_rng(seed)``.
"""
from .geometry import ScanGeometry, VolumeGrid, projection_matrices, rigid_transform  # noqa: F401
from .configs import CONFIGS, make_case  # noqa: F401
