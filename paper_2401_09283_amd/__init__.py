"""MI355X (gfx950) hot path of gradient-based rigid head-motion compensation in cone-beam CT.

Voxel-driven FDK backprojection under per-view rigid motion and its analytic
Jacobian-vector product with respect to the six rigid parameters of every view
(Thies et al., arXiv 2401.09283, Sec. II-B), as HIP kernels behind the C ABI of
include/gmc.h. ``gmc`` is the argument-marshalling binding, ``autograd`` the
torch.autograd.Function, ``solver`` the motion-estimation loop and ``serve``
the continuous-batching request loop.
"""
from ._lib import LIB_PATH, GmcError  # noqa: F401

__all__ = ["LIB_PATH", "GmcError"]
