"""Python binding of libgmc: the C entry points under the same names, taking torch tensors.

Argument marshalling only. Every function checks device, dtype, contiguity and
shape, passes raw device pointers and the current HIP stream, and raises
``GmcError`` on a non-zero status. All arithmetic of the hot path runs in the
HIP kernels of libgmc.so.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import FLAG_FORCE_EDGE, FLAG_FORCE_GLOBAL, GRAD, WORK_PREPARED, WEIGHT, Geometry, GmcError, Work, check, lib  # noqa: F401


def _stream(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t, dtype, shape=None, name="tensor", allow_none=False):
    if t is None:
        if allow_none:
            return None
        raise ValueError("%s is required" % name)
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a CUDA (HIP) tensor" % name)
    if t.dtype != dtype:
        raise TypeError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError("%s must have shape %s, got %s" % (name, tuple(shape), tuple(t.shape)))
    return ctypes.c_void_p(t.data_ptr())


def make_geometry(n_views, det_w, det_h, shape, voxel_mm, origin_mm, weighting="fdk", grad_mode="paper",
                  flags=0) -> Geometry:
    g = Geometry()
    g.n_views, g.det_w, g.det_h = int(n_views), int(det_w), int(det_h)
    g.nx, g.ny, g.nz = (int(s) for s in shape)
    g.voxel_mm = (ctypes.c_double * 3)(*[float(v) for v in voxel_mm])
    g.origin_mm = (ctypes.c_double * 3)(*[float(v) for v in origin_mm])
    g.weighting = WEIGHT[weighting] if isinstance(weighting, str) else int(weighting)
    g.grad_mode = GRAD[grad_mode] if isinstance(grad_mode, str) else int(grad_mode)
    g.flags = int(flags)
    return g


class Plan:
    """Owns a gmc_plan (host object)."""

    def __init__(self, geometry: Geometry, P_nominal=None):
        self.geometry = geometry
        h = ctypes.c_void_p()
        Pn = None
        if P_nominal is not None:
            self._Pn = np.ascontiguousarray(np.asarray(P_nominal, dtype=np.float64).reshape(geometry.n_views, 3, 4))
            Pn = self._Pn.ctypes.data_as(ctypes.c_void_p)
        check(lib().gmc_plan_create(ctypes.byref(geometry), Pn, ctypes.byref(h)), "gmc_plan_create")
        self.handle = h

    @property
    def workspace_bytes(self) -> int:
        return int(lib().gmc_workspace_bytes(self.handle))

    def info(self) -> dict:
        out = (ctypes.c_int64 * 8)()
        check(lib().gmc_plan_info(self.handle, out), "gmc_plan_info")
        return dict(brick=(out[0], out[1], out[2]), tile_pitch=out[3], tile_rows=out[4], n_bricks=out[5],
                    view_chunks=(out[6], out[7]))

    @property
    def vol_shape(self):
        g = self.geometry
        return (g.nx, g.ny, g.nz)

    @property
    def proj_shape(self):
        g = self.geometry
        return (g.n_views, g.det_h, g.det_w)

    def new_workspace(self, device="cuda"):
        return torch.empty(self.workspace_bytes, dtype=torch.uint8, device=device)

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            lib().gmc_plan_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _ws(plan: Plan, workspace):
    if workspace is None or workspace.dtype != torch.uint8 or workspace.numel() < plan.workspace_bytes:
        raise ValueError("workspace must be a uint8 CUDA tensor of at least %d bytes" % plan.workspace_bytes)
    return _ptr(workspace, torch.uint8, name="workspace")


# ----------------------------------------------------------------- entry points, same names as the C ABI

def gmc_compose(plan: Plan, theta, P, Phat, dPhat=None, stream=None):
    n = plan.geometry.n_views
    check(lib().gmc_compose(plan.handle, _ptr(theta, torch.float64, (n, 6), "theta"),
                            _ptr(P, torch.float64, (n, 3, 4), "P"), _ptr(Phat, torch.float64, (n, 3, 4), "Phat"),
                            _ptr(dPhat, torch.float64, (n, 6, 3, 4), "dPhat", True), _stream(stream)), "gmc_compose")


def gmc_backproject(plan: Plan, proj, P, theta, vol, workspace, stream=None):
    n = plan.geometry.n_views
    check(lib().gmc_backproject(plan.handle, _ptr(proj, torch.float32, plan.proj_shape, "proj"),
                                _ptr(P, torch.float64, (n, 3, 4), "P"), _ptr(theta, torch.float64, (n, 6), "theta"),
                                _ptr(vol, torch.float32, plan.vol_shape, "vol"), _ws(plan, workspace),
                                _stream(stream)), "gmc_backproject")


def gmc_backproject_vjp(plan: Plan, proj, P, theta, grad_vol, grad_theta, grad_P, workspace, stream=None):
    n = plan.geometry.n_views
    check(lib().gmc_backproject_vjp(plan.handle, _ptr(proj, torch.float32, plan.proj_shape, "proj"),
                                    _ptr(P, torch.float64, (n, 3, 4), "P"),
                                    _ptr(theta, torch.float64, (n, 6), "theta"),
                                    _ptr(grad_vol, torch.float32, plan.vol_shape, "grad_vol"),
                                    _ptr(grad_theta, torch.float64, (n, 6), "grad_theta"),
                                    _ptr(grad_P, torch.float64, (n, 3, 4), "grad_P", True), _ws(plan, workspace),
                                    _stream(stream)), "gmc_backproject_vjp")


def gmc_backproject_vjp_noalloc(plan: Plan, proj, P, theta, grad_vol, grad_theta, grad_P=None, geometry_flag=None,
                                stream=None):
    n = plan.geometry.n_views
    check(lib().gmc_backproject_vjp_noalloc(plan.handle, _ptr(proj, torch.float32, plan.proj_shape, "proj"),
                                            _ptr(P, torch.float64, (n, 3, 4), "P"),
                                            _ptr(theta, torch.float64, (n, 6), "theta"),
                                            _ptr(grad_vol, torch.float32, plan.vol_shape, "grad_vol"),
                                            _ptr(grad_theta, torch.float64, (n, 6), "grad_theta"),
                                            _ptr(grad_P, torch.float64, (n, 3, 4), "grad_P", True),
                                            _ptr(geometry_flag, torch.int32, (1,), "geometry_flag", True),
                                            _stream(stream)), "gmc_backproject_vjp_noalloc")


def gmc_prepare(plan: Plan, P, theta, with_deriv, workspace, stream=None):
    n = plan.geometry.n_views
    check(lib().gmc_prepare(plan.handle, _ptr(P, torch.float64, (n, 3, 4), "P"),
                            _ptr(theta, torch.float64, (n, 6), "theta"), int(bool(with_deriv)), _ws(plan, workspace),
                            _stream(stream)), "gmc_prepare")


def gmc_bp_forward(plan: Plan, proj, vol, workspace, stream=None):
    check(lib().gmc_bp_forward(plan.handle, _ptr(proj, torch.float32, plan.proj_shape, "proj"),
                               _ptr(vol, torch.float32, plan.vol_shape, "vol"), _ws(plan, workspace), _stream(stream)),
          "gmc_bp_forward")


def gmc_bp_vjp(plan: Plan, proj, grad_vol, workspace, stream=None):
    check(lib().gmc_bp_vjp(plan.handle, _ptr(proj, torch.float32, plan.proj_shape, "proj"),
                           _ptr(grad_vol, torch.float32, plan.vol_shape, "grad_vol"), _ws(plan, workspace),
                           _stream(stream)), "gmc_bp_vjp")


def gmc_bp_vjp_finish(plan: Plan, grad_theta, grad_P, workspace, stream=None):
    n = plan.geometry.n_views
    check(lib().gmc_bp_vjp_finish(plan.handle, _ptr(grad_theta, torch.float64, (n, 6), "grad_theta"),
                                  _ptr(grad_P, torch.float64, (n, 3, 4), "grad_P", True), _ws(plan, workspace),
                                  _stream(stream)), "gmc_bp_vjp_finish")


def gmc_loss_sumsq_grad(plan: Plan, vol, grad_vol, loss, workspace, stream=None):
    check(lib().gmc_loss_sumsq_grad(plan.handle, _ptr(vol, torch.float32, plan.vol_shape, "vol"),
                                    _ptr(grad_vol, torch.float32, plan.vol_shape, "grad_vol"),
                                    _ptr(loss, torch.float64, (1,), "loss"), _ws(plan, workspace), _stream(stream)),
          "gmc_loss_sumsq_grad")


def gmc_loss_entropy_tv(plan: Plan, vol, lam, lo, hi, eps, grad_vol, loss, workspace, stream=None):
    check(lib().gmc_loss_entropy_tv(plan.handle, _ptr(vol, torch.float32, plan.vol_shape, "vol"), float(lam),
                                    float(lo), float(hi), float(eps),
                                    _ptr(grad_vol, torch.float32, plan.vol_shape, "grad_vol"),
                                    _ptr(loss, torch.float64, (5,), "loss"), _ws(plan, workspace), _stream(stream)),
          "gmc_loss_entropy_tv")


def gmc_bspline_theta(n_views, n_nodes, coeffs, theta, stream=None):
    check(lib().gmc_bspline_theta(int(n_views), int(n_nodes), _ptr(coeffs, torch.float64, (6, n_nodes), "coeffs"),
                                  _ptr(theta, torch.float64, (n_views, 6), "theta"), _stream(stream)),
          "gmc_bspline_theta")


def gmc_bspline_grad(n_views, n_nodes, grad_theta, grad_coeffs, stream=None):
    check(lib().gmc_bspline_grad(int(n_views), int(n_nodes),
                                 _ptr(grad_theta, torch.float64, (n_views, 6), "grad_theta"),
                                 _ptr(grad_coeffs, torch.float64, (6, n_nodes), "grad_coeffs"), _stream(stream)),
          "gmc_bspline_grad")


def gmc_forward_project(plan: Plan, vol, P, theta, proj_out, workspace, stream=None):
    n = plan.geometry.n_views
    check(lib().gmc_forward_project(plan.handle, _ptr(vol, torch.float32, plan.vol_shape, "vol"),
                                    _ptr(P, torch.float64, (n, 3, 4), "P"), _ptr(theta, torch.float64, (n, 6), "theta"),
                                    _ptr(proj_out, torch.float32, plan.proj_shape, "proj_out"), _ws(plan, workspace),
                                    _stream(stream)), "gmc_forward_project")


def gmc_forward_project_parts(plan: Plan, vol, labels, n_parts, P, theta, proj_out, workspace, stream=None):
    n = plan.geometry.n_views
    check(lib().gmc_forward_project_parts(plan.handle, _ptr(vol, torch.float32, plan.vol_shape, "vol"),
                                          _ptr(labels, torch.uint8, plan.vol_shape, "labels", allow_none=n_parts == 1),
                                          int(n_parts), _ptr(P, torch.float64, (n, 3, 4), "P"),
                                          _ptr(theta, torch.float64, (n_parts, n, 6), "theta"),
                                          _ptr(proj_out, torch.float32, plan.proj_shape, "proj_out"),
                                          _ws(plan, workspace), _stream(stream)), "gmc_forward_project_parts")


def gmc_akima_theta(n_views, n_nodes, coeffs, theta, stream=None):
    check(lib().gmc_akima_theta(int(n_views), int(n_nodes), _ptr(coeffs, torch.float64, (6, n_nodes), "coeffs"),
                                _ptr(theta, torch.float64, (n_views, 6), "theta"), _stream(stream)),
          "gmc_akima_theta")


def gmc_akima_grad(n_views, n_nodes, coeffs, grad_theta, grad_coeffs, stream=None):
    check(lib().gmc_akima_grad(int(n_views), int(n_nodes), _ptr(coeffs, torch.float64, (6, n_nodes), "coeffs"),
                               _ptr(grad_theta, torch.float64, (n_views, 6), "grad_theta"),
                               _ptr(grad_coeffs, torch.float64, (6, n_nodes), "grad_coeffs"), _stream(stream)),
          "gmc_akima_grad")


def gmc_adam_step(x, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    n = x.numel()
    check(lib().gmc_adam_step(n, _ptr(x, torch.float64, x.shape, "x"), _ptr(g, torch.float64, x.shape, "g"),
                              _ptr(m, torch.float64, x.shape, "m"), _ptr(v, torch.float64, x.shape, "v"), int(t),
                              float(lr), float(beta1), float(beta2), float(eps), _stream(stream)), "gmc_adam_step")


def gmc_gd_step(x, g, n_iter, s0, decay, stream=None):
    check(lib().gmc_gd_step(x.numel(), _ptr(x, torch.float64, x.shape, "x"), _ptr(g, torch.float64, x.shape, "g"),
                            int(n_iter), float(s0), float(decay), _stream(stream)), "gmc_gd_step")


def gmc_debug_project(plan: Plan, voxel, view, cell, frac, workspace, stream=None):
    n = voxel.numel()
    check(lib().gmc_debug_project(plan.handle, n, _ptr(voxel, torch.int64, (n,), "voxel"),
                                  _ptr(view, torch.int32, (n,), "view"), _ptr(cell, torch.int32, (n, 2), "cell"),
                                  _ptr(frac, torch.float32, (n, 2), "frac"), _ws(plan, workspace), _stream(stream)),
          "gmc_debug_project")


def gmc_launch_batch(items, stream=None):
    arr = (Work * max(1, len(items)))()
    keep = []
    for q, it in enumerate(items):
        plan = it["plan"]
        n = plan.geometry.n_views
        w = arr[q]
        w.plan = plan.handle
        w.proj = _ptr(it["proj"], torch.float32, plan.proj_shape, "proj")
        w.P = _ptr(it.get("P"), torch.float64, (n, 3, 4), "P", True)
        w.theta = _ptr(it.get("theta"), torch.float64, (n, 6), "theta", True)
        w.vol = _ptr(it.get("vol"), torch.float32, plan.vol_shape, "vol", True)
        w.grad_vol = _ptr(it.get("grad_vol"), torch.float32, plan.vol_shape, "grad_vol", True)
        w.grad_theta = _ptr(it.get("grad_theta"), torch.float64, (n, 6), "grad_theta", True)
        w.grad_P = _ptr(it.get("grad_P"), torch.float64, (n, 3, 4), "grad_P", True)
        w.workspace = _ws(plan, it["workspace"])
        w.phase = int(it["phase"])
        w.flags = int(it.get("flags", 0))
        keep.append(it)
    check(lib().gmc_launch_batch(arr, len(items), _stream(stream)), "gmc_launch_batch")


def gmc_check(plan: Plan, workspace, stream=None):
    check(lib().gmc_check(plan.handle, _ws(plan, workspace), _stream(stream)), "gmc_check")
