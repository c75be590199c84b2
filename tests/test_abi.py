"""Host-side checks of the C ABI (no GPU): the library loads, exports every entry point that
include/gmc.h declares, validates plans and sizes workspaces. No kernel is launched."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2401_09283_amd import _lib, gmc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_entry_points():
    src = open(os.path.join(ROOT, "include", "gmc.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gmc_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_entry_point():
    names = declared_entry_points()
    assert len(names) >= 15
    L = _lib.lib()
    for n in names:
        assert hasattr(L, n), n
    assert sorted(names) == sorted(_lib.EXPORTS)


def test_status_strings():
    L = _lib.lib()
    for code, name in _lib.STATUS.items():
        assert L.gmc_status_string(code).decode() == name


def _geom(**kw):
    d = dict(n_views=10, det_w=64, det_h=48, shape=(20, 18, 17), voxel_mm=(1.0, 1.0, 1.0), origin_mm=(-9.5, -8.5, -8.0))
    d.update(kw)
    return gmc.make_geometry(d["n_views"], d["det_w"], d["det_h"], d["shape"], d["voxel_mm"], d["origin_mm"],
                             d.get("weighting", "fdk"), d.get("grad_mode", "paper"), d.get("flags", 0))


@pytest.mark.parametrize("bad", [dict(n_views=0), dict(det_w=0), dict(shape=(0, 4, 4)), dict(voxel_mm=(1.0, -1.0, 1.0)),
                                 dict(weighting=7), dict(grad_mode=3), dict(flags=8),
                                 dict(origin_mm=(float("nan"), 0.0, 0.0))])
def test_invalid_geometry_is_rejected(bad):
    with pytest.raises(gmc.GmcError) as e:
        gmc.Plan(_geom(**bad))
    assert e.value.status == -1


@pytest.mark.parametrize("big", [dict(shape=(1 << 14, 1 << 14, 1 << 13)),              # > 2^40 voxels
                                 dict(shape=(1 << 13, 1 << 13, 1 << 13)),              # 2^27 bricks
                                 dict(shape=(1 << 12, 1 << 12, 1 << 10), n_views=1 << 16)])  # 2^34 pairs
def test_oversized_geometry_is_unsupported(big):
    """Work items are numbered in 32 bits: plans beyond 2^26 bricks or 2^33 (brick, view) pairs
    are refused before anything is sized."""
    with pytest.raises(gmc.GmcError) as e:
        gmc.Plan(_geom(**big))
    assert e.value.status == -5


def test_plan_bricks_and_workspace():
    p = gmc.Plan(_geom())
    info = p.info()
    assert info["brick"] == (16, 16, 16)
    assert info["n_bricks"] == 2 * 2 * 2           # ragged: 20, 18, 17 -> 2, 2 and 2 bricks
    n, nb = 10, 8
    # at least: Phat + dPhat + descriptors (64 B) + partials (64 B) per (view, brick)
    assert p.workspace_bytes >= n * 12 * 8 + n * 72 * 8 + 2 * n * nb * 64
    assert p.workspace_bytes % 256 == 0


def test_view_chunks_follow_the_brick_count():
    # 8 bricks and 10 views: the views of every brick split into as many chunks as there are
    # views (forward 8, VJP 10), with room for the forward's seven extra partial volumes
    p = gmc.Plan(_geom())
    assert p.info()["view_chunks"] == (8, 10)
    assert p.workspace_bytes >= 7 * 20 * 18 * 17 * 4
    # never more chunks than views
    assert gmc.Plan(_geom(n_views=2)).info()["view_chunks"] == (2, 2)
    assert gmc.Plan(_geom(n_views=1)).info()["view_chunks"] == (1, 1)
    # a volume that fills the GPU by its bricks alone: 4 forward chunks, 16 VJP chunks
    g = gmc.make_geometry(16, 64, 64, (256, 256, 256), (1.0, 1.0, 1.0), (0.0, 0.0, 0.0))
    info = gmc.Plan(g).info()
    assert info["n_bricks"] == 16 * 16 * 16 and info["view_chunks"] == (4, 16)
    # with more views the VJP takes 32 chunks, fewer where 32 would pass 2^30 work items
    g = gmc.make_geometry(64, 64, 64, (256, 256, 256), (1.0, 1.0, 1.0), (0.0, 0.0, 0.0))
    assert gmc.Plan(g).info()["view_chunks"] == (4, 32)
    g = gmc.make_geometry(64, 64, 64, (1 << 13, 1 << 13, 1 << 12), (1.0, 1.0, 1.0), (0.0, 0.0, 0.0))
    info = gmc.Plan(g).info()
    assert info["n_bricks"] == 1 << 26 and info["view_chunks"][1] == 16
    # the forward's partial volumes stay within 4 GiB
    g = gmc.make_geometry(16, 64, 64, (1024, 1024, 1024), (1.0, 1.0, 1.0), (0.0, 0.0, 0.0))
    assert gmc.Plan(g).info()["view_chunks"] == (2, 16)


def test_nominal_geometry_picks_the_tile():
    from synth import CONFIGS
    from synth.geometry import projection_matrices

    # deep bricks where their tiles fit the small or middle tile; the paper's coarse voxels on a
    # fine detector project 16-voxel bricks taller than the largest tile holds: shallow bricks
    for name, pitch, rows, bz in (("tiny", 40, 64, 16), ("head256", 80, 64, 16), ("serve384", 80, 64, 16),
                                  ("paper128", 128, 64, 8)):
        cfg = CONFIGS[name]
        g = gmc.make_geometry(cfg.n_views, cfg.det_w, cfg.det_h, cfg.grid.shape, cfg.grid.voxel_mm, cfg.grid.origin_mm)
        info = gmc.Plan(g, projection_matrices(cfg.scan)).info()
        assert (info["tile_pitch"], info["tile_rows"], info["brick"]) == (pitch, rows, (16, 16, bz)), name


@pytest.mark.parametrize("geo", [dict(shape=(1 << 23, 2, 2)),                                  # axis > 2^22
                                 dict(shape=(4096, 4096, 64), voxel_mm=(1.0, 1.0, 1e-4))])   # > 2^24 steps
def test_forward_projection_refuses_rays_it_cannot_count(geo):
    """The projector's march counts samples in FP32: geometries beyond 2^24 steps per ray (or an
    axis beyond 2^22 voxels) are refused before anything is launched (the pointers here are
    never dereferenced)."""
    L = _lib.lib()
    p = gmc.Plan(_geom(**geo))
    fake = ctypes.c_void_p(256)
    assert L.gmc_forward_project(p.handle, fake, fake, fake, fake, fake, None) == -5
    assert b"2^24" in L.gmc_last_error()


def test_null_workspace_and_arguments_are_rejected_without_launching():
    L = _lib.lib()
    p = gmc.Plan(_geom())
    st = L.gmc_backproject(p.handle, None, None, None, None, None, None)
    assert st == -2  # workspace checked first
    st = L.gmc_backproject(p.handle, None, None, None, None, ctypes.c_void_p(256), None)
    assert st == -1
    st = L.gmc_backproject(p.handle, None, None, None, None, ctypes.c_void_p(257), None)
    assert st == -2  # misaligned
    assert L.gmc_bspline_theta(10, 3, None, None, None) == -1
    assert L.gmc_adam_step(5, None, None, None, None, 0, 0.1, 0.9, 0.999, 1e-8, None) == -1
    assert b"t >= 1" in L.gmc_last_error()


def test_allocation_free_vjp_refuses_plans_beyond_its_static_buffer():
    """The 256^3 x 496-view plan needs ~0.5 GB of VJP scratch: refused before any launch or device
    query (the pointers are never touched, so host stand-ins suffice)."""
    g = gmc.make_geometry(496, 620, 480, (256, 256, 256), (1.0, 1.0, 1.0), (-127.5, -127.5, -127.5))
    plan = gmc.Plan(g)
    dummy = ctypes.c_void_p(256)
    st = _lib.lib().gmc_backproject_vjp_noalloc(plan.handle, dummy, dummy, dummy, dummy, dummy, None, None, None)
    assert st == -5
    msg = _lib.lib().gmc_last_error().decode()
    assert "static" in msg and "gmc_backproject_vjp" in msg
    # a plan that fits is not refused by size (it would then need a GPU): 128^3 x 248 views
    small = gmc.Plan(gmc.make_geometry(248, 310, 240, (128, 128, 128), (2.0, 2.0, 2.0), (-127.0, -127.0, -127.0)))
    assert 128 * 248 * 1024 < _lib.NOALLOC_SCRATCH_BYTES
    st = _lib.lib().gmc_backproject_vjp_noalloc(small.handle, None, dummy, dummy, dummy, dummy, None, None, None)
    assert st == -1   # NULL proj: an argument error, returned before the size check matters
