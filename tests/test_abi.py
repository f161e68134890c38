"""Host-side checks of the C ABI: the built library loads, exports every
function include/quadbox.h declares, and rejects bad arguments before any
device work (these calls return before touching the GPU)."""
import ctypes as C
import os
import re

import pytest

from paper_2605_04844_amd import quadbox as qb

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "quadbox.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(qb_[a-z_]+)\s*\(", text)))


def test_header_declares_entry_points():
    fns = header_functions()
    for name in ("qb_project", "qb_intersect", "qb_sort", "qb_render", "qb_status_string"):
        assert name in fns


def test_library_exports_every_declared_symbol():
    L = qb.lib()
    for name in header_functions():
        assert hasattr(L, name), name


def test_status_strings_and_version():
    assert qb.status_string(0) == "ok"
    assert qb.status_string(-1) == "invalid argument"
    assert qb.status_string(-2) == "pair capacity exceeded"
    assert qb.lib().qb_version() >= 100


def _cam(w=64, h=48, fx=64.0):
    c = qb.CCamera()
    c.width, c.height, c.fx, c.fy, c.cx, c.cy, c.near_plane = w, h, fx, fx, w / 2, h / 2, 0.2
    c.R[0] = c.R[4] = c.R[8] = 1.0
    return c


def test_project_rejects_bad_arguments():
    L = qb.lib()
    cam = _cam()
    dummy = C.c_void_p(16)
    args = lambda n=4, deg=0, mode=2, c=cam: (n, dummy, dummy, dummy, dummy, dummy, deg, C.byref(c), mode,
                                              dummy, dummy, dummy, None)
    assert L.qb_project(*args(n=-1)) == qb.QB_ERR_INVALID_ARG
    assert L.qb_project(*args(deg=4)) == qb.QB_ERR_INVALID_ARG
    assert L.qb_project(*args(mode=7)) == qb.QB_ERR_INVALID_ARG
    bad = _cam(w=0)
    assert L.qb_project(*args(c=bad)) == qb.QB_ERR_INVALID_ARG
    bad = _cam(fx=0.0)
    assert L.qb_project(*args(c=bad)) == qb.QB_ERR_INVALID_ARG
    assert L.qb_project(4, None, dummy, dummy, dummy, dummy, 0, C.byref(cam), 2, dummy, dummy, dummy,
                        None) == qb.QB_ERR_INVALID_ARG
    assert L.qb_project(0, None, None, None, None, None, 0, C.byref(cam), 2, None, None, None, None) == qb.QB_OK
    # qb_project_ex checks the same arguments (the keys pointer may be NULL)
    for kw in (dict(n=-1), dict(deg=4), dict(mode=7), dict(c=_cam(w=0))):
        assert L.qb_project_ex(*args(**kw)[:-1], dummy, None) == qb.QB_ERR_INVALID_ARG
    assert L.qb_project_ex(0, None, None, None, None, None, 0, C.byref(cam), 2, None, None, None, None,
                           None) == qb.QB_OK


def test_intersect_sort_render_reject_bad_arguments():
    L = qb.lib()
    d = C.c_void_p(256)
    ws = qb.intersect_workspace_size(10)
    assert ws > 0
    assert L.qb_intersect(10, d, d, d, 64, 48, 2, 100, d, d, d, d, ws - 1, None) == qb.QB_ERR_INVALID_ARG
    assert L.qb_intersect(10, d, d, d, 0, 48, 2, 100, d, d, d, d, ws, None) == qb.QB_ERR_INVALID_ARG
    assert L.qb_intersect(-1, d, d, d, 64, 48, 2, 100, d, d, d, d, ws, None) == qb.QB_ERR_INVALID_ARG
    assert L.qb_intersect(10, d, d, d, 64, 48, 2, -1, d, d, d, d, ws, None) == qb.QB_ERR_INVALID_ARG
    assert L.qb_intersect(10, d, d, d, 64, 48, 2, 100, d, d, None, d, ws, None) == qb.QB_ERR_INVALID_ARG
    assert L.qb_intersect(10, d, d, d, 64, 48, 2, 100, None, d, d, d, ws, None) == qb.QB_ERR_INVALID_ARG
    assert L.qb_intersect(10, d, d, d, 64, 48, 5, 100, d, d, d, d, ws, None) == qb.QB_ERR_INVALID_ARG
    assert L.qb_intersect(10, d, d, d, 64, 48, -1, 100, d, d, d, d, ws, None) == qb.QB_ERR_INVALID_ARG
    assert L.qb_intersect(10, d, d, d, 16 * 300, 16 * 300, 2, 100, d, d, d, d, 1 << 40, None) == \
        qb.QB_ERR_UNSUPPORTED
    sws = qb.sort_workspace_size(100)
    assert L.qb_sort(100, d, 12, d, d, d, d, C.c_void_p(512), d, d, sws - 1, None) == qb.QB_ERR_INVALID_ARG
    assert L.qb_sort(100, d, 0, d, d, d, d, C.c_void_p(512), d, d, sws, None) == qb.QB_ERR_INVALID_ARG
    assert L.qb_sort(100, d, 12, d, d, d, d, d, d, d, sws, None) == qb.QB_ERR_INVALID_ARG
    assert L.qb_sort(100, d, 12, d, d, None, d, C.c_void_p(512), d, d, sws, None) == qb.QB_ERR_INVALID_ARG
    assert L.qb_sort(100, None, 12, d, d, d, d, C.c_void_p(512), d, d, sws, None) == qb.QB_ERR_INVALID_ARG
    assert L.qb_render(0, 48, d, d, d, d, d, None, None, None, None) == qb.QB_ERR_INVALID_ARG
    assert L.qb_render(64, 48, None, d, d, d, d, None, None, None, None) == qb.QB_ERR_INVALID_ARG


def test_intersect_noalloc_rejects_bad_arguments_and_fits_its_scratch():
    """qb_intersect_noalloc checks its arguments as qb_intersect does and
    rejects n above QB_NOALLOC_MAX_GAUSSIANS before any device work; the
    workspace of the largest accepted n fits the library's 60 MiB static
    scratch."""
    L = qb.lib()
    d = C.c_void_p(256)
    cap = qb.NOALLOC_MAX_GAUSSIANS
    assert qb.intersect_workspace_size(cap) <= 60 << 20
    assert L.qb_intersect_noalloc(cap + 1, d, d, d, 64, 48, 2, 100, d, d, d, None) == qb.QB_ERR_INVALID_ARG
    assert L.qb_intersect_noalloc(-1, d, d, d, 64, 48, 2, 100, d, d, d, None) == qb.QB_ERR_INVALID_ARG
    assert L.qb_intersect_noalloc(10, d, d, d, 0, 48, 2, 100, d, d, d, None) == qb.QB_ERR_INVALID_ARG
    assert L.qb_intersect_noalloc(10, d, d, d, 64, 48, 2, -1, d, d, d, None) == qb.QB_ERR_INVALID_ARG
    assert L.qb_intersect_noalloc(10, d, d, d, 64, 48, 2, 100, d, d, None, None) == qb.QB_ERR_INVALID_ARG
    assert L.qb_intersect_noalloc(10, None, d, d, 64, 48, 2, 100, d, d, d, None) == qb.QB_ERR_INVALID_ARG
    assert L.qb_intersect_noalloc(10, d, d, d, 64, 48, 5, 100, d, d, d, None) == qb.QB_ERR_INVALID_ARG
    assert L.qb_intersect_noalloc(10, d, d, d, 16 * 300, 16 * 300, 2, 100, d, d, d, None) == \
        qb.QB_ERR_UNSUPPORTED


def test_activations_and_shape_entry_points_reject_bad_arguments():
    L = qb.lib()
    d = C.c_void_p(256)
    L.qb_activations.argtypes = [C.c_int64, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]
    assert L.qb_activations(-1, d, 0, d, None) == qb.QB_ERR_INVALID_ARG
    assert L.qb_activations(4, d, 3, d, None) == qb.QB_ERR_INVALID_ARG
    assert L.qb_activations(4, d, -1, d, None) == qb.QB_ERR_INVALID_ARG
    assert L.qb_activations(4, None, 0, d, None) == qb.QB_ERR_INVALID_ARG
    assert L.qb_activations(0, None, 0, None, None) == qb.QB_OK   # nothing to do, nothing launched
    ws = qb.intersect_workspace_size(10)
    for dv, ev in ((4, 0), (-1, 0), (0, 5), (0, -1)):
        assert L.qb_intersect_ex(10, d, d, d, 64, 48, 2, 100, d, d, d, d, ws, None, dv, ev, 0, None) == \
            qb.QB_ERR_INVALID_ARG
        assert L.qb_intersect_ex(10, d, d, d, 64, 48, 2, 100, d, d, d, d, ws, d, dv, ev, 0, None) == \
            qb.QB_ERR_INVALID_ARG
    sws = qb.sort_workspace_size(100)
    for v in (-1, 6):
        assert L.qb_sort_ex(100, d, 12, d, d, d, None, C.c_void_p(512), d, d, sws, v, 0, None) == \
            qb.QB_ERR_INVALID_ARG


def test_packed_pair_format_arguments():
    """qb_pair_id_bits: ceil(log2 n) id bits when they and the tile id fit 32
    bits, else 0; qb_intersect_ex and qb_sort_ex reject a packed format that
    cannot hold the ids or the tiles, and accept a NULL pair_tiles with it."""
    L = qb.lib()
    assert qb.pair_id_bits(1_000_000, 1280, 720) == 20        # 3600 tiles: 12 bits
    assert qb.pair_id_bits(1 << 20, 1280, 720) == 20
    assert qb.pair_id_bits((1 << 20) + 1, 1280, 720) == 0     # 21 + 12 bits
    assert qb.pair_id_bits(2_000_000, 640, 360) == 21         # 920 tiles: 10 bits
    assert qb.pair_id_bits(2_000_000, 1920, 1080) == 0
    assert qb.pair_id_bits(1, 64, 64) == 1 and qb.pair_id_bits(0, 64, 64) == 1
    assert qb.pair_id_bits(5, 0, 64) == 0 and qb.pair_id_bits(-1, 64, 64) == 0
    d = C.c_void_p(256)
    ws = qb.intersect_workspace_size(10)
    args = lambda n, bits: (n, d, d, d, 64, 48, 2, 100, None, d, d, d, ws, None, 0, 0, bits, None)
    for bits in (-1, 32, 3):   # 3 bits cannot hold 10 ids
        assert L.qb_intersect_ex(*args(10, bits)) == qb.QB_ERR_INVALID_ARG, bits
    wsb = qb.intersect_workspace_size(1 << 20)
    big = (1 << 20, d, d, d, 16 * 256, 16 * 256, 2, 100, None, d, d, d, wsb, None, 0, 0, 20, None)
    assert L.qb_intersect_ex(*big) == qb.QB_ERR_INVALID_ARG   # 65536 tiles: 16 bits + 20 > 32
    sws = qb.sort_workspace_size(100)
    for bits in (-1, 32, 21):   # 21 + 12 tile bits > 32
        assert L.qb_sort_ex(100, d, 3600, None, d, d, None, d, d, d, sws, 0, bits, None) == \
            qb.QB_ERR_INVALID_ARG, bits
    # split pairs still need pair_tiles
    assert L.qb_sort_ex(100, d, 3600, None, d, d, None, d, d, d, sws, 0, 0, None) == qb.QB_ERR_INVALID_ARG


def test_launch_shape_and_view_entry_points_reject_bad_arguments():
    L = qb.lib()
    d = C.c_void_p(256)
    bg = (C.c_float * 3)(0.0, 0.0, 0.0)
    bgp = C.cast(bg, C.c_void_p)
    # launch shapes out of range
    nv = len(qb.RENDER_VARIANTS)   # QB_RENDER_VARIANTS: one past the last launch shape
    assert L.qb_render_ex(64, 48, d, d, d, bgp, d, None, None, None, nv, None, None) == qb.QB_ERR_INVALID_ARG
    assert L.qb_render_ex(64, 48, d, d, d, bgp, d, None, None, None, -1, None, None) == qb.QB_ERR_INVALID_ARG
    assert L.qb_render_backward_ex(64, 48, d, d, d, bgp, d, d, d, 10, d, 3, None, None) == qb.QB_ERR_INVALID_ARG
    # view tables: count, null table, bad sizes, missing buffers
    views = (qb.CView * (qb.MAX_VIEWS + 1))()
    for v in views:
        v.width, v.height = 64, 48
        v.ranges = v.ids = v.splats = v.image = v.final_T = v.n_contrib = v.dL_dimage = v.grad2d = 256
    assert L.qb_render_views(0, views, bgp, None) == qb.QB_ERR_INVALID_ARG
    assert L.qb_render_views(qb.MAX_VIEWS + 1, views, bgp, None) == qb.QB_ERR_INVALID_ARG
    assert L.qb_render_views(1, None, bgp, None) == qb.QB_ERR_INVALID_ARG
    assert L.qb_render_views_ex(1, views, bgp, nv, None, None) == qb.QB_ERR_INVALID_ARG
    views[1].width = 0
    assert L.qb_render_views(2, views, bgp, None) == qb.QB_ERR_INVALID_ARG
    views[1].width = 64
    views[1].image = None
    assert L.qb_render_views(2, views, bgp, None) == qb.QB_ERR_INVALID_ARG
    views[1].dL_dimage = None
    assert L.qb_render_backward_views(2, views, bgp, 10, None) == qb.QB_ERR_INVALID_ARG
    assert L.qb_render_backward_views_ex(1, views, bgp, 10, 4, None, None) == qb.QB_ERR_INVALID_ARG
    # tile order: sizes, null buffers, view tables
    assert L.qb_tile_order(0, 48, d, d, d, d, d, None) == qb.QB_ERR_INVALID_ARG
    assert L.qb_tile_order(64, 48, None, d, d, d, d, None) == qb.QB_ERR_INVALID_ARG
    assert L.qb_tile_order(64, 48, d, d, d, None, d, None) == qb.QB_ERR_INVALID_ARG
    assert L.qb_tile_order(64, 48, d, d, d, d, None, None) == qb.QB_ERR_INVALID_ARG
    assert L.qb_tile_order_views(0, views, d, d, None) == qb.QB_ERR_INVALID_ARG
    assert L.qb_tile_order_views(1, views, None, d, None) == qb.QB_ERR_INVALID_ARG
    assert L.qb_tile_order_views(2, views, d, d, None) == qb.QB_ERR_INVALID_ARG   # view 1 has no image
    cams = (qb.CCamera * (qb.MAX_VIEWS + 1))(*[_cam() for _ in range(qb.MAX_VIEWS + 1)])
    assert L.qb_project_views(10, d, d, d, d, d, 0, cams, 0, 2, d, d, d, None) == qb.QB_ERR_INVALID_ARG
    assert L.qb_project_views(10, d, d, d, d, d, 0, cams, qb.MAX_VIEWS + 1, 2, d, d, d, None) == \
        qb.QB_ERR_INVALID_ARG
    assert L.qb_project_views(10, d, d, d, d, d, 0, cams, 2, 7, d, d, d, None) == qb.QB_ERR_INVALID_ARG
    cams[1].fx = 0.0
    assert L.qb_project_views(10, d, d, d, d, d, 0, cams, 2, 2, d, d, d, None) == qb.QB_ERR_INVALID_ARG
    assert L.qb_project_backward_views(10, d, d, d, d, d, 0, cams, 2, d, d, d, d, d, d, d, None) == \
        qb.QB_ERR_INVALID_ARG
    assert L.qb_project_backward_views_ex(10, d, d, d, d, d, 0, cams, 2, d, d, d, d, d, d, d, 1, None) == \
        qb.QB_ERR_INVALID_ARG
    cams[1].fx = 64.0
    assert L.qb_project_backward_views(10, d, d, d, d, d, 4, cams, 2, d, d, d, d, d, d, d, None) == \
        qb.QB_ERR_INVALID_ARG
    # the clear flag is 0 or 1; the adding render backward checks like the clearing one
    for flag in (-1, 2):
        assert L.qb_project_backward_views_ex(10, d, d, d, d, d, 0, cams, 2, d, d, d, d, d, d, d, flag, None) == \
            qb.QB_ERR_INVALID_ARG
    assert L.qb_render_backward_views_acc(2, views, bgp, 10, 0, None, None) == qb.QB_ERR_INVALID_ARG
    assert L.qb_render_backward_views_acc(1, views, bgp, 10, 4, None, None) == qb.QB_ERR_INVALID_ARG
    assert L.qb_render_backward_views_acc(1, views, None, 10, 0, None, None) == qb.QB_ERR_INVALID_ARG


def test_cameras_need_a_positive_near_plane_and_finite_fields():
    """Depth keys are the binary32 bits of the view depth, which order
    correctly only for positive depths: every entry point that takes a camera
    rejects near_plane <= 0 (or NaN) and any non-finite field."""
    L = qb.lib()
    d = C.c_void_p(256)

    def proj(c):
        return L.qb_project(4, d, d, d, d, d, 0, C.byref(c), 2, d, d, d, None)

    def proj_bwd(c):
        return L.qb_project_backward(4, d, d, d, d, d, 0, C.byref(c), d, d, d, d, d, d, d, None)

    def views(c):
        cams = (qb.CCamera * 2)(_cam(), c)
        return (L.qb_project_views(4, d, d, d, d, d, 0, cams, 2, 2, d, d, d, None),
                L.qb_project_backward_views(4, d, d, d, d, d, 0, cams, 2, d, d, d, d, d, d, d, None))

    for near in (0.0, -0.5, float("nan")):
        c = _cam()
        c.near_plane = near
        assert proj(c) == qb.QB_ERR_INVALID_ARG
        assert proj_bwd(c) == qb.QB_ERR_INVALID_ARG
        assert views(c) == (qb.QB_ERR_INVALID_ARG, qb.QB_ERR_INVALID_ARG)
    for field, k in (("R", 4), ("t", 2), ("campos", 0)):
        c = _cam()
        getattr(c, field)[k] = float("inf")
        assert proj(c) == qb.QB_ERR_INVALID_ARG and proj_bwd(c) == qb.QB_ERR_INVALID_ARG
    c = _cam()
    c.cx = float("nan")
    assert proj(c) == qb.QB_ERR_INVALID_ARG
    # a valid camera with n = 0 is accepted without touching the device
    assert L.qb_project(0, None, None, None, None, None, 0, C.byref(_cam()), 2, None, None, None, None) == qb.QB_OK


def test_check_capacity_rejects_bad_arguments():
    """qb_check_capacity validates everything on the host before it reads
    the device counts."""
    L = qb.lib()
    d = C.c_void_p(256)
    caps = (C.c_int64 * 65)(*([10] * 65))
    neg = (C.c_int64 * 2)(10, -1)
    cp = C.cast(caps, C.c_void_p)
    assert L.qb_check_capacity(0, d, cp, None, None) == qb.QB_ERR_INVALID_ARG
    assert L.qb_check_capacity(1, None, cp, None, None) == qb.QB_ERR_INVALID_ARG
    assert L.qb_check_capacity(1, d, None, None, None) == qb.QB_ERR_INVALID_ARG
    assert L.qb_check_capacity(2, d, C.cast(neg, C.c_void_p), None, None) == qb.QB_ERR_INVALID_ARG
    assert L.qb_check_capacity(65, d, cp, None, None) == qb.QB_ERR_INVALID_ARG   # > 64 needs out_counts


def test_l1_grad_rejects_bad_arguments():
    """qb_l1_grad checks its items before any device work: item counts out
    of range, a missing item array, a negative count or a missing pointer
    where the count is positive; empty items launch nothing."""
    L = qb.lib()
    d = 256
    good = qb.CL1Item(8, d, d, d, 0.5)
    arr = (qb.CL1Item * 2)(good, good)
    assert L.qb_l1_grad(-1, arr, None) == qb.QB_ERR_INVALID_ARG
    assert L.qb_l1_grad(qb.MAX_VIEWS + 1, arr, None) == qb.QB_ERR_INVALID_ARG
    assert L.qb_l1_grad(1, None, None) == qb.QB_ERR_INVALID_ARG
    for bad in (qb.CL1Item(-1, d, d, d, 1.0), qb.CL1Item(8, None, d, d, 1.0), qb.CL1Item(8, d, None, d, 1.0),
                qb.CL1Item(8, d, d, None, 1.0)):
        arr2 = (qb.CL1Item * 2)(good, bad)
        assert L.qb_l1_grad(2, arr2, None) == qb.QB_ERR_INVALID_ARG
    empty = (qb.CL1Item * 2)(qb.CL1Item(0, None, None, None, 1.0), qb.CL1Item(0, d, d, d, 1.0))
    assert L.qb_l1_grad(2, empty, None) == qb.QB_OK
    assert L.qb_l1_grad(0, None, None) == qb.QB_OK
