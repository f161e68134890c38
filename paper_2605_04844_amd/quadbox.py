"""Thin Python binding of libquadbox (the C ABI in include/quadbox.h).

Only argument marshalling lives here: torch supplies device memory and the
current HIP stream, every step of the rasterizer runs in the library's HIP
kernels.  The library must be built (``python -m paper_2605_04844_amd.build``);
without it every call raises -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libquadbox.so")

BOX_MODES = {"3sigma": 0, "adr": 1, "quadbox": 2, "dualbox": 3, "quadbox_naive": 4}
CLIP_3SIGMA = 16   # QB_CLIP_3SIGMA: added to an opacity-aware mode
BOX_MODES.update({m + "_clip3sigma": BOX_MODES[m] | CLIP_3SIGMA for m in ("adr", "quadbox", "dualbox", "quadbox_naive")})
TILE = 16
SPLAT_FLOATS = 12   # qb_splat: u v depth o | a b c gamma | r g b visible
RECT_SHORTS = 16    # qb_rects: 4 x (tx0, tx1, ty0, ty1)

QB_OK, QB_ERR_INVALID_ARG, QB_ERR_CAPACITY, QB_ERR_HIP, QB_ERR_UNSUPPORTED = 0, -1, -2, -3, -4
# render launch shapes (qb_render_variant): pixels per lane of a tile row, and
# (_rows) whether waves drop batch entries whose ellipse misses their rows,
# (_xrow) whether the row terms of the quadratic form are computed by one lane
# per tile row and shared with the row's other lanes, (_xrow1) the same with
# one branch per entry instead of one per pair of entries
RENDER_VARIANTS = {"2px": 0, "1px": 1, "4px": 2, "2px_rows": 3, "1px_rows": 4, "2px_xrow": 5, "4px_xrow": 6,
                   "2px_xrow1": 7}
BACKWARD_VARIANTS = {"2px": 0, "1px": 1, "4px": 2}
# tile-sort radix workgroups (qb_sort_variant): lanes x pairs per lane, and
# two digit-width variants of 512 x 8 (first pass 2 bits narrower / wider)
SORT_VARIANTS = {"512x8": 0, "1024x8": 1, "512x16": 2, "256x16": 3, "512x8_narrow_first": 4,
                 "512x8_wide_first": 5}
# qb_intersect's depth-sort radix workgroups (qb_depth_variant) and emission
# workgroup sizes (qb_emit_variant)
DEPTH_VARIANTS = {"512x4": 0, "256x8": 1, "512x8": 2, "1024x4": 3}
EMIT_VARIANTS = {"256": 0, "128": 1, "512": 2, "256x2": 3, "128x2": 4}


class QBError(RuntimeError):
    def __init__(self, fn, status):
        super().__init__(f"{fn} failed: {status_string(status)} ({status})")
        self.status = status


class CCamera(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("fx", C.c_float), ("fy", C.c_float),
                ("cx", C.c_float), ("cy", C.c_float), ("near_plane", C.c_float),
                ("R", C.c_float * 9), ("t", C.c_float * 3), ("campos", C.c_float * 3)]


class CView(C.Structure):
    """qb_view: per-view buffers of a batched call."""
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("ranges", C.c_void_p), ("ids", C.c_void_p),
                ("splats", C.c_void_p), ("image", C.c_void_p), ("final_T", C.c_void_p), ("n_contrib", C.c_void_p),
                ("dL_dimage", C.c_void_p), ("grad2d", C.c_void_p)]


class CL1Item(C.Structure):
    """qb_l1_item: one (image, target, grad, scale) of qb_l1_grad."""
    _fields_ = [("count", C.c_int64), ("image", C.c_void_p), ("target", C.c_void_p), ("grad", C.c_void_p),
                ("scale", C.c_float)]


MAX_VIEWS = 32

_lib = None


def lib():
    """Load libquadbox.so (raises when it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libquadbox.so not built at {LIB_PATH}; run python -m paper_2605_04844_amd.build")
    L = C.CDLL(LIB_PATH)
    vp, i64, i32, sz = C.c_void_p, C.c_int64, C.c_int32, C.c_size_t
    L.qb_project.argtypes = [i64, vp, vp, vp, vp, vp, i32, C.POINTER(CCamera), i32, vp, vp, vp, vp]
    L.qb_project.restype = i32
    L.qb_project_ex.argtypes = [i64, vp, vp, vp, vp, vp, i32, C.POINTER(CCamera), i32, vp, vp, vp, vp, vp]
    L.qb_project_ex.restype = i32
    L.qb_intersect_workspace_size.argtypes = [i64]
    L.qb_intersect_workspace_size.restype = sz
    L.qb_intersect.argtypes = [i64, vp, vp, vp, i32, i32, i32, i64, vp, vp, vp, vp, sz, vp]
    L.qb_intersect.restype = i32
    L.qb_intersect_ex.argtypes = [i64, vp, vp, vp, i32, i32, i32, i64, vp, vp, vp, vp, sz, vp, i32, i32, i32, vp]
    L.qb_intersect_ex.restype = i32
    L.qb_sort_ex.argtypes = [i64, vp, i32, vp, vp, vp, vp, vp, vp, vp, sz, i32, i32, vp]
    L.qb_pair_id_bits.argtypes = [i64, i32, i32]
    L.qb_pair_id_bits.restype = i32
    L.qb_sort_ex.restype = i32
    L.qb_sort_workspace_size.argtypes = [i64]
    L.qb_sort_workspace_size.restype = sz
    L.qb_sort.argtypes = [i64, vp, i32, vp, vp, vp, vp, vp, vp, vp, sz, vp]
    L.qb_sort.restype = i32
    L.qb_render.argtypes = [i32, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    L.qb_render.restype = i32
    L.qb_render_ex.argtypes = [i32, i32, vp, vp, vp, vp, vp, vp, vp, vp, i32, vp, vp]
    L.qb_render_ex.restype = i32
    L.qb_render_backward.argtypes = [i32, i32, vp, vp, vp, vp, vp, vp, vp, i64, vp, vp]
    L.qb_render_backward.restype = i32
    L.qb_render_backward_ex.argtypes = [i32, i32, vp, vp, vp, vp, vp, vp, vp, i64, vp, i32, vp, vp]
    L.qb_tile_order.argtypes = [i32, i32, vp, vp, vp, vp, vp, vp]
    L.qb_tile_order.restype = i32
    L.qb_render_backward_ex.restype = i32
    L.qb_project_backward.argtypes = [i64, vp, vp, vp, vp, vp, i32, C.POINTER(CCamera), vp, vp, vp, vp, vp, vp, vp,
                                      vp]
    L.qb_project_backward.restype = i32
    pc = C.POINTER(CCamera)
    L.qb_project_views.argtypes = [i64, vp, vp, vp, vp, vp, i32, pc, i32, i32, vp, vp, vp, vp]
    L.qb_project_views.restype = i32
    L.qb_project_views_ex.argtypes = [i64, vp, vp, vp, vp, vp, i32, pc, i32, i32, vp, vp, vp, vp, vp]
    L.qb_project_views_ex.restype = i32
    L.qb_render_views.argtypes = [i32, C.POINTER(CView), vp, vp]
    L.qb_render_views.restype = i32
    L.qb_render_views_ex.argtypes = [i32, C.POINTER(CView), vp, i32, vp, vp]
    L.qb_tile_order_views.argtypes = [i32, C.POINTER(CView), vp, vp, vp]
    L.qb_tile_order_views.restype = i32
    L.qb_render_views_ex.restype = i32
    L.qb_render_backward_views.argtypes = [i32, C.POINTER(CView), vp, i64, vp]
    L.qb_render_backward_views.restype = i32
    L.qb_render_backward_views_ex.argtypes = [i32, C.POINTER(CView), vp, i64, i32, vp, vp]
    L.qb_render_backward_views_ex.restype = i32
    L.qb_project_backward_views.argtypes = [i64, vp, vp, vp, vp, vp, i32, pc, i32, vp, vp, vp, vp, vp, vp, vp, vp]
    L.qb_project_backward_views.restype = i32
    L.qb_render_backward_views_acc.argtypes = [i32, C.POINTER(CView), vp, i64, i32, vp, vp]
    L.qb_render_backward_views_acc.restype = i32
    L.qb_project_backward_views_ex.argtypes = [i64, vp, vp, vp, vp, vp, i32, pc, i32, vp, vp, vp, vp, vp, vp, vp,
                                               i32, vp]
    L.qb_project_backward_views_ex.restype = i32
    L.qb_status_string.argtypes = [i32]
    L.qb_status_string.restype = C.c_char_p
    L.qb_version.argtypes = []
    L.qb_version.restype = i32
    L.qb_render_stats.argtypes = [i32, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp, i32, vp, vp]
    L.qb_render_stats.restype = i32
    L.qb_check_capacity.argtypes = [i32, vp, vp, vp, vp]
    L.qb_check_capacity.restype = i32
    L.qb_intersect_noalloc.argtypes = [i64, vp, vp, vp, i32, i32, i32, i64, vp, vp, vp, vp]
    L.qb_intersect_noalloc.restype = i32
    L.qb_l1_grad.argtypes = [i32, C.POINTER(CL1Item), vp]
    L.qb_l1_grad.restype = i32
    _lib = L
    return L


def status_string(s: int) -> str:
    return lib().qb_status_string(int(s)).decode()


def _check(fn, s):
    if s != QB_OK:
        raise QBError(fn, s)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _need(cond, msg):
    if not cond:
        raise ValueError(msg)


def _rows(t):
    return 0 if t is None else int(t.shape[0])


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def camera_struct(cam) -> CCamera:
    c = CCamera()
    c.width, c.height = int(cam.width), int(cam.height)
    c.fx, c.fy, c.cx, c.cy, c.near_plane = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy), float(cam.near)
    R = [float(x) for x in np.asarray(cam.R, dtype=np.float32).reshape(9)]
    t = [float(x) for x in np.asarray(cam.t, dtype=np.float32).reshape(3)]
    p = [float(x) for x in np.asarray(cam.campos, dtype=np.float32).reshape(3)]
    for k in range(9):
        c.R[k] = R[k]
    for k in range(3):
        c.t[k] = t[k]
        c.campos[k] = p[k]
    return c


def _mode(mode) -> int:
    return BOX_MODES[mode] if isinstance(mode, str) else int(mode)


def _dev_f32(x, device):
    return torch.as_tensor(x, dtype=torch.float32, device=device).contiguous()


class Gaussians:
    """Device-resident SoA parameters (see scenes.Scene for the layouts)."""

    def __init__(self, scene=None, device="cuda", tensors=None):
        if tensors is not None:
            self.means, self.log_scales, self.quats, self.logits, self.sh = [t.contiguous() for t in tensors]
            self.sh_degree = int(round((self.sh.shape[0] // 3) ** 0.5)) - 1
        else:
            self.means = _dev_f32(scene.means, device)
            self.log_scales = _dev_f32(scene.log_scales, device)
            self.quats = _dev_f32(scene.quats, device)
            self.logits = _dev_f32(scene.logits, device)
            self.sh = _dev_f32(scene.sh, device)
            self.sh_degree = int(scene.sh_degree)
        self.n = int(self.means.shape[1])
        for name in ("means", "log_scales", "quats", "sh"):
            assert getattr(self, name).shape[-1] == self.n, name
        assert self.sh.shape[0] == 3 * (self.sh_degree + 1) ** 2
        for t in (self.means, self.log_scales, self.quats, self.logits, self.sh):
            assert t.dtype == torch.float32 and t.is_contiguous()

    def tensors(self):
        return self.means, self.log_scales, self.quats, self.logits, self.sh


# ---- one call per ABI entry point --------------------------------------------

def project(g: Gaussians, cam, mode, splats, rects, counts, depth_keys=None):
    """qb_project_ex: with depth_keys ([n] int32 tensor) the depth-sort keys
    are written as well (qb_intersect's depth_keys)."""
    _need(min(_rows(splats), _rows(rects), _rows(counts)) >= g.n, "qb_project: output buffers hold fewer than n rows")
    _need(depth_keys is None or _rows(depth_keys) >= g.n, "qb_project_ex: depth_keys holds fewer than n entries")
    _check("qb_project_ex", lib().qb_project_ex(
        g.n, _ptr(g.means), _ptr(g.log_scales), _ptr(g.quats), _ptr(g.logits), _ptr(g.sh), g.sh_degree,
        C.byref(camera_struct(cam)), _mode(mode), _ptr(splats), _ptr(rects), _ptr(counts), _ptr(depth_keys),
        _stream()))


def intersect_workspace_size(n: int) -> int:
    return int(lib().qb_intersect_workspace_size(n))


def pair_id_bits(n, width, height) -> int:
    """qb_pair_id_bits: the id width of packed pairs, 0 if they cannot be
    packed."""
    return int(lib().qb_pair_id_bits(n, width, height))


def intersect(n, splats, rects, counts, width, height, capacity, pair_tiles, pair_ids, num_pairs, ws,
              mode="quadbox", depth_variant=0, emit_variant=0, depth_keys=None, packed_id_bits=0):
    """qb_intersect_ex; depth_keys: the keys qb_project_ex wrote for this
    projection, or None to derive them from the splats; packed_id_bits > 0
    packs each pair into pair_ids (pair_tiles unused)."""
    _need(min(_rows(splats), _rows(rects), _rows(counts)) >= n, "qb_intersect: inputs hold fewer than n rows")
    _need(depth_keys is None or _rows(depth_keys) >= n, "qb_intersect_ex: depth_keys holds fewer than n entries")
    _need(capacity == 0 or (_rows(pair_ids) >= capacity and (packed_id_bits or _rows(pair_tiles) >= capacity)),
          "qb_intersect: pair buffers hold fewer than capacity entries")
    _check("qb_intersect_ex", lib().qb_intersect_ex(
        n, _ptr(splats), _ptr(rects), _ptr(counts), width, height, _mode(mode), capacity, _ptr(pair_tiles),
        _ptr(pair_ids), _ptr(num_pairs), _ptr(ws), ws.numel() * ws.element_size(), _ptr(depth_keys),
        int(depth_variant), int(emit_variant), int(packed_id_bits), _stream()))


# QB_NOALLOC_MAX_GAUSSIANS: the largest n qb_intersect_noalloc accepts
NOALLOC_MAX_GAUSSIANS = 2097152


def intersect_noalloc(n, splats, rects, counts, width, height, capacity, pair_tiles, pair_ids, num_pairs,
                      mode="quadbox"):
    """qb_intersect_noalloc: qb_intersect with the library's static scratch
    instead of a workspace (allocates nothing; calls overlapping on one GPU
    race)."""
    _need(min(_rows(splats), _rows(rects), _rows(counts)) >= n, "qb_intersect_noalloc: inputs hold fewer than n rows")
    _need(capacity == 0 or min(_rows(pair_tiles), _rows(pair_ids)) >= capacity,
          "qb_intersect_noalloc: pair buffers hold fewer than capacity entries")
    _check("qb_intersect_noalloc", lib().qb_intersect_noalloc(
        n, _ptr(splats), _ptr(rects), _ptr(counts), width, height, _mode(mode), capacity, _ptr(pair_tiles),
        _ptr(pair_ids), _ptr(num_pairs), _stream()))


def sort_workspace_size(capacity: int) -> int:
    return int(lib().qb_sort_workspace_size(capacity))


def sort(capacity, num_pairs, num_tiles, pair_tiles, pair_ids, splats, keys, ids, ranges, ws, variant=0,
         packed_id_bits=0):
    """qb_sort_ex; packed_id_bits as given to qb_intersect_ex."""
    _check("qb_sort_ex", lib().qb_sort_ex(
        capacity, _ptr(num_pairs), num_tiles, _ptr(pair_tiles), _ptr(pair_ids), _ptr(splats), _ptr(keys),
        _ptr(ids), _ptr(ranges), _ptr(ws), ws.numel() * ws.element_size(), int(variant), int(packed_id_bits),
        _stream()))


def tile_order(width, height, ranges, ids, splats, work, order):
    _check("qb_tile_order", lib().qb_tile_order(
        width, height, _ptr(ranges), _ptr(ids), _ptr(splats), _ptr(work), _ptr(order), _stream()))


def render(width, height, ranges, ids, splats, bg, image, final_T=None, n_contrib=None, n_touched=None,
           variant=0, order=None):
    bgv = (C.c_float * 3)(*[float(x) for x in bg])
    _check("qb_render_ex", lib().qb_render_ex(
        width, height, _ptr(ranges), _ptr(ids), _ptr(splats), C.cast(bgv, C.c_void_p), _ptr(image), _ptr(final_T),
        _ptr(n_contrib), _ptr(n_touched), int(variant), _ptr(order), _stream()))


def render_stats(width, height, ranges, ids, splats, bg, image, final_T, n_contrib, n_touched, n_composited,
                 variant=0, order=None):
    """qb_render_stats: the render plus per-pixel counts of the examined and
    the composited list entries."""
    bgv = (C.c_float * 3)(*[float(x) for x in bg])
    _check("qb_render_stats", lib().qb_render_stats(
        width, height, _ptr(ranges), _ptr(ids), _ptr(splats), C.cast(bgv, C.c_void_p), _ptr(image), _ptr(final_T),
        _ptr(n_contrib), _ptr(n_touched), _ptr(n_composited), int(variant), _ptr(order), _stream()))


def render_backward(width, height, ranges, ids, splats, bg, final_T, n_contrib, dl_dimage, n, grad2d, variant=0,
                    order=None):
    _need(n == 0 or min(_rows(grad2d), _rows(splats)) >= n, "qb_render_backward: grad2d/splats hold fewer than n rows")
    bgv = (C.c_float * 3)(*[float(x) for x in bg])
    _check("qb_render_backward_ex", lib().qb_render_backward_ex(
        width, height, _ptr(ranges), _ptr(ids), _ptr(splats), C.cast(bgv, C.c_void_p), _ptr(final_T),
        _ptr(n_contrib), _ptr(dl_dimage), n, _ptr(grad2d), int(variant), _ptr(order), _stream()))


def l1_grad(items):
    """qb_l1_grad over items [(image, target, grad, scale), ...] (float32
    device tensors of one size each): grad = scale * sign(image - target),
    one launch for all items."""
    _need(len(items) <= MAX_VIEWS, f"qb_l1_grad: at most {MAX_VIEWS} items per call")
    arr = (CL1Item * max(len(items), 1))()
    for k, (image, target, grad, scale) in enumerate(items):
        _need(image.numel() == target.numel() == grad.numel(), "qb_l1_grad: image, target and grad differ in size")
        _need(all(t.dtype == torch.float32 and t.is_contiguous() for t in (image, target, grad)),
              "qb_l1_grad: contiguous float32 tensors only")
        arr[k] = CL1Item(image.numel(), image.data_ptr(), target.data_ptr(), grad.data_ptr(), float(scale))
    _check("qb_l1_grad", lib().qb_l1_grad(len(items), arr, _stream()))


def project_backward(g: Gaussians, cam, splats, grad2d, d_means, d_log_scales, d_quats, d_logits, d_sh):
    _need(min(_rows(splats), _rows(grad2d)) >= g.n, "qb_project_backward: splats/grad2d hold fewer than n rows")
    _check("qb_project_backward", lib().qb_project_backward(
        g.n, _ptr(g.means), _ptr(g.log_scales), _ptr(g.quats), _ptr(g.logits), _ptr(g.sh), g.sh_degree,
        C.byref(camera_struct(cam)), _ptr(splats), _ptr(grad2d), _ptr(d_means), _ptr(d_log_scales), _ptr(d_quats),
        _ptr(d_logits), _ptr(d_sh), _stream()))


def check_capacity(num_pairs, capacities, raise_on_overflow=True):
    """qb_check_capacity: waits for the work queued on the current stream,
    returns the pair counts of the frames whose device counts `num_pairs`
    (int64 [count]) holds, and raises QBError(QB_ERR_CAPACITY) when one
    exceeds its capacity (unless raise_on_overflow is False)."""
    caps = [int(c) for c in capacities]
    _need(num_pairs.dtype == torch.int64 and num_pairs.numel() >= len(caps) >= 1, "check_capacity: bad arguments")
    cap_arr = (C.c_int64 * len(caps))(*caps)
    out = (C.c_int64 * len(caps))()
    s = lib().qb_check_capacity(len(caps), _ptr(num_pairs), C.cast(cap_arr, C.c_void_p), C.cast(out, C.c_void_p),
                                _stream())
    if s != QB_ERR_CAPACITY or raise_on_overflow:
        _check("qb_check_capacity", s)
    return list(out)


# ---- whole forward with persistent buffers -------------------------------------

class Rasterizer:
    """Runs project -> intersect -> sort -> render for one camera size,
    keeping device buffers between frames.  The pair buffers grow when a frame
    needs more than the current capacity: with ``sync_count=True`` the pair
    count is read back after qb_intersect (one host synchronisation) and the
    frame's qb_intersect is re-run with enough room; with ``sync_count=False``
    nothing is read back and a frame that overflowed renders empty tiles
    (check ``pairs() <= capacity`` afterwards).  ``write_keys`` selects
    whether the sorted 64-bit keys are materialised (the render needs only
    the sorted ids).  With ``balance`` (the default) the forward runs
    qb_tile_order after the sort and the render and its backward take the
    tiles heaviest first; results are the same either way."""

    def __init__(self, n: int, cam, device="cuda", capacity: int = 0, write_keys: bool = True,
                 balance: bool = True):
        self.n, self.cam, self.device = n, cam, device
        self.generation = 0   # forwards run so far (a backward must follow its own forward)
        self.balance = balance
        self.W, self.H = int(cam.width), int(cam.height)
        self.num_tiles = cam.tiles_x * cam.tiles_y
        self.write_keys = write_keys
        self.mode = "quadbox"
        self.render_variant = RENDER_VARIANTS["2px"]
        self.backward_variant = RENDER_VARIANTS["2px"]
        self.sort_variant = SORT_VARIANTS["512x8"]
        self.depth_variant = DEPTH_VARIANTS["512x4"]
        self.emit_variant = EMIT_VARIANTS["256"]
        # packed pairs (tile << id_bits | id, 4 bytes) where they fit 32 bits
        self.packed = True
        self.id_bits = pair_id_bits(n, self.W, self.H)
        d = device
        self.splats = torch.empty((max(n, 1), SPLAT_FLOATS), dtype=torch.float32, device=d)
        self.rects = torch.empty((max(n, 1), RECT_SHORTS), dtype=torch.int16, device=d)
        self.counts = torch.empty(max(n, 1), dtype=torch.int32, device=d)
        self.depth_keys = torch.empty(max(n, 1), dtype=torch.int32, device=d)
        self.num_pairs = torch.zeros(1, dtype=torch.int64, device=d)
        self.ws_isect = torch.empty(intersect_workspace_size(n), dtype=torch.uint8, device=d)
        self.ranges = torch.empty((self.num_tiles, 2), dtype=torch.int32, device=d)
        self.work = torch.zeros(self.num_tiles, dtype=torch.int32, device=d)
        self.order = torch.arange(self.num_tiles, dtype=torch.int32, device=d)
        self.image = torch.empty((3, self.H, self.W), dtype=torch.float32, device=d)
        self.final_T = torch.empty((self.H, self.W), dtype=torch.float32, device=d)
        self.n_contrib = torch.empty((self.H, self.W), dtype=torch.int32, device=d)
        self.n_touched = None   # set to an int32 [H, W] tensor to count evaluations
        self.capacity = 0
        self._alloc_pairs(capacity)

    def _alloc_pairs(self, cap):
        cap = int(cap)
        c1 = max(cap, 1)
        d = self.device
        self.pair_tiles = torch.empty(c1, dtype=torch.int16, device=d)
        self.pair_ids = torch.empty(c1, dtype=torch.int32, device=d)
        self.keys_sorted = torch.empty(c1, dtype=torch.int64, device=d) if self.write_keys else None
        self.ids_sorted = torch.empty(c1, dtype=torch.int32, device=d)
        self.ws_sort = torch.empty(sort_workspace_size(cap), dtype=torch.uint8, device=d)
        self.capacity = cap

    def use_camera(self, cam):
        """Render later frames from `cam` (same image size: the image, tile
        and range buffers are sized for it)."""
        _need(int(cam.width) == self.W and int(cam.height) == self.H,
              f"camera {cam.width}x{cam.height} does not match the rasterizer's {self.W}x{self.H}")
        self.cam = cam

    def project(self, g: Gaussians, mode):
        _need(g.n == self.n, f"{g.n} Gaussians given to a rasterizer sized for {self.n}")
        project(g, self.cam, mode, self.splats, self.rects, self.counts, self.depth_keys)
        self.mode = mode

    def packed_id_bits(self) -> int:
        """The pair format intersect() and sort() use: id bits of packed
        pairs, or 0 for tiles and ids apart."""
        return self.id_bits if self.packed else 0

    def intersect(self):
        intersect(self.n, self.splats, self.rects, self.counts, self.W, self.H, self.capacity, self.pair_tiles,
                  self.pair_ids, self.num_pairs, self.ws_isect, self.mode, self.depth_variant, self.emit_variant,
                  self.depth_keys, self.packed_id_bits())

    def sort(self):
        sort(self.capacity, self.num_pairs, self.num_tiles, self.pair_tiles, self.pair_ids, self.splats,
             self.keys_sorted, self.ids_sorted, self.ranges, self.ws_sort, self.sort_variant, self.packed_id_bits())

    def schedule(self):
        """qb_tile_order for the sorted frame (a no-op without balance)."""
        if self.balance:
            tile_order(self.W, self.H, self.ranges, self.ids_sorted, self.splats, self.work, self.order)

    def tile_order(self):
        """The order the render takes tiles in (None: row-major)."""
        return self.order if self.balance else None

    def render(self, bg=(0.0, 0.0, 0.0)):
        render(self.W, self.H, self.ranges, self.ids_sorted, self.splats, bg, self.image, self.final_T,
               self.n_contrib, self.n_touched, self.render_variant, self.tile_order())

    def forward(self, g: Gaussians, mode="quadbox", bg=(0.0, 0.0, 0.0), sync_count=True, cam=None):
        """One frame.  With sync_count, the pair count is checked after
        qb_intersect (qb_check_capacity) and the pair buffers grown and the
        intersection re-run when it overflowed; without it nothing is read
        back, and check_capacity() afterwards raises if the frame overflowed
        (it then rendered no Gaussian).  `cam` (same size) replaces the
        rasterizer's camera from this frame on."""
        if cam is not None:
            self.use_camera(cam)
        self.generation += 1
        self.project(g, mode)
        self.intersect()
        if sync_count:
            p = check_capacity(self.num_pairs, [self.capacity], raise_on_overflow=False)[0]
            if p > self.capacity:
                self._alloc_pairs(int(p * 1.1) + 1024)
                self.intersect()
        self.sort()
        self.schedule()
        self.render(bg)
        return self.image

    def pairs(self) -> int:
        return int(self.num_pairs.item())

    def check_capacity(self) -> int:
        """The last frame's pair count; raises QBError(QB_ERR_CAPACITY) when
        it exceeded the pair capacity."""
        return check_capacity(self.num_pairs, [self.capacity])[0]


# ---- autograd ------------------------------------------------------------------

class _Rasterize(torch.autograd.Function):
    """Forward: qb_project -> qb_intersect -> qb_sort -> qb_render.
    Backward: qb_render_backward (in the forward's tile order) ->
    qb_project_backward."""

    @staticmethod
    def forward(ctx, means, log_scales, quats, logits, sh, cam, mode, bg, rast):
        g = Gaussians(tensors=(means.detach(), log_scales.detach(), quats.detach(), logits.detach(), sh.detach()))
        rast.forward(g, mode, bg, cam=cam)
        ctx.rast, ctx.cam, ctx.bg, ctx.g = rast, cam, bg, g
        ctx.generation = rast.generation
        return rast.image.clone()

    @staticmethod
    def backward(ctx, dl_dimage):
        r, g = ctx.rast, ctx.g
        if r.generation != ctx.generation:
            raise RuntimeError("the Rasterizer ran another forward since this one; its backward needs that "
                               "forward's buffers (use one Rasterizer per pending backward)")
        dl = dl_dimage.contiguous().float()
        grad2d = torch.empty((max(g.n, 1), 9), dtype=torch.float32, device=dl.device)
        render_backward(r.W, r.H, r.ranges, r.ids_sorted, r.splats, ctx.bg, r.final_T, r.n_contrib, dl, g.n, grad2d,
                        r.backward_variant, r.tile_order())
        d = [torch.empty_like(t) for t in g.tensors()]
        project_backward(g, ctx.cam, r.splats, grad2d, *d)
        ctx.grad2d = grad2d
        return d[0], d[1], d[2], d[3], d[4], None, None, None, None


def rasterize(means, log_scales, quats, logits, sh, cam, mode="quadbox", bg=(0.0, 0.0, 0.0), rasterizer=None):
    """Differentiable render of one camera: image [3, H, W].  The parameter
    tensors are float32 CUDA tensors in the structure-of-arrays layouts of
    Gaussians; pass a persistent Rasterizer to reuse its buffers."""
    n = int(means.shape[1])
    if rasterizer is None:
        rasterizer = Rasterizer(n, cam, device=means.device, write_keys=False)
    _need(rasterizer.n == n, f"rasterizer sized for {rasterizer.n} Gaussians, {n} given")
    _need(int(cam.width) == rasterizer.W and int(cam.height) == rasterizer.H,
          "camera size differs from the rasterizer's")
    return _Rasterize.apply(means, log_scales, quats, logits, sh, cam, mode, tuple(bg), rasterizer)


# ---- several views of one Gaussian set -----------------------------------------

def project_views(g: Gaussians, cam_array, num_views, mode, splats, rects, counts, depth_keys=None):
    """qb_project_views_ex (depth_keys: [num_views][n] int32, or None)."""
    _check("qb_project_views_ex", lib().qb_project_views_ex(
        g.n, _ptr(g.means), _ptr(g.log_scales), _ptr(g.quats), _ptr(g.logits), _ptr(g.sh), g.sh_degree, cam_array,
        num_views, _mode(mode), _ptr(splats), _ptr(rects), _ptr(counts), _ptr(depth_keys), _stream()))


def tile_order_views(view_array, num_views, work, order):
    _check("qb_tile_order_views", lib().qb_tile_order_views(num_views, view_array, _ptr(work), _ptr(order),
                                                            _stream()))


def render_views(view_array, num_views, bg, variant=0, order=None):
    bgv = (C.c_float * 3)(*[float(x) for x in bg])
    _check("qb_render_views_ex", lib().qb_render_views_ex(num_views, view_array, C.cast(bgv, C.c_void_p),
                                                          int(variant), _ptr(order), _stream()))


def render_backward_views(view_array, num_views, bg, n, variant=0, order=None, accumulate=False):
    """qb_render_backward_views_ex, or with ``accumulate``
    qb_render_backward_views_acc (adds to grad2d, which must hold zeros)."""
    bgv = (C.c_float * 3)(*[float(x) for x in bg])
    name = "qb_render_backward_views_acc" if accumulate else "qb_render_backward_views_ex"
    _check(name, getattr(lib(), name)(num_views, view_array, C.cast(bgv, C.c_void_p), n, int(variant), _ptr(order),
                                      _stream()))


def project_backward_views(g: Gaussians, cam_array, num_views, splats, grad2d, d_means, d_log_scales, d_quats,
                           d_logits, d_sh, clear_grad2d=False):
    """qb_project_backward_views, or with ``clear_grad2d``
    qb_project_backward_views_ex leaving every grad2d row at zero."""
    args = (g.n, _ptr(g.means), _ptr(g.log_scales), _ptr(g.quats), _ptr(g.logits), _ptr(g.sh), g.sh_degree,
            cam_array, num_views, _ptr(splats), _ptr(grad2d), _ptr(d_means), _ptr(d_log_scales), _ptr(d_quats),
            _ptr(d_logits), _ptr(d_sh))
    if clear_grad2d:
        _check("qb_project_backward_views_ex", lib().qb_project_backward_views_ex(*args, 1, _stream()))
    else:
        _check("qb_project_backward_views", lib().qb_project_backward_views(*args, _stream()))


class MultiView:
    """Forward and backward of one Gaussian set seen by up to MAX_VIEWS
    cameras.  Forward: qb_project_views (one launch for all views), then
    qb_intersect and qb_sort per view, then qb_render_views (one launch over
    every tile of every view).  Backward: qb_render_backward_views and
    qb_project_backward_views (gradients summed over views).  The buffers
    persist, so a whole step can be captured in a HIP graph once the pair
    buffers are sized (size_pairs); a frame whose pair count exceeds its
    view's capacity renders that view empty (check overflowed()).  With
    ``balance`` (the default) qb_tile_order_views orders every view's tiles
    in one list, heaviest first, for the render and its backward.  grad2d
    stays all zero between backward calls (the projection backward clears
    the rows it reads), so the render backward adds into it without a
    separate clear."""

    def __init__(self, n: int, cams, device="cuda", streams: int = 4, balance: bool = True):
        self.V = len(cams)
        if not 1 <= self.V <= MAX_VIEWS:
            raise ValueError(f"1..{MAX_VIEWS} views per MultiView")
        self.n, self.cams, self.device = n, list(cams), device
        # the per-view intersect and sort chains are independent: views go
        # round-robin to `streams` side streams (default priority), each with
        # its own workspaces, and join the caller's stream before the render
        self.S = max(1, min(int(streams), self.V))
        self.streams = [torch.cuda.Stream(device=device) for _ in range(self.S)] if self.S > 1 else []
        self.cam_array = (CCamera * self.V)(*[camera_struct(c) for c in cams])
        d, V, n1 = device, self.V, max(n, 1)
        self.splats = torch.empty((V, n1, SPLAT_FLOATS), dtype=torch.float32, device=d)
        self.rects = torch.empty((V, n1, RECT_SHORTS), dtype=torch.int16, device=d)
        self.counts = torch.empty((V, n1), dtype=torch.int32, device=d)
        self.depth_keys = torch.empty((V, n1), dtype=torch.int32, device=d)
        self.num_pairs = torch.zeros(V, dtype=torch.int64, device=d)
        self.ws_isect = [torch.empty(intersect_workspace_size(n), dtype=torch.uint8, device=d) for _ in range(self.S)]
        self.sizes = [(int(c.width), int(c.height)) for c in cams]
        self.num_tiles = [int(c.tiles_x * c.tiles_y) for c in cams]
        self.ranges = [torch.zeros(2 * t, dtype=torch.int32, device=d) for t in self.num_tiles]
        self.images = [torch.zeros((3, h, w), dtype=torch.float32, device=d) for w, h in self.sizes]
        self.final_T = [torch.zeros((h, w), dtype=torch.float32, device=d) for w, h in self.sizes]
        self.n_contrib = [torch.zeros((h, w), dtype=torch.int32, device=d) for w, h in self.sizes]
        self.dl = [torch.zeros((3, h, w), dtype=torch.float32, device=d) for w, h in self.sizes]
        self.grad2d = torch.zeros((V, n1, 9), dtype=torch.float32, device=d)
        self.grad2d_zero = True  # whether grad2d holds only zeros
        self.balance = balance
        total_tiles = sum(self.num_tiles)
        self.work = torch.zeros(total_tiles, dtype=torch.int32, device=d)
        self.order = torch.arange(total_tiles, dtype=torch.int32, device=d)
        self.capacity = [0] * V
        self._groups = []
        self.mode = "quadbox"
        self.render_variant = RENDER_VARIANTS["2px"]
        self.backward_variant = RENDER_VARIANTS["2px"]
        self.sort_variant = SORT_VARIANTS["512x8"]
        self.depth_variant = DEPTH_VARIANTS["512x4"]
        self.emit_variant = EMIT_VARIANTS["256"]
        # per view: packed pairs where tile and id fit 32 bits
        self.packed = True
        self.id_bits = [pair_id_bits(n, w, h) for w, h in self.sizes]
        self.grads = None
        self._table = None

    def _slice(self, v):
        return self.splats[v], self.rects[v], self.counts[v], self.num_pairs[v:v + 1]

    # slot: the side stream the call is issued on, whose workspaces it uses
    # (calls on different streams may run at once; each stream's calls run
    # one after another, so they can share that stream's workspaces)
    def _intersect(self, v, slot=0):
        s, r, c, npairs = self._slice(v)
        w, h = self.sizes[v]
        cap = self.capacity[v]
        intersect(self.n, s, r, c, w, h, cap, self.pair_tiles[v] if cap else None,
                  self.pair_ids[v] if cap else None, npairs, self.ws_isect[slot], self.mode,
                  self.depth_variant, self.emit_variant, self.depth_keys[v], self._packed_bits(v))

    def _packed_bits(self, v):
        return self.id_bits[v] if self.packed else 0

    def _sort(self, v, slot=0):
        sort(self.capacity[v], self.num_pairs[v:v + 1], self.num_tiles[v], self.pair_tiles[v], self.pair_ids[v],
             self.splats[v], None, self.ids_sorted[v], self.ranges[v], self.ws_sort[slot], self.sort_variant,
             self._packed_bits(v))

    def intersect_all(self):
        """qb_intersect of every view (side streams, joined back)."""
        self._per_view(self._intersect)

    def sort_all(self):
        """qb_sort of every view (side streams, joined back)."""
        self._per_view(self._sort)

    def size_pairs(self, g: Gaussians, mode="quadbox", slack=1.1, pad=1024):
        """Runs the projection and counting once (one host synchronisation)
        and sizes every view's pair buffers: count * slack + pad, rounded up
        to 256 pairs."""
        _need(g.n == self.n, f"{g.n} Gaussians given to a MultiView sized for {self.n}")
        self.mode = mode
        self.capacity = [0] * self.V
        project_views(g, self.cam_array, self.V, mode, self.splats, self.rects, self.counts, self.depth_keys)
        for v in range(self.V):
            self._intersect(v)
        counts = self.num_pairs.cpu().tolist()
        # capacities in multiples of 256 pairs keep every view's slice of the
        # flat pair buffers 512-byte aligned
        self.capacity = [(int(p * slack) + int(pad) + 255) // 256 * 256 for p in counts]
        total = sum(self.capacity)
        d = self.device
        flat_t = torch.empty(total, dtype=torch.int16, device=d)
        flat_i = torch.empty(total, dtype=torch.int32, device=d)
        flat_s = torch.empty(total, dtype=torch.int32, device=d)
        self.pair_tiles, self.pair_ids, self.ids_sorted = [], [], []
        o = 0
        for cap in self.capacity:
            self.pair_tiles.append(flat_t[o:o + cap])
            self.pair_ids.append(flat_i[o:o + cap])
            self.ids_sorted.append(flat_s[o:o + cap])
            o += cap
        self._flat = (flat_t, flat_i, flat_s)
        self.ws_sort = [torch.empty(max(sort_workspace_size(c) for c in self.capacity), dtype=torch.uint8, device=d)
                        for _ in range(self.S)]
        views = (CView * self.V)()
        for v in range(self.V):
            w, h = self.sizes[v]
            views[v].width, views[v].height = w, h
            views[v].ranges = self.ranges[v].data_ptr()
            views[v].ids = self.ids_sorted[v].data_ptr()
            views[v].splats = self.splats[v].data_ptr()
            views[v].image = self.images[v].data_ptr()
            views[v].final_T = self.final_T[v].data_ptr()
            views[v].n_contrib = self.n_contrib[v].data_ptr()
            views[v].dL_dimage = self.dl[v].data_ptr()
            views[v].grad2d = self.grad2d[v].data_ptr()
        self._table = views
        self._make_groups()
        return counts

    def _per_view(self, fn):
        """Runs fn(v, slot) for every view, round-robin over the side streams
        (view v on stream slot v % S, forked from and joined back into the
        current stream).  Placing the views longest first on the least loaded
        stream evened the streams' pair counts (within 5 %, against 17 %) but
        made the 32-view step 0.1-0.3 ms slower."""
        if not self.streams:
            for v in range(self.V):
                fn(v, 0)
            return
        main = torch.cuda.current_stream()
        for st in self.streams:
            st.wait_stream(main)
        for v in range(self.V):
            st = v % self.S
            with torch.cuda.stream(self.streams[st]):
                fn(v, st)
        for st in self.streams:
            main.wait_stream(st)

    def forward(self, g: Gaussians, bg=(0.0, 0.0, 0.0)):
        if self._table is None:
            raise RuntimeError("call size_pairs() first")
        _need(g.n == self.n, f"{g.n} Gaussians given to a MultiView sized for {self.n}")
        project_views(g, self.cam_array, self.V, self.mode, self.splats, self.rects, self.counts, self.depth_keys)

        def prep(v, slot):
            self._intersect(v, slot)
            self._sort(v, slot)

        self._per_view(prep)
        if self.balance:
            tile_order_views(self._table, self.V, self.work, self.order)
        self.render(bg)
        return self.images

    def tile_order(self):
        """The order the render takes global tiles in (None: row-major)."""
        return self.order if self.balance else None

    def render(self, bg=(0.0, 0.0, 0.0)):
        render_views(self._table, self.V, bg, self.render_variant, self.tile_order())

    def backward(self, g: Gaussians, bg=(0.0, 0.0, 0.0)):
        """Gradients of sum over views of <dl[v], image[v]> (fill self.dl
        first); returns (d_means, d_log_scales, d_quats, d_logits, d_sh)."""
        if self.grads is None:
            self.grads = [torch.empty_like(t) for t in g.tensors()]
        render_backward_views(self._table, self.V, bg, self.n, self.backward_variant, self.tile_order(),
                              accumulate=self.grad2d_zero)
        project_backward_views(g, self.cam_array, self.V, self.splats, self.grad2d, *self.grads, clear_grad2d=True)
        self.grad2d_zero = True
        return self.grads

    def _make_groups(self):
        """step()'s groups: per side stream, its views (v % S == slot), their
        view table and the work / order buffers of their tiles."""
        self._groups = []
        for slot in range(self.S if self.streams else 0):
            vs = [v for v in range(self.V) if v % self.S == slot]
            tiles = sum(self.num_tiles[v] for v in vs)
            self._groups.append((vs, (CView * len(vs))(*[self._table[v] for v in vs]),
                                 torch.zeros(tiles, dtype=torch.int32, device=self.device),
                                 torch.arange(tiles, dtype=torch.int32, device=self.device)))

    def step(self, g: Gaussians, targets, bg=(0.0, 0.0, 0.0)):
        """One training step over every view: forward, dL/dimage of the mean
        absolute error against targets[v] (qb_l1_grad, scale 1 / element
        count, into dl[v]) and backward; returns the gradients as backward()
        does.  Each side stream renders, takes the loss gradient of and runs
        the render backward of its own views (v % S == slot) right behind
        their intersections and sorts, so the streams that finish their sorts
        first start on this work while the others still sort; the projection
        backward then sums every view on the current stream.  Images, dl and
        gradients are those of forward(), l1_grad() and backward() in turn,
        the rounding of the render backward's float atomics aside (tiles are
        ordered within each stream's views rather than over all views).
        Without side streams: forward(), l1_grad() and backward()."""
        if self._table is None:
            raise RuntimeError("call size_pairs() first")
        _need(len(targets) == self.V, f"{len(targets)} targets for {self.V} views")
        if not self.streams:
            self.forward(g, bg)
            l1_grad([(self.images[v], targets[v], self.dl[v], 1.0 / self.images[v].numel()) for v in range(self.V)])
            return self.backward(g, bg)
        _need(g.n == self.n, f"{g.n} Gaussians given to a MultiView sized for {self.n}")
        if self.grads is None:
            self.grads = [torch.empty_like(t) for t in g.tensors()]
        project_views(g, self.cam_array, self.V, self.mode, self.splats, self.rects, self.counts, self.depth_keys)
        main = torch.cuda.current_stream()
        for st in self.streams:
            st.wait_stream(main)
        # every view's intersection and sort first, round-robin, then each
        # stream's render chain behind its own sorts
        for v in range(self.V):
            slot = v % self.S
            with torch.cuda.stream(self.streams[slot]):
                self._intersect(v, slot)
                self._sort(v, slot)
        accumulate = self.grad2d_zero
        for slot, (vs, table, work, order) in enumerate(self._groups):
            with torch.cuda.stream(self.streams[slot]):
                o = None
                if self.balance:
                    tile_order_views(table, len(vs), work, order)
                    o = order
                render_views(table, len(vs), bg, self.render_variant, o)
                l1_grad([(self.images[v], targets[v], self.dl[v], 1.0 / self.images[v].numel()) for v in vs])
                render_backward_views(table, len(vs), bg, self.n, self.backward_variant, o, accumulate=accumulate)
        for st in self.streams:
            main.wait_stream(st)
        project_backward_views(g, self.cam_array, self.V, self.splats, self.grad2d, *self.grads, clear_grad2d=True)
        self.grad2d_zero = True
        return self.grads

    def overflowed(self) -> bool:
        """Whether a view of the last step had more pairs than its capacity
        (that view then rendered no Gaussian and got no gradient)."""
        counts = check_capacity(self.num_pairs, self.capacity, raise_on_overflow=False)
        return any(p > c for p, c in zip(counts, self.capacity))

    def check_capacity(self):
        """Per-view pair counts of the last step; raises
        QBError(QB_ERR_CAPACITY) when a view overflowed (call once per step,
        outside a graph capture, e.g. after each replay; re-size with
        size_pairs and capture again on overflow)."""
        return check_capacity(self.num_pairs, self.capacity)


# ---- autotuner -----------------------------------------------------------------

def _interleaved_best(fns, reps, trials):
    """{name: best ms per call} of every callable in `fns`, each run once
    untimed first; the timed trials go round-robin over the callables so
    that a clock ramp or drift during tuning falls on every shape alike
    rather than on the one timed first."""
    for fn in fns.values():
        fn()
    torch.cuda.synchronize()
    best = {name: float("inf") for name in fns}
    for _ in range(trials):
        for name, fn in fns.items():
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                fn()
            e1.record()
            torch.cuda.synchronize()
            best[name] = min(best[name], e0.elapsed_time(e1) / reps)
    return best


def autotune_backward(run, bg=(0.0, 0.0, 0.0), dl=None, grad2d=None, reps=5, trials=3):
    """Times every launch shape of the render backward on the frame `run`
    holds -- a MultiView after forward with its dl filled, or a Rasterizer
    after forward given dl [3, H, W] and a grad2d [n, 9] buffer -- keeps the
    fastest in run.backward_variant and returns {shape: ms}."""
    fns = {}
    for name, v in BACKWARD_VARIANTS.items():
        if isinstance(run, MultiView):
            # timed without the clear; the sums these calls leave in grad2d
            # make the next backward clear it
            run.grad2d_zero = False
            fns[name] = (lambda v=v: render_backward_views(run._table, run.V, bg, run.n, v, run.tile_order(),
                                                           accumulate=True))
        else:
            fns[name] = (lambda v=v: render_backward(run.W, run.H, run.ranges, run.ids_sorted, run.splats, bg,
                                                     run.final_T, run.n_contrib, dl, run.n, grad2d, v,
                                                     run.tile_order()))
    times = _interleaved_best(fns, reps, trials)
    pick = min(times, key=times.get)
    run.backward_variant = BACKWARD_VARIANTS[pick]
    return times


def autotune_render(run, bg=(0.0, 0.0, 0.0), reps=10, trials=3):
    """Times every render launch shape on the frame `run` (a Rasterizer or a
    MultiView after a forward) holds, keeps the fastest in
    run.render_variant and returns {shape: ms}.  The shapes give identical
    images, so the choice only affects speed."""
    def shape(v):
        def fn():
            run.render_variant = v
            run.render(bg)
        return fn

    times = _interleaved_best({name: shape(v) for name, v in RENDER_VARIANTS.items()}, reps, trials)
    pick = min(times, key=times.get)
    run.render_variant = RENDER_VARIANTS[pick]
    run.render(bg)
    return times


def autotune_sort(run, reps=5, trials=3):
    """Times every tile-sort launch shape on the pairs `run` (a Rasterizer or
    a MultiView after a forward) holds, keeps the fastest in run.sort_variant
    and returns {shape: ms} (per frame: every view's sort for a MultiView).
    The shapes give identical lists, so the choice only affects speed."""
    def shape(v):
        def fn():
            run.sort_variant = v
            if isinstance(run, MultiView):
                run.sort_all()
            else:
                run.sort()
        return fn

    times = _interleaved_best({name: shape(v) for name, v in SORT_VARIANTS.items()}, reps, trials)
    run.sort_variant = SORT_VARIANTS[min(times, key=times.get)]
    shape(run.sort_variant)()
    return times


def autotune_intersect(run, reps=5, trials=3):
    """Times every pair of depth-sort and emission launch shapes of
    qb_intersect on the frame `run` (a Rasterizer or a MultiView after a
    forward) holds, keeps the fastest in run.depth_variant /
    run.emit_variant and returns {"depth/emit": ms}.  Every pair writes the
    same pairs; the sort and render are left as they were (the frame's
    pairs are rewritten identically)."""
    def shape(dv, ev):
        def fn():
            run.depth_variant, run.emit_variant = dv, ev
            if isinstance(run, MultiView):
                run.intersect_all()
            else:
                run.intersect()
        return fn

    fns = {f"{dn}/{en}": shape(dv, ev) for dn, dv in DEPTH_VARIANTS.items() for en, ev in EMIT_VARIANTS.items()}
    times = _interleaved_best(fns, reps, trials)
    dn, en = min(times, key=times.get).split("/")
    shape(DEPTH_VARIANTS[dn], EMIT_VARIANTS[en])()
    return times
