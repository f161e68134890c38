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

BOX_MODES = {"3sigma": 0, "adr": 1, "quadbox": 2, "dualbox": 3}
TILE = 16
SPLAT_FLOATS = 12   # qb_splat: u v depth o | a b c gamma | r g b visible
RECT_SHORTS = 16    # qb_rects: 4 x (tx0, tx1, ty0, ty1)

QB_OK, QB_ERR_INVALID_ARG, QB_ERR_CAPACITY, QB_ERR_HIP, QB_ERR_UNSUPPORTED = 0, -1, -2, -3, -4


class QBError(RuntimeError):
    def __init__(self, fn, status):
        super().__init__(f"{fn} failed: {status_string(status)} ({status})")
        self.status = status


class CCamera(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("fx", C.c_float), ("fy", C.c_float),
                ("cx", C.c_float), ("cy", C.c_float), ("near_plane", C.c_float),
                ("R", C.c_float * 9), ("t", C.c_float * 3), ("campos", C.c_float * 3)]


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
    L.qb_intersect_workspace_size.argtypes = [i64]
    L.qb_intersect_workspace_size.restype = sz
    L.qb_intersect.argtypes = [i64, vp, vp, vp, i32, i32, i64, vp, vp, vp, vp, sz, vp]
    L.qb_intersect.restype = i32
    L.qb_sort_workspace_size.argtypes = [i64]
    L.qb_sort_workspace_size.restype = sz
    L.qb_sort.argtypes = [i64, vp, i32, vp, vp, vp, vp, vp, vp, vp, sz, vp]
    L.qb_sort.restype = i32
    L.qb_render.argtypes = [i32, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    L.qb_render.restype = i32
    L.qb_status_string.argtypes = [i32]
    L.qb_status_string.restype = C.c_char_p
    L.qb_version.argtypes = []
    L.qb_version.restype = i32
    _lib = L
    return L


def status_string(s: int) -> str:
    return lib().qb_status_string(int(s)).decode()


def _check(fn, s):
    if s != QB_OK:
        raise QBError(fn, s)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


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

    def __init__(self, scene, device="cuda"):
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


# ---- one call per ABI entry point --------------------------------------------

def project(g: Gaussians, cam, mode, splats, rects, counts):
    _check("qb_project", lib().qb_project(
        g.n, _ptr(g.means), _ptr(g.log_scales), _ptr(g.quats), _ptr(g.logits), _ptr(g.sh), g.sh_degree,
        C.byref(camera_struct(cam)), _mode(mode), _ptr(splats), _ptr(rects), _ptr(counts), _stream()))


def intersect_workspace_size(n: int) -> int:
    return int(lib().qb_intersect_workspace_size(n))


def intersect(n, splats, rects, counts, width, height, capacity, pair_tiles, pair_ids, num_pairs, ws):
    _check("qb_intersect", lib().qb_intersect(
        n, _ptr(splats), _ptr(rects), _ptr(counts), width, height, capacity, _ptr(pair_tiles), _ptr(pair_ids),
        _ptr(num_pairs), _ptr(ws), ws.numel() * ws.element_size(), _stream()))


def sort_workspace_size(capacity: int) -> int:
    return int(lib().qb_sort_workspace_size(capacity))


def sort(capacity, num_pairs, num_tiles, pair_tiles, pair_ids, splats, keys, ids, ranges, ws):
    _check("qb_sort", lib().qb_sort(
        capacity, _ptr(num_pairs), num_tiles, _ptr(pair_tiles), _ptr(pair_ids), _ptr(splats), _ptr(keys),
        _ptr(ids), _ptr(ranges), _ptr(ws), ws.numel() * ws.element_size(), _stream()))


def render(width, height, ranges, ids, splats, bg, image, final_T=None, n_contrib=None, n_touched=None):
    bgv = (C.c_float * 3)(*[float(x) for x in bg])
    _check("qb_render", lib().qb_render(
        width, height, _ptr(ranges), _ptr(ids), _ptr(splats), C.cast(bgv, C.c_void_p), _ptr(image),
        _ptr(final_T), _ptr(n_contrib), _ptr(n_touched), _stream()))


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
    the sorted ids)."""

    def __init__(self, n: int, cam, device="cuda", capacity: int = 0, write_keys: bool = True):
        self.n, self.cam, self.device = n, cam, device
        self.W, self.H = int(cam.width), int(cam.height)
        self.num_tiles = cam.tiles_x * cam.tiles_y
        self.write_keys = write_keys
        d = device
        self.splats = torch.empty((max(n, 1), SPLAT_FLOATS), dtype=torch.float32, device=d)
        self.rects = torch.empty((max(n, 1), RECT_SHORTS), dtype=torch.int16, device=d)
        self.counts = torch.empty(max(n, 1), dtype=torch.int32, device=d)
        self.num_pairs = torch.zeros(1, dtype=torch.int64, device=d)
        self.ws_isect = torch.empty(intersect_workspace_size(n), dtype=torch.uint8, device=d)
        self.ranges = torch.empty((self.num_tiles, 2), dtype=torch.int32, device=d)
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

    def project(self, g: Gaussians, mode):
        project(g, self.cam, mode, self.splats, self.rects, self.counts)

    def intersect(self):
        intersect(self.n, self.splats, self.rects, self.counts, self.W, self.H, self.capacity, self.pair_tiles,
                  self.pair_ids, self.num_pairs, self.ws_isect)

    def sort(self):
        sort(self.capacity, self.num_pairs, self.num_tiles, self.pair_tiles, self.pair_ids, self.splats,
             self.keys_sorted, self.ids_sorted, self.ranges, self.ws_sort)

    def render(self, bg=(0.0, 0.0, 0.0)):
        render(self.W, self.H, self.ranges, self.ids_sorted, self.splats, bg, self.image, self.final_T,
               self.n_contrib, self.n_touched)

    def forward(self, g: Gaussians, mode="quadbox", bg=(0.0, 0.0, 0.0), sync_count=True):
        self.project(g, mode)
        self.intersect()
        if sync_count:
            p = int(self.num_pairs.item())
            if p > self.capacity:
                self._alloc_pairs(int(p * 1.1) + 1024)
                self.intersect()
        self.sort()
        self.render(bg)
        return self.image

    def pairs(self) -> int:
        return int(self.num_pairs.item())
