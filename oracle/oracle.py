"""ctypes view of the C oracle (test infrastructure only).

Every function mirrors one routine of ``quadbox_oracle.c``; arrays are numpy.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

BOX_3SIGMA, BOX_ADR, BOX_QUADBOX, BOX_DUALBOX = 0, 1, 2, 3
# "quadbox_naive" (the ablation without QPass, Sec. 3.2) only changes how the
# tiles are enumerated; its tile set is the QuadBox union by definition.
CLIP_3SIGMA = 16   # added to an opacity-aware mode: sub-box tile rects cut to the 3-sigma square's
MODES = {"3sigma": BOX_3SIGMA, "adr": BOX_ADR, "quadbox": BOX_QUADBOX, "dualbox": BOX_DUALBOX,
         "quadbox_naive": BOX_QUADBOX, "quadbox_clip3sigma": BOX_QUADBOX | CLIP_3SIGMA,
         "adr_clip3sigma": BOX_ADR | CLIP_3SIGMA, "dualbox_clip3sigma": BOX_DUALBOX | CLIP_3SIGMA,
         "quadbox_naive_clip3sigma": BOX_QUADBOX | CLIP_3SIGMA}
TILE = 16

GAUSS_DTYPE = np.dtype({
    "names": ["u", "v", "depth", "A", "B", "C", "a", "b", "c", "opacity", "gamma",
              "visible", "nrect", "rect", "rgb"],
    "formats": ["<f4"] * 11 + ["<i4", "<i4", ("<i4", (4, 4)), ("<f8", (3,))],
    "offsets": [0, 4, 8, 12, 16, 20, 24, 28, 32, 36, 40, 44, 48, 52, 120],
    "itemsize": 144,
})


class _Cam(C.Structure):
    _fields_ = [("W", C.c_int32), ("H", C.c_int32), ("fx", C.c_float), ("fy", C.c_float),
                ("cx", C.c_float), ("cy", C.c_float), ("near_plane", C.c_float),
                ("R", C.c_float * 9), ("t", C.c_float * 3), ("campos", C.c_float * 3)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path):
            _build.build()
        L = C.CDLL(path)
        vp, i64, i32, dbl = C.c_void_p, C.c_int64, C.c_int32, C.c_double
        L.oc_project.argtypes = [vp, i64, vp, vp, vp, vp, vp, i32, i32, vp]
        L.oc_build_boxes.argtypes = [vp, i32, i32, i32]
        L.oc_tile_set.argtypes = [vp, i32, vp]
        L.oc_tile_set.restype = i64
        L.oc_tile_counts.argtypes = [vp, i64, i32, vp]
        L.oc_pairs.argtypes = [vp, i64, i32, i64, vp, vp]
        L.oc_pairs.restype = i64
        L.oc_ranges.argtypes = [vp, i64, i32, vp]
        L.oc_tile_list.argtypes = [vp, i64, i32, i64, vp]
        L.oc_tile_list.restype = i64
        L.oc_render.argtypes = [vp, i32, i32, vp, vp, vp, dbl, vp, vp, vp, vp]
        L.oc_render_pixels.argtypes = [vp, i64, i32, i64, vp, vp, dbl, vp, vp, vp, vp]
        L.oc_render_brute.argtypes = [vp, i64, i32, i32, vp, dbl, vp, vp, vp, vp]
        L.oc_coverage_audit.argtypes = [vp, i64, i32, i32, dbl, vp, vp, i64]
        L.oc_coverage_audit.restype = i64
        L.oc_sh_basis.argtypes = [dbl, dbl, dbl, vp]
        L.oc_power.argtypes = [vp, C.c_float, C.c_float]
        L.oc_power.restype = C.c_float
        L.oc_layout.argtypes = [vp]
        L.oc_forward64.argtypes = [vp, i64, vp, vp, vp, vp, vp, i32, vp, i64, i32, dbl, vp]
        L.oc_backward64.argtypes = [vp, i64, vp, vp, vp, vp, vp, i32, vp, vp, dbl, vp, vp, vp]
        L.oc_pixel_boxes.argtypes = [vp, i32, vp]
        L.oc_pixel_boxes.restype = i32
        L.oc_project64.argtypes = [vp, i64, vp, vp, vp, vp, vp, i32, vp]
        L.oc_activations.argtypes = [i64, vp, i32, vp]
        L.oc_set_threads.argtypes = [i32]
        L.oc_threads.restype = i32
        lay = np.zeros(6, np.int64)
        L.oc_layout(lay.ctypes.data)
        assert lay[0] == GAUSS_DTYPE.itemsize and lay[1] == 44 and lay[2] == 48
        assert lay[3] == 52 and lay[4] == 120 and lay[5] == C.sizeof(_Cam), lay
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data


ACTIVATIONS = {"scale": 0, "opacity": 1, "gamma": 2}


def activations(x, which):
    """Activation `which` ("scale": exp, "opacity": sigmoid, "gamma":
    2 ln(255 o)) of every binary32 in x, each evaluated in binary64 and
    rounded once, exactly as the projection evaluates it (Eq. (3) for
    gamma)."""
    x = np.ascontiguousarray(x, np.float32)
    out = np.empty_like(x)
    lib().oc_activations(x.size, _p(x), ACTIVATIONS[which], _p(out))
    return out


def set_threads(t: int) -> None:
    """Worker threads of the oracle's parallel loops."""
    lib().oc_set_threads(int(t))


def threads() -> int:
    return int(lib().oc_threads())


def camera_struct(cam) -> _Cam:
    c = _Cam()
    c.W, c.H = cam.width, cam.height
    c.fx, c.fy, c.cx, c.cy, c.near_plane = cam.fx, cam.fy, cam.cx, cam.cy, cam.near
    R = np.asarray(cam.R, np.float32).reshape(9)
    t = np.asarray(cam.t, np.float32).reshape(3)
    p = np.asarray(cam.campos, np.float32).reshape(3)
    for k in range(9):
        c.R[k] = float(R[k])
    for k in range(3):
        c.t[k] = float(t[k])
        c.campos[k] = float(p[k])
    return c


def project(scene, cam, mode) -> np.ndarray:
    """Per-Gaussian projection, boxes and tile rects (structured array)."""
    mode = MODES[mode] if isinstance(mode, str) else int(mode)
    n = scene.n
    out = np.zeros(n, GAUSS_DTYPE)
    cs = camera_struct(cam)
    arrs = [np.ascontiguousarray(x, np.float32) for x in
            (scene.means, scene.log_scales, scene.quats, scene.logits, scene.sh)]
    lib().oc_project(C.byref(cs), n, *[_p(a) for a in arrs], scene.sh_degree, mode, _p(out))
    return out


def build_boxes(g: np.ndarray, mode, W: int, H: int) -> np.ndarray:
    """Re-run the box construction on records whose u, v, A, B, C, gamma are set."""
    mode = MODES[mode] if isinstance(mode, str) else int(mode)
    g = np.ascontiguousarray(g.copy())
    for i in range(len(g)):
        lib().oc_build_boxes(g.ctypes.data + i * g.itemsize, mode, W, H)
    return g


def tile_set(g: np.ndarray, i: int, tiles_x: int) -> np.ndarray:
    rec = np.ascontiguousarray(g[i:i + 1])
    m = lib().oc_tile_set(_p(rec), tiles_x, None)
    out = np.zeros(max(m, 1), np.int64)
    lib().oc_tile_set(_p(rec), tiles_x, _p(out))
    return out[:m]


def tile_counts(g: np.ndarray, tiles_x: int) -> np.ndarray:
    out = np.zeros(len(g), np.int64)
    lib().oc_tile_counts(_p(g), len(g), tiles_x, _p(out))
    return out


def pairs(g: np.ndarray, tiles_x: int):
    """Sorted (key, id) pair list."""
    total = int(tile_counts(g, tiles_x).sum())
    keys = np.zeros(max(total, 1), np.uint64)
    ids = np.zeros(max(total, 1), np.uint32)
    got = lib().oc_pairs(_p(g), len(g), tiles_x, total, _p(keys), _p(ids))
    assert got == total
    return keys[:total], ids[:total]


def ranges(keys: np.ndarray, num_tiles: int) -> np.ndarray:
    out = np.zeros((num_tiles, 2), np.uint32)
    keys = np.ascontiguousarray(keys, np.uint64)
    lib().oc_ranges(_p(keys), len(keys), num_tiles, _p(out))
    return out


def tile_list(g: np.ndarray, tiles_x: int, tile: int) -> np.ndarray:
    out = np.zeros(max(len(g), 1), np.uint32)
    m = lib().oc_tile_list(_p(g), len(g), tiles_x, tile, _p(out))
    return out[:m]


def render(g, W, H, rng_tbl, ids, bg=(0.0, 0.0, 0.0), band=1e-4):
    """Tiled render over the sorted list; returns image[3,H,W], T, n_contrib, near mask."""
    bgv = np.asarray(bg, np.float64)
    img = np.zeros((3, H, W), np.float64)
    T = np.zeros((H, W), np.float64)
    nc = np.zeros((H, W), np.uint32)
    near = np.zeros((H, W), np.uint8)
    rng_tbl = np.ascontiguousarray(rng_tbl, np.uint32)
    ids = np.ascontiguousarray(ids if len(ids) else np.zeros(1, np.uint32), np.uint32)
    lib().oc_render(_p(g), W, H, _p(rng_tbl), _p(ids), _p(bgv), band, _p(img), _p(T), _p(nc), _p(near))
    return img, T, nc, near.astype(bool)


def render_pixels(g, W, pix, bg=(0.0, 0.0, 0.0), band=1e-4):
    """Render selected pixels [(x, y), ...] from per-tile lists built directly."""
    pix = np.ascontiguousarray(pix, np.int32).reshape(-1, 2)
    bgv = np.asarray(bg, np.float64)
    k = len(pix)
    rgb = np.zeros((k, 3), np.float64)
    T = np.zeros(k, np.float64)
    nc = np.zeros(k, np.uint32)
    near = np.zeros(k, np.uint8)
    lib().oc_render_pixels(_p(g), len(g), W, k, _p(pix), _p(bgv), band, _p(rgb), _p(T), _p(nc), _p(near))
    return rgb, T, nc, near.astype(bool)


def render_brute(g, W, H, bg=(0.0, 0.0, 0.0), band=1e-4):
    bgv = np.asarray(bg, np.float64)
    img = np.zeros((3, H, W), np.float64)
    T = np.zeros((H, W), np.float64)
    nc = np.zeros((H, W), np.uint32)
    near = np.zeros((H, W), np.uint8)
    lib().oc_render_brute(_p(g), len(g), W, H, _p(bgv), band, _p(img), _p(T), _p(nc), _p(near))
    return img, T, nc, near.astype(bool)


def coverage_audit(g, W, H, margin=2e-3, max_missed=1024):
    """(missed pairs, exact-sample pair count, ids of missed Gaussians)."""
    exact = np.zeros(1, np.int64)
    ids = np.zeros(max_missed, np.int64)
    missed = lib().oc_coverage_audit(_p(g), len(g), W, H, margin, _p(exact), _p(ids), max_missed)
    return int(missed), int(exact[0]), ids[:min(missed, max_missed)]


def sh_basis(x, y, z) -> np.ndarray:
    out = np.zeros(16, np.float64)
    lib().oc_sh_basis(float(x), float(y), float(z), _p(out))
    return out


def power(rec, px, py) -> np.float32:
    r = np.ascontiguousarray(np.asarray(rec).reshape(1).astype(GAUSS_DTYPE))
    return np.float32(lib().oc_power(_p(r), float(px), float(py)))


def forward(scene, cam, mode="quadbox", bg=(0.0, 0.0, 0.0), band=1e-4):
    """Whole oracle forward: project, pairs, ranges, render."""
    g = project(scene, cam, mode)
    keys, ids = pairs(g, cam.tiles_x)
    rt = ranges(keys, cam.num_tiles)
    img, T, nc, near = render(g, cam.width, cam.height, rt, ids, bg, band)
    return dict(g=g, keys=keys, ids=ids, ranges=rt, image=img, T=T, n_contrib=nc, near=near)


def pixel_boxes(rec, mode) -> np.ndarray:
    """Pixel-space boxes [k, (x0, x1, y0, y1)] of one record."""
    mode = MODES[mode] if isinstance(mode, str) else int(mode)
    r = np.ascontiguousarray(np.asarray(rec).reshape(1).astype(GAUSS_DTYPE))
    out = np.zeros((4, 4), np.float32)
    nb = lib().oc_pixel_boxes(_p(r), mode, _p(out))
    return out[:nb]


PARAMS_PER_GAUSSIAN = 59   # mean 3, log_scale 3, quat 4, logit 1, sh 48 (coefficient k*3 + ch)
GROUPS = {"means": slice(0, 3), "log_scales": slice(3, 6), "quats": slice(6, 10), "logits": slice(10, 11),
          "sh": slice(11, 59)}


def _scene_arrays(scene):
    return [np.ascontiguousarray(x, np.float32) for x in
            (scene.means, scene.log_scales, scene.quats, scene.logits, scene.sh)]


def forward64(scene, cam, bg=(0.0, 0.0, 0.0), pert=None) -> np.ndarray:
    """Binary64 image [3, H, W]; pert = (gaussian, parameter index, step)."""
    L = lib()
    arrs = _scene_arrays(scene)
    cs = camera_struct(cam)
    bgv = np.asarray(bg, np.float64)
    img = np.zeros((3, cam.height, cam.width), np.float64)
    pi, pp, ph = pert if pert is not None else (-1, 0, 0.0)
    L.oc_forward64(C.byref(cs), scene.n, *[_p(a) for a in arrs], scene.sh_degree, _p(bgv), pi, pp, ph, _p(img))
    return img


PROJ64_FIELDS = ("visible", "u", "v", "depth", "A", "B", "C", "a", "b", "c", "opacity", "gamma", "r", "g", "b_")


def project64(scene, cam) -> dict:
    """The binary64 projection behind forward64/backward64: {field: [N]}."""
    arrs = _scene_arrays(scene)
    cs = camera_struct(cam)
    out = np.zeros((scene.n, 16), np.float64)
    lib().oc_project64(C.byref(cs), scene.n, *[_p(a) for a in arrs], scene.sh_degree, _p(out))
    return {f: out[:, k] for k, f in enumerate(PROJ64_FIELDS)}


def backward64(scene, cam, dl_dimg, bg=(0.0, 0.0, 0.0), band=1e-4, with_near=False, with_2d=False):
    """Gradient [N, 59] of sum(dl_dimg * forward64(...)) by reverse mode.
    with_near: also return the [H, W] mask of pixels (among those with a
    non-zero dl_dimg) whose stop test or 0.99 cap came within `band`
    (relative) of its threshold.  with_2d: also return the gradient [N, 9]
    with respect to the projected quantities (u v a b c o r g b)."""
    L = lib()
    arrs = _scene_arrays(scene)
    cs = camera_struct(cam)
    bgv = np.asarray(bg, np.float64)
    dl = np.ascontiguousarray(dl_dimg, np.float64)
    out = np.zeros((scene.n, PARAMS_PER_GAUSSIAN), np.float64)
    near = np.zeros((cam.height, cam.width), np.uint8)
    g2 = np.zeros((scene.n, 9), np.float64)
    L.oc_backward64(C.byref(cs), scene.n, *[_p(a) for a in arrs], scene.sh_degree, _p(bgv), _p(dl), band,
                    _p(near), _p(out), _p(g2))
    res = (out,)
    if with_near:
        res += (near.astype(bool),)
    if with_2d:
        res += (g2,)
    return res if len(res) > 1 else out
