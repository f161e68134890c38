"""Pins of the oracle's box construction (Sec. 3.1) and tile sets (Sec. 3.2)
against facts that do not come from the oracle itself: brute-force sampling of
the ellipse boundary (the support function of Eq. (8)), the exact pixel-sample
coverage of the 1/255 region (conservativeness), special cases and set
inclusions stated by the paper."""
import math

import numpy as np
import pytest

from paper_2605_04844_amd import scenes


def rec(O, u, v, A, B, C, gamma):
    r = np.zeros(1, O.GAUSS_DTYPE)
    r["u"], r["v"], r["A"], r["B"], r["C"], r["gamma"] = u, v, A, B, C, gamma
    det = A * C - B * B
    r["a"], r["b"], r["c"] = C / det, -B / det, A / det
    r["opacity"] = math.exp(gamma / 2.0) / 255.0
    r["visible"] = 1
    return r


def boundary(A, B, C, gamma, n=400_000):
    """Points of {d : d^T Sigma^-1 d = gamma} as sqrt(gamma) L (cos t, sin t),
    Sigma = L L^T (Cholesky), in float64; centred at the origin."""
    L = np.linalg.cholesky(np.array([[A, B], [B, C]], np.float64))
    t = np.linspace(0.0, 2.0 * np.pi, n, endpoint=False)
    # add the parameters where the curve crosses the axes (x = 0 at t = +-pi/2
    # since L is lower triangular; y = 0 where L10 cos t + L11 sin t = 0), so the
    # quadrant pieces' end points are sampled exactly
    ty = math.atan2(-L[1, 0], L[1, 1])
    t = np.concatenate([t, [0.5 * np.pi, 1.5 * np.pi, ty, ty + np.pi]])
    return math.sqrt(gamma) * (L @ np.stack([np.cos(t), np.sin(t)]))


def random_cov(rng):
    """Random SPD Sigma2D with axis ratio up to 100 and any orientation."""
    l1 = math.exp(rng.uniform(-1.0, 6.0))
    l2 = l1 / math.exp(rng.uniform(0.0, math.log(100.0 ** 2)))
    th = rng.uniform(0.0, np.pi)
    c, s = math.cos(th), math.sin(th)
    Rm = np.array([[c, -s], [s, c]])
    S = Rm @ np.diag([l1, l2]) @ Rm.T
    S = S.astype(np.float32).astype(np.float64)
    if S[0, 0] * S[1, 1] - S[0, 1] ** 2 <= 0:
        return random_cov(rng)
    return S[0, 0], S[0, 1], S[1, 1]


def test_adr_extents_equal_support_function(oracle):
    """AdR half extents equal max_d d_x and max_d d_y over the ellipse boundary (Eqs. (8), (9))."""
    rng = np.random.default_rng(11)
    for _ in range(200):
        A, B, C = random_cov(rng)
        gamma = float(np.float32(rng.uniform(0.1, 11.0)))
        u, v = rng.uniform(-50, 300, 2)
        r = rec(oracle, u, v, A, B, C, gamma)
        box = oracle.pixel_boxes(r, "adr")[0]
        pts = boundary(A, B, C, gamma)
        u32, v32 = float(r["u"][0]), float(r["v"][0])
        xm_true, ym_true = pts[0].max(), pts[1].max()
        scale = max(abs(u32), abs(v32), xm_true, ym_true)
        assert abs((box[1] - u32) - xm_true) <= 1e-6 * xm_true + 4e-7 * scale
        assert abs((u32 - box[0]) - xm_true) <= 1e-6 * xm_true + 4e-7 * scale
        assert abs((box[3] - v32) - ym_true) <= 1e-6 * ym_true + 4e-7 * scale
        assert abs((v32 - box[2]) - ym_true) <= 1e-6 * ym_true + 4e-7 * scale


def test_quadbox_boxes_are_tight_quadrant_aabbs(oracle):
    """Each QuadBox sub-box is the tight AABB of the part of the filled ellipse
    in its quadrant: the two major-axis quadrants reach (x_max, y_max) and the
    other two reach the axis intercepts (Eqs. (5), (6), (12)).  A wrong
    quadrant choice or a wrong stretching factor fails here."""
    rng = np.random.default_rng(12)
    for trial in range(300):
        A, B, C = random_cov(rng)
        if trial % 7 == 0:
            B = -B
        gamma = float(np.float32(rng.uniform(0.5, 11.0)))
        r = rec(oracle, 0.0, 0.0, A, B, C, gamma)
        boxes = oracle.pixel_boxes(r, "quadbox")
        assert boxes.shape == (4, 4)
        pts = boundary(A, B, C, gamma)
        for bx in boxes:
            sx = 1 if bx[0] == 0.0 else -1
            sy = 1 if bx[2] == 0.0 else -1
            assert (bx[1] == 0.0) == (sx < 0) and (bx[3] == 0.0) == (sy < 0)
            tol = 1e-12 * np.abs(pts).max()
            sel = (sx * pts[0] >= -tol) & (sy * pts[1] >= -tol)
            # the filled quadrant piece is bounded by its arc and the two axis
            # segments from the centre; its extents are the arc's extents
            wx = (sx * pts[0][sel]).max()
            wy = (sy * pts[1][sel]).max()
            w = bx[1] - bx[0]
            h = bx[3] - bx[2]
            assert abs(w - wx) <= 2e-6 * math.sqrt(gamma * A) + 1e-9, (trial, sx, sy, w, wx)
            assert abs(h - wy) <= 2e-6 * math.sqrt(gamma * C) + 1e-9, (trial, sx, sy, h, wy)


def test_stretch_factor_independent_of_gamma_and_centre(oracle):
    """f depends on Lambda only (text after Eq. (12)): minor/major extent ratios
    do not change with gamma or the centre."""
    rng = np.random.default_rng(13)
    for _ in range(100):
        A, B, C = random_cov(rng)
        ratios, tol = [], 4e-6
        for gamma, u, v in [(1.0, 0.0, 0.0), (4.0, 0.0, 0.0), (9.5, 37.25, -12.5)]:
            bx = oracle.pixel_boxes(rec(oracle, u, v, A, B, C, gamma), "quadbox").astype(np.float64)
            w = bx[:, 1] - bx[:, 0]
            ratios.append(w.min() / w.max())
            # box corners are rounded to binary32 around the centre
            tol += 4.0 * float(np.spacing(np.float32(max(abs(u), abs(v))))) / w.min()
        assert max(ratios) - min(ratios) <= tol


def test_axis_aligned_quadbox_equals_adr(oracle):
    """b = 0 gives f = 1 (Eq. (12)), so QuadBox and AdR-AABB cover the same tiles."""
    rng = np.random.default_rng(14)
    for _ in range(300):
        A = float(np.float32(math.exp(rng.uniform(-1, 7))))
        C = float(np.float32(math.exp(rng.uniform(-1, 7))))
        gamma = float(np.float32(rng.uniform(0.1, 11)))
        u, v = rng.uniform(-40, 300, 2)
        r = rec(oracle, u, v, A, 0.0, C, gamma)
        q = oracle.build_boxes(r, "quadbox", 256, 256)
        a = oracle.build_boxes(r, "adr", 256, 256)
        assert np.array_equal(oracle.tile_set(q, 0, 16), oracle.tile_set(a, 0, 16))


def test_quadbox_area_ratio(oracle):
    """Continuous area of the four sub-boxes over the AdR box is (1 + f^2)/2,
    with f^2 = 1 - B^2/(AC) (Eq. (12))."""
    rng = np.random.default_rng(15)
    for _ in range(100):
        A, B, C = random_cov(rng)
        bx = oracle.pixel_boxes(rec(oracle, 0.0, 0.0, A, B, C, 4.0), "quadbox")
        area = float(((bx[:, 1] - bx[:, 0]) * (bx[:, 3] - bx[:, 2])).sum())
        ad = oracle.pixel_boxes(rec(oracle, 0.0, 0.0, A, B, C, 4.0), "adr")[0]
        full = float((ad[1] - ad[0]) * (ad[3] - ad[2]))
        f2 = 1.0 - B * B / (A * C)
        assert abs(area / full - (1.0 + f2) / 2.0) <= 1e-5


def _required_tiles(g, W, H, margin):
    """Tiles holding a pixel sample strictly inside the 1/255 ellipse shrunk by
    `margin` pixels (float64 quadratic form), computed here with numpy."""
    A, B, C, gam = float(g["A"]), float(g["B"]), float(g["C"]), float(g["gamma"])
    u, v = float(g["u"]), float(g["v"])
    det = A * C - B * B
    lmin = 0.5 * (A + C) - math.sqrt(0.25 * (A - C) ** 2 + B * B)
    rmin = math.sqrt(gam * max(lmin, 0.0))
    s = max(0.0, 1.0 - margin / rmin) if rmin > 0 else 0.0
    xr, yr = math.sqrt(gam * A) + 1, math.sqrt(gam * C) + 1
    x0, x1 = max(0, math.floor(u - xr)), min(W - 1, math.ceil(u + xr))
    y0, y1 = max(0, math.floor(v - yr)), min(H - 1, math.ceil(v + yr))
    if x0 > x1 or y0 > y1:
        return set(), set()
    xs, ys = np.meshgrid(np.arange(x0, x1 + 1, dtype=np.float64), np.arange(y0, y1 + 1, dtype=np.float64))
    dx, dy = xs - u, ys - v
    q = (C * dx * dx - 2.0 * B * dx * dy + A * dy * dy) / det
    tid = (ys.astype(np.int64) // 16) * ((W + 15) // 16) + xs.astype(np.int64) // 16
    return set(np.unique(tid[q <= gam * s * s]).tolist()), set(np.unique(tid[q <= gam]).tolist())


@pytest.mark.parametrize("which", ["small", "aniso"])
def test_conservative_by_brute_force(oracle, which):
    """Every tile with a pixel sample inside the alpha >= 1/255 ellipse is in the
    QuadBox tile set (Sec. 1, Sec. 3: tight but conservative coverage); the
    same holds for AdR-AABB, and fails for DualBox (Sec. 4.4, Table 3)."""
    if which == "small":
        scene, cam = scenes.small_scene(n=3000)
    else:
        scene, cam = scenes.random_scene(5, 3000, 256, 192, 700.0, sh_degree=0, log_scale_mu=-4.0)
        rng = np.random.default_rng(5)
        half = 0.5 * rng.uniform(0, math.log(100.0), scene.n).astype(np.float32)
        scene.log_scales[0] += half
        scene.log_scales[1] -= half
        scene.log_scales[2] -= half
    W, H, tx = cam.width, cam.height, cam.tiles_x
    g = {m: oracle.project(scene, cam, m) for m in ("quadbox", "adr", "dualbox")}
    dual_missed = 0
    exact_total = 0
    for i in range(scene.n):
        gi = g["quadbox"][i]
        if not gi["visible"]:
            continue
        need, exact = _required_tiles(gi, W, H, 2e-3)
        exact_total += len(exact)
        q = set(oracle.tile_set(g["quadbox"], i, tx).tolist())
        a = set(oracle.tile_set(g["adr"], i, tx).tolist())
        d = set(oracle.tile_set(g["dualbox"], i, tx).tolist())
        assert need <= q, (i, sorted(need - q))
        assert need <= a
        assert d <= q <= a
        dual_missed += len(need - d)
    assert dual_missed > 0
    missed, exact_c, _ = oracle.coverage_audit(g["quadbox"], W, H, 2e-3)
    assert missed == 0 and exact_c == exact_total


def test_quadbox_inside_3sigma_when_gamma_at_most_9(oracle):
    """QuadBox tiles are a subset of the 3-sigma square's tiles whenever the
    1/255 level gamma is at most 9 (the 3-sigma level); above it the square can
    cut the 1/255 ellipse, which the audit counts."""
    scene, cam = scenes.small_scene()
    gq = oracle.project(scene, cam, "quadbox")
    g3 = oracle.project(scene, cam, "3sigma")
    above = 0
    for i in range(scene.n):
        if not gq[i]["visible"]:
            continue
        q = set(oracle.tile_set(gq, i, cam.tiles_x).tolist())
        s = set(oracle.tile_set(g3, i, cam.tiles_x).tolist())
        if gq[i]["gamma"] <= 9.0 * (1 - 1e-6):
            assert q <= s, i
        elif not q <= s:
            above += 1
    missed3, _, _ = oracle.coverage_audit(g3, cam.width, cam.height)
    assert above > 0 and missed3 > 0


def test_tile_mapping_pixel_exact(oracle):
    """A box covers a tile iff one of its integer pixel samples lies in it."""
    rng = np.random.default_rng(16)
    for _ in range(2000):
        u, v = rng.uniform(-30, 290, 2)
        A, C = np.exp(rng.uniform(-3, 5, 2))
        gamma = rng.uniform(0.05, 11)
        r = rec(oracle, u, v, A, 0.0, C, gamma)
        box = oracle.pixel_boxes(r, "adr")[0].astype(np.float64)
        xs = np.arange(256)
        ok_x = xs[(xs >= box[0]) & (xs <= box[1])]
        ok_y = xs[(xs >= box[2]) & (xs <= box[3])]
        want = {int(y // 16) * 16 + int(x // 16) for x in ok_x for y in ok_y}
        got = set(oracle.tile_set(oracle.build_boxes(r, "adr", 256, 256), 0, 16).tolist())
        assert got == want


def test_pair_counts_ordering(oracle):
    """Exact-sample count <= QuadBox <= AdR <= 3-sigma-or-more pair counts."""
    scene, cam = scenes.small_scene()
    counts = {m: int(oracle.tile_counts(oracle.project(scene, cam, m), cam.tiles_x).sum())
              for m in ("3sigma", "adr", "quadbox", "dualbox")}
    _, exact, _ = oracle.coverage_audit(oracle.project(scene, cam, "quadbox"), cam.width, cam.height)
    assert exact <= counts["quadbox"] <= counts["adr"]
    assert counts["dualbox"] <= counts["quadbox"]
    assert counts["adr"] < counts["3sigma"]


@pytest.mark.parametrize("which", ["small", "aniso"])
def test_clip_3sigma_tile_sets(oracle, which):
    """The 3-sigma clip (each sub-box tile rect cut to the 3-sigma square's
    tile rect): the clipped QuadBox tile set is the QuadBox set intersected
    with the 3-sigma set for every Gaussian (rect-wise cuts distribute over
    the union), so it lies inside the 3-sigma set even where gamma > 9; it
    still holds every tile of the 3-sigma set with a pixel sample inside the
    1/255 ellipse (conservative relative to the 3-sigma pipeline); DualBox and
    AdR clip the same way."""
    if which == "small":
        scene, cam = scenes.small_scene(n=3000)
    else:
        scene, cam = scenes.random_scene(6, 3000, 256, 192, 700.0, sh_degree=0, log_scale_mu=-4.0)
        rng = np.random.default_rng(6)
        half = 0.5 * rng.uniform(0, math.log(100.0), scene.n).astype(np.float32)
        scene.log_scales[0] += half
        scene.log_scales[1] -= half
        scene.log_scales[2] -= half
    W, H, tx = cam.width, cam.height, cam.tiles_x
    modes = ("quadbox", "3sigma", "quadbox_clip3sigma", "adr", "adr_clip3sigma", "dualbox", "dualbox_clip3sigma")
    g = {m: oracle.project(scene, cam, m) for m in modes}
    cut = 0
    for i in range(scene.n):
        if not g["quadbox"][i]["visible"]:
            assert not g["quadbox_clip3sigma"][i]["visible"]
            continue
        ts = {m: set(oracle.tile_set(g[m], i, tx).tolist()) for m in modes}
        s = ts["3sigma"]
        for base in ("quadbox", "adr", "dualbox"):
            assert ts[base + "_clip3sigma"] == ts[base] & s, (i, base)
        need, _ = _required_tiles(g["quadbox"][i], W, H, 2e-3)
        assert need & s <= ts["quadbox_clip3sigma"], i
        cut += not ts["quadbox"] <= s
    assert cut > 0   # the clip changes some Gaussians (gamma > 9)


def test_clip_3sigma_image_equals_3sigma_image(oracle):
    """With the clip, the render sees every contribution the 3-sigma pipeline
    sees and no other (QuadBox is conservative, and the clipped set is inside
    the 3-sigma set), so the image and final T equal the 3-sigma ones; the
    unclipped QuadBox image differs where gamma > 9 ellipses leave the
    3-sigma squares."""
    scene, cam = scenes.small_scene(n=4000)
    f3 = oracle.forward(scene, cam, "3sigma")
    fc = oracle.forward(scene, cam, "quadbox_clip3sigma")
    fq = oracle.forward(scene, cam, "quadbox")
    assert np.array_equal(fc["image"], f3["image"])
    assert np.array_equal(fc["T"], f3["T"])
    assert len(fc["ids"]) <= len(f3["ids"]) and len(fc["ids"]) <= len(fq["ids"])
    assert not np.array_equal(fq["image"], f3["image"])
