"""Pins of the oracle's 3-sigma baseline box (Sec. 2: a square of side
6 sqrt(lambda_max) around the projected mean) against numpy's symmetric
eigen-solver and a brute-force enumeration of pixel samples, both outside
the oracle.  The reading pinned here: radius r = ceil(3 sqrt(lambda_1)),
lambda_1 the larger eigenvalue of Sigma2D, with the discriminant of the 2x2
eigenvalue formula floored at 0.1 (the 3DGS convention for near-isotropic
Sigma2D; it can only enlarge the square)."""
import math

import numpy as np

from paper_2605_04844_amd import scenes

FLOOR = 0.1


def rec(O, u, v, A, B, C):
    r = np.zeros(1, O.GAUSS_DTYPE)
    r["u"], r["v"], r["A"], r["B"], r["C"] = u, v, A, B, C
    det = float(np.float32(A)) * float(np.float32(C)) - float(np.float32(B)) ** 2
    r["a"], r["b"], r["c"] = C / det, -B / det, A / det
    r["gamma"], r["opacity"], r["visible"] = 4.0, 0.5, 1
    return r


def lam_max(A, B, C):
    """Largest eigenvalue of the stored (binary32) Sigma2D, by LAPACK."""
    S = np.array([[A, B], [B, C]], np.float64)
    return float(np.linalg.eigvalsh(S)[-1])


def radius(O, A, B, C):
    """The oracle's radius: the right edge of the square centred at 0 (exact,
    since 0 + r is r)."""
    box = O.pixel_boxes(rec(O, 0.0, 0.0, A, B, C), "3sigma")
    assert box.shape == (1, 4)
    x0, x1, y0, y1 = (float(x) for x in box[0])
    assert x0 == -x1 and y0 == -y1 and x1 == y1   # a square around the mean
    return x1


def random_sigma(rng, kind):
    if kind == "aniso":
        l1 = math.exp(rng.uniform(math.log(0.3), 12.0))
        l2 = l1 / math.exp(rng.uniform(0.0, 9.0))
        th = rng.uniform(0.0, math.pi)
    else:   # near-isotropic: the eigenvalues differ by less than the floor allows
        l1 = math.exp(rng.uniform(math.log(0.3), 9.0))
        l2 = l1 - rng.uniform(0.0, 0.6)
        th = rng.uniform(0.0, math.pi)
    c, s = math.cos(th), math.sin(th)
    Rm = np.array([[c, -s], [s, c]])
    S = (Rm @ np.diag([l1, max(l2, 0.3)]) @ Rm.T).astype(np.float32)
    return float(S[0, 0]), float(S[0, 1]), float(S[1, 1])


def test_radius_is_ceil_of_three_sqrt_lambda_max(oracle):
    """Away from the floor, r = ceil(3 sqrt(lambda_max)) with lambda_max from
    numpy.linalg.eigvalsh; where 3 sqrt(lambda_max) lies within binary32
    rounding of an integer k, r may be k or k + 1."""
    rng = np.random.default_rng(31)
    checked = 0
    for _ in range(800):
        A, B, C = random_sigma(rng, "aniso")
        disc = 0.25 * (A - C) ** 2 + B * B
        if disc < FLOOR * 1.01:
            continue
        x = 3.0 * math.sqrt(lam_max(A, B, C))
        r = radius(oracle, A, B, C)
        k = round(x)
        if abs(x - k) <= 1e-5 * x:
            assert r in (k, k + 1), (A, B, C, x, r)
        else:
            assert r == math.ceil(x), (A, B, C, x, r)
        checked += 1
    assert checked > 700


def test_radius_floor_regime(oracle):
    """Near-isotropic Sigma2D (discriminant below the floor): the radius is
    never smaller than the true 3-sigma radius, exceeds it only by what the
    floor adds to the eigenvalue (at most sqrt(0.1)), and for an exactly
    isotropic Sigma2D = aI (lambda_max = a) equals ceil(3 sqrt(a + sqrt(0.1)))."""
    rng = np.random.default_rng(32)
    seen = 0
    for _ in range(400):
        A, B, C = random_sigma(rng, "iso")
        if 0.25 * (A - C) ** 2 + B * B >= FLOOR * 0.99:
            continue
        lm = lam_max(A, B, C)
        r = radius(oracle, A, B, C)
        assert math.ceil(3.0 * math.sqrt(lm) * (1 - 1e-6)) <= r
        assert r <= math.ceil(3.0 * math.sqrt(lm + math.sqrt(FLOOR)) * (1 + 1e-6))
        seen += 1
    assert seen > 100
    for a in np.float32(np.exp(rng.uniform(math.log(0.3), 12.0, 300))):
        a = float(a)
        x = 3.0 * math.sqrt(a + math.sqrt(FLOOR))
        r = radius(oracle, a, 0.0, a)
        k = round(x)
        if abs(x - k) <= 1e-5 * x:
            assert r in (k, k + 1)
        else:
            assert r == math.ceil(x), (a, x, r)


def test_3sigma_tile_set_by_pixel_enumeration(oracle):
    """The 3-sigma tile set of a Gaussian is exactly the set of tiles holding
    an integer pixel sample (x, y) of the image with |x - u| <= R and
    |y - v| <= R, R = ceil(3 sqrt(lambda_max)) by eigvalsh (samples within
    1e-3 px of the square's edge, where binary32 rounding of u +- R decides,
    are left out of both directions of the check)."""
    rng = np.random.default_rng(33)
    W, H = 200, 136
    tiles_x = (W + 15) // 16
    xs, ys = np.meshgrid(np.arange(W), np.arange(H))
    tid = (ys // 16) * tiles_x + xs // 16
    checked = 0
    for _ in range(600):
        A, B, C = random_sigma(rng, "aniso")
        A, B, C = A * 1e-2, B * 1e-2, C * 1e-2   # squares of a few to a few hundred pixels
        if 0.25 * (A - C) ** 2 + B * B < FLOOR * 1.01:
            continue
        x = 3.0 * math.sqrt(lam_max(A, B, C))
        if abs(x - round(x)) <= 1e-5 * x:
            continue
        R = math.ceil(x)
        u, v = (float(np.float32(t)) for t in rng.uniform(-60, 260, 2))
        g = oracle.build_boxes(rec(oracle, u, v, A, B, C), "3sigma", W, H)
        got = set(oracle.tile_set(g, 0, tiles_x).tolist())
        d = np.maximum(np.abs(xs - u), np.abs(ys - v))
        need = set(np.unique(tid[d <= R - 1e-3]).tolist())
        may = set(np.unique(tid[d <= R + 1e-3]).tolist())
        assert need <= got <= may, (A, B, C, u, v)
        checked += 1
    assert checked > 300


def test_3sigma_square_contains_three_sigma_ellipse(oracle):
    """On a projected scene: every pixel sample inside the 3-sigma ellipse of
    a Gaussian (d^T Sigma2D^-1 d <= 9, binary64) lies in its square's tiles
    (the square circumscribes the circle of radius 3 sqrt(lambda_max), which
    holds that ellipse)."""
    scene, cam = scenes.small_scene(n=2000)
    g = oracle.project(scene, cam, "3sigma")
    W, H, tx = cam.width, cam.height, cam.tiles_x
    for i in range(scene.n):
        if not g[i]["visible"]:
            continue
        A, B, C = (float(g[i][f]) for f in "ABC")
        u, v = float(g[i]["u"]), float(g[i]["v"])
        det = A * C - B * B
        rx, ry = math.sqrt(9 * A) + 1, math.sqrt(9 * C) + 1
        x0, x1 = max(0, math.floor(u - rx)), min(W - 1, math.ceil(u + rx))
        y0, y1 = max(0, math.floor(v - ry)), min(H - 1, math.ceil(v + ry))
        if x0 > x1 or y0 > y1:
            continue
        px, py = np.meshgrid(np.arange(x0, x1 + 1, dtype=np.float64), np.arange(y0, y1 + 1, dtype=np.float64))
        dx, dy = px - u, py - v
        q = (C * dx * dx - 2 * B * dx * dy + A * dy * dy) / det
        need = set(np.unique((py[q <= 9 * (1 - 1e-6)] // 16) * tx + px[q <= 9 * (1 - 1e-6)] // 16).astype(int).tolist())
        assert need <= set(oracle.tile_set(g, i, tx).tolist()), i
