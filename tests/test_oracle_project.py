"""Pins of the oracle's projection step (Sec. 2: EWA projection of each 3D
Gaussian, Eq. (1); opacity threshold of Eqs. (3)-(4)) against independent
computations: scipy rotations, finite-difference Jacobians of the pinhole map,
scipy's complex spherical harmonics, and textbook special cases."""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation
from scipy.special import expit, sph_harm_y

from paper_2605_04844_amd import scenes


def _one_scene(means, log_scales, quats, logits, sh=None, sh_degree=0):
    n = np.asarray(means).shape[1]
    if sh is None:
        sh = np.zeros((3 * (sh_degree + 1) ** 2, n), np.float32)
    f = lambda a: np.ascontiguousarray(np.asarray(a, np.float32))
    return scenes.Scene(f(means), f(log_scales), f(quats), f(logits), f(sh), sh_degree)


def _pinhole_jacobian(cam, p):
    """d(u, v)/d(p_cam) by central differences of the pinhole map."""
    def proj(q):
        return np.array([cam.fx * q[0] / q[2] + cam.cx, cam.fy * q[1] / q[2] + cam.cy])
    J = np.zeros((2, 3))
    for k in range(3):
        h = 1e-6 * max(1.0, abs(p[k]))
        e = np.zeros(3)
        e[k] = h
        J[:, k] = (proj(p + e) - proj(p - e)) / (2 * h)
    return J


def test_isotropic_on_axis(oracle):
    """An isotropic Gaussian of scale s on the optical axis at depth z projects to
    the principal point with Sigma2D = (f s / z)^2 I plus the 0.3 low-pass."""
    cam = scenes.pinhole(256, 256, 300.0)
    zs = np.array([1.0, 2.5, 4.0, 7.0], np.float32)
    n = len(zs)
    s = np.log(np.array([0.01, 0.05, 0.02, 0.1], np.float32))
    sc = _one_scene(np.stack([np.zeros(n), np.zeros(n), zs]), np.stack([s, s, s]),
                    np.stack([np.ones(n), np.zeros(n), np.zeros(n), np.zeros(n)]), np.zeros(n))
    g = oracle.project(sc, cam, "quadbox")
    for i in range(n):
        var = (300.0 * math.exp(float(s[i])) / float(zs[i])) ** 2 + 0.3
        assert abs(g["A"][i] - var) <= 2e-6 * var and abs(g["C"][i] - var) <= 2e-6 * var
        assert abs(g["B"][i]) <= 1e-6 * var
        assert g["u"][i] == np.float32(cam.cx) and g["v"][i] == np.float32(cam.cy)
        assert g["depth"][i] == zs[i]


def test_ewa_against_finite_difference_jacobian(oracle):
    """Sigma2D = J W Sigma3D W^T J^T + 0.3 I with Sigma3D = R S S^T R^T (Eq. (1)
    covariance from scale and rotation), J the Jacobian of the pinhole map,
    W the camera rotation; all built independently with scipy and numpy."""
    rng = np.random.default_rng(21)
    n = 400
    Rc = Rotation.random(random_state=7).as_matrix().astype(np.float32)
    eye = np.array([0.3, -0.2, -4.0])
    t = (-(Rc.astype(np.float64) @ eye)).astype(np.float32)
    cam = scenes.pinhole(640, 480, 600.0, Rc, t)
    # points inside the view frustum (well away from the 1.3x clamp)
    pc = np.stack([rng.uniform(-0.3, 0.3, n), rng.uniform(-0.25, 0.25, n), rng.uniform(2, 6, n)])
    pc[0] *= pc[2]
    pc[1] *= pc[2]
    means = (Rc.astype(np.float64).T @ (pc - t[:, None].astype(np.float64))).astype(np.float32)
    ls = rng.normal(-3.0, 1.0, (3, n)).astype(np.float32)
    q = rng.standard_normal((4, n)).astype(np.float32)
    sc = _one_scene(means, ls, q, rng.normal(1.0, 0.5, n))
    g = oracle.project(sc, cam, "adr")
    for i in range(n):
        m = sc.means[:, i].astype(np.float64)
        p = Rc.astype(np.float64) @ m + t.astype(np.float64)
        rot = Rotation.from_quat([q[1, i], q[2, i], q[3, i], q[0, i]]).as_matrix()
        S3 = rot @ np.diag(np.exp(2.0 * ls[:, i].astype(np.float64))) @ rot.T
        J = _pinhole_jacobian(cam, p) @ Rc.astype(np.float64)
        S2 = J @ S3 @ J.T + 0.3 * np.eye(2)
        scale = math.sqrt(S2[0, 0] * S2[1, 1])
        assert abs(g["A"][i] - S2[0, 0]) <= 1e-5 * scale
        assert abs(g["B"][i] - S2[0, 1]) <= 1e-5 * scale
        assert abs(g["C"][i] - S2[1, 1]) <= 1e-5 * scale
        assert abs(g["depth"][i] - p[2]) <= 1e-6 * p[2]
        uv = np.array([cam.fx * p[0] / p[2] + cam.cx, cam.fy * p[1] / p[2] + cam.cy])
        assert abs(g["u"][i] - uv[0]) <= 2e-4 and abs(g["v"][i] - uv[1]) <= 2e-4
        inv = np.linalg.inv(np.array([[g["A"][i], g["B"][i]], [g["B"][i], g["C"][i]]], np.float64))
        A_, B_, C_ = (float(g[f][i]) for f in ("A", "B", "C"))
        # binary32 determinant A*C - B*B loses digits in proportion to its condition
        cond = (abs(A_ * C_) + B_ * B_) / (A_ * C_ - B_ * B_)
        tol = 8 * 2.0 ** -24 * cond * abs(inv).max()
        assert abs(g["a"][i] - inv[0, 0]) <= tol
        assert abs(g["b"][i] - inv[0, 1]) <= tol
        assert abs(g["c"][i] - inv[1, 1]) <= tol


def test_jacobian_clamped_outside_frustum(oracle):
    """Far outside the view the affine approximation is taken at the point whose
    image-plane slope is clamped to 1.3x the half field of view: Sigma2D equals
    that of the same Gaussian moved to the clamped point."""
    cam = scenes.pinhole(200, 100, 100.0)   # tan half-fov: 1.0 (x), 0.5 (y)
    z = np.float32(3.0)
    xs = np.array([5.0 * z, -4.0 * z, 0.2 * z], np.float32)
    ys = np.array([0.1 * z, -3.0 * z, 2.0 * z], np.float32)
    xc = np.clip(xs / z, -1.3, 1.3) * z
    yc = np.clip(ys / z, -0.65, 0.65) * z
    n = 3
    ls = np.full((3, 2 * n), -2.0, np.float32)
    ls[0] = -1.0
    q = np.tile(np.array([[0.9], [0.1], [0.3], [0.2]], np.float32), (1, 2 * n))
    sc = _one_scene(np.stack([np.concatenate([xs, xc]), np.concatenate([ys, yc]), np.full(2 * n, z)]),
                    ls, q, np.zeros(2 * n))
    g = oracle.project(sc, cam, "3sigma")
    for i in range(n):
        for f in ("A", "B", "C"):
            assert abs(g[f][i] - g[f][n + i]) <= 1e-5 * abs(g[f][n + i]) + 1e-6


def test_activations_and_gamma(oracle):
    """Scales exp(l), opacity sigmoid(logit), and gamma = 2 ln(o / (1/255))
    (Eq. (3)) agree with numpy/scipy to binary32 rounding."""
    rng = np.random.default_rng(22)
    n = 5000
    logits = rng.normal(0.0, 2.0, n).astype(np.float32)
    s = scenes.small_scene(n=n)[0]
    s.logits[:] = logits
    cam = scenes.pinhole(256, 256, 256.0)
    g = oracle.project(s, cam, "3sigma")
    o = expit(logits.astype(np.float64))
    assert np.all(np.abs(g["opacity"] - o) <= np.spacing(o.astype(np.float32)))
    gam = 2.0 * np.log(255.0 * g["opacity"].astype(np.float64))
    ok = g["visible"] == 1
    assert np.all(np.abs(g["gamma"][ok] - gam[ok]) <= np.spacing(np.abs(gam[ok]).astype(np.float32)))


def test_activation_function_against_numpy(oracle):
    """oracle.activations (the functions the projection evaluates, which the
    GPU sweep compares with the library on every binary32 of their ranges):
    exp, scipy's expit and 2 ln(255 o) in binary64 rounded once, equal bit
    for bit to numpy/scipy's binary64 results rounded once on 3e6 values
    (spread over the swept ranges, plus their end points)."""
    rng = np.random.default_rng(23)
    cases = {"scale": (-20.0, 5.0, lambda x: np.exp(x)),
             "opacity": (-5.6, 17.0, lambda x: expit(x)),
             "gamma": (1.0 / 255.0, 1.0, lambda x: 2.0 * np.log(255.0 * x))}
    for name, (lo, hi, ref) in cases.items():
        x = np.concatenate([rng.uniform(lo, hi, 1_000_000), [lo, hi]]).astype(np.float32)
        got = oracle.activations(x, name)
        want = ref(x.astype(np.float64)).astype(np.float32)
        assert np.array_equal(got.view(np.uint32), want.view(np.uint32)), name
    # the projection's own values are these functions of its inputs
    s = scenes.small_scene(n=2000)[0]
    g = oracle.project(s, scenes.pinhole(256, 256, 256.0), "3sigma")
    assert np.array_equal(g["opacity"], oracle.activations(s.logits, "opacity"))
    ok = g["visible"] == 1
    assert np.array_equal(g["gamma"][ok], oracle.activations(g["opacity"][ok], "gamma"))


def test_culling(oracle):
    """Behind the near plane, degenerate rotation, and (opacity-aware modes
    only) o <= 1/255 are culled."""
    n = 4
    means = np.array([[0, 0, 0, 0], [0, 0, 0, 0], [0.1, 3.0, 3.0, 3.0]], np.float32)
    quats = np.array([[1, 0, 1, 1], [0, 0, 0, 0], [0, 0, 0, 0], [0, 0, 0, 0]], np.float32)
    logits = np.array([0.0, 0.0, -6.0, 0.0], np.float32)   # sigmoid(-6) < 1/255
    sc = _one_scene(means, np.full((3, n), -3.0), quats, logits)
    cam = scenes.pinhole(64, 64, 64.0)
    ga = oracle.project(sc, cam, "quadbox")
    g3 = oracle.project(sc, cam, "3sigma")
    assert list(ga["visible"]) == [0, 0, 0, 1]
    assert list(g3["visible"]) == [0, 0, 1, 1]


def _real_sh(l, m, theta, phi):
    """Real SH from scipy's complex SH (Condon-Shortley phase included)."""
    y = sph_harm_y(l, abs(m), theta, phi)
    if m > 0:
        return math.sqrt(2.0) * y.real
    if m < 0:
        return math.sqrt(2.0) * y.imag
    return y.real


def test_sh_basis_against_scipy(oracle):
    rng = np.random.default_rng(23)
    for _ in range(200):
        d = rng.standard_normal(3)
        d /= np.linalg.norm(d)
        theta, phi = math.acos(d[2]), math.atan2(d[1], d[0])
        got = oracle.sh_basis(*d)
        for l in range(4):
            for m in range(-l, l + 1):
                assert abs(got[l * l + l + m] - _real_sh(l, m, theta, phi)) <= 1e-12


def test_colour_from_sh(oracle):
    """rgb = max(0, sum_k Y_k(dir) sh_k + 0.5), dir from the camera centre."""
    sc, cam = scenes.cluster_scene(n=300, clusters=4)
    Rc = Rotation.random(random_state=3).as_matrix().astype(np.float32)
    cam = scenes.pinhole(1280, 720, 1280.0, Rc, np.array([0.1, 0.2, 4.0], np.float32))
    sc.means[2] -= 4.0
    g = oracle.project(sc, cam, "3sigma")
    cp = cam.campos.astype(np.float64)
    checked = 0
    for i in range(sc.n):
        if not g["visible"][i]:
            continue
        d = sc.means[:, i].astype(np.float64) - cp
        d /= np.linalg.norm(d)
        theta, phi = math.acos(np.clip(d[2], -1, 1)), math.atan2(d[1], d[0])
        Y = np.array([_real_sh(l, m, theta, phi) for l in range(4) for m in range(-l, l + 1)])
        coef = sc.sh[:, i].astype(np.float64).reshape(16, 3)
        rgb = np.maximum(Y @ coef + 0.5, 0.0)
        assert np.abs(g["rgb"][i] - rgb).max() <= 1e-10
        checked += 1
    assert checked > 50


def test_rotation_invariance_of_isotropic(oracle):
    """Sigma3D of an isotropic Gaussian does not depend on its quaternion."""
    rng = np.random.default_rng(24)
    n = 50
    means = np.stack([rng.uniform(-0.5, 0.5, n), rng.uniform(-0.5, 0.5, n), rng.uniform(2, 5, n)])
    ls = np.tile(rng.normal(-3, 0.5, n), (3, 1))
    sc1 = _one_scene(means, ls, rng.standard_normal((4, n)), np.zeros(n))
    sc2 = _one_scene(means, ls, np.stack([np.ones(n), np.zeros(n), np.zeros(n), np.zeros(n)]), np.zeros(n))
    cam = scenes.pinhole(256, 256, 256.0)
    g1, g2 = oracle.project(sc1, cam, "adr"), oracle.project(sc2, cam, "adr")
    scale = np.sqrt(g2["A"].astype(np.float64) * g2["C"])
    for f in ("A", "B", "C"):
        assert np.all(np.abs(g1[f].astype(np.float64) - g2[f]) <= 1e-5 * scale)
