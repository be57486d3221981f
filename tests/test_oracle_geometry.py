"""Pins of the FP64 oracle's camera, intersection and normal routines against
closed forms and an independent root finder (numpy.roots on the defining
polynomial).  CPU only."""
import math

import numpy as np
import pytest

import scenegen


def test_camera_centre_pixel_is_view_axis(oracle_mod):
    cam = scenegen.Camera((0.0, 0.0, 30.0), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 50.0, 129, 97)
    o, d = oracle_mod.camera_ray(cam, 64, 48)
    assert tuple(o) == (0.0, 0.0, 30.0)
    assert tuple(d) == (0.0, 0.0, -1.0)


@pytest.mark.parametrize("W,H", [(128, 128), (965, 1137), (7, 3)])
def test_camera_corner_angle(oracle_mod, W, H):
    # top-right pixel centre lies at (1-1/W, 1-1/H) of the half-extents
    cam = scenegen.Camera((0.0, 0.0, 30.0), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 50.0, W, H)
    th = math.tan(math.radians(25.0))
    x = (1.0 - 1.0 / W) * th * (W / H)
    y = (1.0 - 1.0 / H) * th
    _, d = oracle_mod.camera_ray(cam, W - 1, 0)
    ang = math.acos(-d[2])
    assert abs(ang - math.atan(math.hypot(x, y))) < 1e-13
    assert d[0] > 0 and d[1] > 0  # right and up


def test_camera_inverse_projection(oracle_mod):
    # projecting each ray back onto the image plane returns the pixel centre
    rng = np.random.default_rng(0)
    cam = scenegen.Camera((3.0, -2.0, 40.0), (1.0, 2.0, -1.0), (0.0, 1.0, 0.0), 37.0, 640, 480)
    f = np.subtract(cam.lookat, cam.eye); f /= np.linalg.norm(f)
    r = np.cross(f, cam.up); r /= np.linalg.norm(r)
    u = np.cross(r, f)
    th = math.tan(math.radians(cam.fovy_deg / 2))
    for _ in range(50):
        i, j = int(rng.integers(cam.width)), int(rng.integers(cam.height))
        _, d = oracle_mod.camera_ray(cam, i, j)
        assert abs(np.linalg.norm(d) - 1) < 1e-15
        px = (d @ r) / (d @ f) / (th * cam.width / cam.height)
        py = (d @ u) / (d @ f) / th
        assert abs(px - (2 * (i + 0.5) / cam.width - 1)) < 1e-12
        assert abs(py - (1 - 2 * (j + 0.5) / cam.height)) < 1e-12


def test_sphere_closed_forms(oracle_mod):
    hs = oracle_mod.hit_sphere
    z = (0.0, 0.0, 1.0)
    assert hs((0, 0, 0), 1.0, (0, 0, -10.0), z) == 9.0
    for h in (0.0, 0.3, 0.7, 0.99):
        t = hs((0, 0, 0), 1.0, (0, h, -10.0), z)
        assert abs(t - (10 - math.sqrt(1 - h * h))) < 1e-13
    assert hs((0, 0, 0), 1.0, (0, 1.0, -10.0), z) == 10.0        # tangent
    assert hs((0, 0, 0), 1.0, (0, 1.0 + 1e-9, -10.0), z) is None  # just outside
    assert hs((0, 0, 0), 1.0, (0, 0, 0.0), z) == 1.0              # inside -> far root
    assert hs((0, 0, 0), 1.0, (0, 0, 5.0), z) is None             # sphere behind
    assert hs((0, 0, 0), 1.0, (0, 0, -10.0), z, tmax=8.5) is None  # beyond tmax
    assert hs((0, 0, 0), 1.0, (0, 0, -10.0), z, tmin=9.5) == 11.0  # near root excluded


def _quad_roots(poly):
    rts = np.roots(poly)
    return sorted(float(x.real) for x in rts if abs(x.imag) < 1e-9)


def test_sphere_vs_polynomial_roots(oracle_mod):
    rng = np.random.default_rng(1)
    n_hit = 0
    for _ in range(400):
        c = rng.uniform(-3, 3, 3); r = rng.uniform(0.3, 2.0)
        o = rng.uniform(-10, 10, 3)
        d = c + rng.uniform(-1.5 * r, 1.5 * r, 3) - o; d /= np.linalg.norm(d)
        q = o - c
        roots = [t for t in _quad_roots([d @ d, 2 * (q @ d), q @ q - r * r]) if t > 0]
        t = oracle_mod.hit_sphere(c, r, o, d)
        if not roots:
            assert t is None
        else:
            n_hit += 1
            assert t is not None and abs(t - roots[0]) < 1e-8 * max(1, roots[0])
    assert n_hit > 20


def test_cylinder_closed_forms(oracle_mod):
    hc = oracle_mod.hit_cylinder
    a, b = (0, -1.0, 0), (0, 1.0, 0)
    assert hc(a, b, 0.5, (-10.0, 0, 0), (1.0, 0, 0)) == 9.5
    assert hc(a, b, 0.5, (-10.0, 1.5, 0), (1.0, 0, 0)) is None    # beyond the end
    assert hc(a, b, 0.5, (0.2, -5.0, 0), (0, 1.0, 0)) is None     # parallel to axis
    assert hc(a, b, 0.5, (0.0, 0.0, 0), (1.0, 0, 0)) == 0.5       # inside -> far wall
    # open: a ray down the axis direction through the cap region misses
    d = np.array([0.05, 1.0, 0.0]); d /= np.linalg.norm(d)
    assert hc(a, b, 0.5, (0.0, -5.0, 0.0), d) is None
    # oblique ray: closed form through the x = -0.5 wall
    d = np.array([1.0, 0.05, 0.0]); d /= np.linalg.norm(d)
    t = hc(a, b, 0.5, (-10.0, 0.0, 0.0), d)
    assert abs(t - 9.5 / d[0]) < 1e-12


def test_cylinder_vs_polynomial_roots(oracle_mod):
    rng = np.random.default_rng(2)
    n_hit = 0
    for _ in range(400):
        a = rng.uniform(-2, 2, 3); b = rng.uniform(-2, 2, 3); rho = rng.uniform(0.2, 1.0)
        o = rng.uniform(-8, 8, 3)
        d = 0.5 * (a + b) + rng.uniform(-1.5, 1.5, 3) - o; d /= np.linalg.norm(d)
        L = np.linalg.norm(b - a); w = (b - a) / L
        D = o - a
        dp = d - (d @ w) * w; Dp = D - (D @ w) * w
        roots = _quad_roots([dp @ dp, 2 * (dp @ Dp), Dp @ Dp - rho * rho])
        ok = [t for t in roots if t > 0 and 0 <= (D + t * d) @ w <= L]
        t = oracle_mod.hit_cylinder(a, b, rho, o, d)
        if not ok:
            assert t is None
        else:
            n_hit += 1
            assert t is not None and abs(t - ok[0]) < 1e-8 * max(1, ok[0])
    assert n_hit > 20


def test_normals(oracle_mod):
    sc = scenegen.Scene(np.array([[1.0, 2.0, 3.0]]), np.array([2.0]), np.ones((1, 3), np.float32),
                        np.array([[0.0, 0, 0]]), np.array([[0.0, 4.0, 0]]), np.array([0.5]),
                        np.ones((1, 3), np.float32), np.zeros((0, 3)), np.zeros((0, 3)))
    o = np.array([1.0, 2.0, -20.0]); d = np.array([0.0, 0.0, 1.0])
    t = oracle_mod.hit_sphere(sc.sph_center[0], 2.0, o, d)
    assert t == 21.0
    assert np.allclose(oracle_mod.normal(sc, 0, o, d, t), [0, 0, -1], atol=1e-15)
    o = np.array([-5.0, 1.0, 0.3]); d = np.array([1.0, 0.0, 0.0])
    t = oracle_mod.hit_cylinder(sc.cyl_a[0], sc.cyl_b[0], 0.5, o, d)
    n = oracle_mod.normal(sc, 1, o, d, t)
    assert abs(np.linalg.norm(n) - 1) < 1e-14 and abs(n[1]) < 1e-15
    assert np.allclose(n, [-math.sqrt(0.25 - 0.09) / 0.5, 0, 0.3 / 0.5], atol=1e-14)
