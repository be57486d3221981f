"""Pins of the oracle's triangles (a third primitive type, for surface
representations; two-sided, Moller-Trumbore):
  * closed forms: interior hit, outside an edge, on an edge (edges belong to
    the triangle), a ray in the plane's direction, the back side, t-range cuts;
  * random rays against an independent solve of o + t d = v0 + u e1 + v e2
    (numpy.linalg.solve), away from the edges;
  * normal = unit e1 x e2;
  * grid == brute force on a scene of all three primitive types;
  * shading: a large triangle lit by one light, S = 0, is
    albedo * (rescale * |N.L| + sky) wherever it is seen (normal facing the
    viewer), and a point on it beside a sphere sees the closed-form
    cosine-weighted visibility 8/9.
CPU only."""
import math

import numpy as np
import pytest

import scenegen

V0, V1, V2 = np.array([0.0, 0.0, 0.0]), np.array([1.0, 0.0, 0.0]), np.array([0.0, 1.0, 0.0])


def test_closed_forms(oracle_mod):
    down = np.array([0.0, 0.0, -1.0])
    h = oracle_mod.hit_triangle
    assert h(V0, V1, V2, np.array([0.25, 0.25, 5.0]), down) == 5.0
    assert h(V0, V1, V2, np.array([0.6, 0.6, 5.0]), down) is None      # u + v > 1
    assert h(V0, V1, V2, np.array([-0.1, 0.5, 5.0]), down) is None     # u < 0 side
    assert h(V0, V1, V2, np.array([0.5, 0.5, 5.0]), down) == 5.0       # on the hypotenuse
    assert h(V0, V1, V2, np.array([0.0, 0.0, 5.0]), down) == 5.0       # a vertex
    assert h(V0, V1, V2, np.array([-1.0, 0.2, 0.0]), np.array([1.0, 0.0, 0.0])) is None  # det = 0
    assert h(V0, V1, V2, np.array([0.25, 0.25, -5.0]), -down) == 5.0   # two-sided
    assert h(V0, V1, V2, np.array([0.25, 0.25, 5.0]), down, tmin=5.0) is None
    assert h(V0, V1, V2, np.array([0.25, 0.25, 5.0]), down, tmax=4.9) is None
    assert h(V0, V1, V2, np.array([0.25, 0.25, 5.0]), down, tmax=5.0) == 5.0
    assert h(V0, V1, V2, np.array([0.25, 0.25, 5.0]), -down) is None   # behind the origin
    # oblique: from (0.2, 0.1, 3) towards (0.4, 0.3, 0): t = |(0.2, 0.2, -3)|
    o = np.array([0.2, 0.1, 3.0])
    v = np.array([0.2, 0.2, -3.0])
    t = h(V0, V1, V2, o, v / np.linalg.norm(v))
    assert abs(t - np.linalg.norm(v)) < 1e-14


def test_random_rays_against_linear_solve(oracle_mod):
    rng = np.random.default_rng(21)
    n_hit = 0
    for _ in range(3000):
        v = rng.normal(size=(3, 3)) * 3.0
        o = rng.normal(size=3) * 6.0
        target = v[0] + rng.uniform(-0.3, 1.2) * (v[1] - v[0]) + rng.uniform(-0.3, 1.2) * (v[2] - v[0])
        d = target - o
        d /= np.linalg.norm(d)
        M = np.stack([-d, v[1] - v[0], v[2] - v[0]], axis=1)
        if abs(np.linalg.det(M)) < 1e-6:
            continue
        t, uu, vv = np.linalg.solve(M, o - v[0])
        margin = min(uu, vv, 1.0 - uu - vv)
        if abs(margin) < 1e-6 or abs(t) < 1e-6:
            continue  # too close to an edge or the origin to call
        want = margin > 0 and t > 0
        got = oracle_mod.hit_triangle(v[0], v[1], v[2], o, d)
        assert (got is not None) == want, (v, o, d, t, uu, vv)
        if want:
            n_hit += 1
            assert abs(got - t) <= 1e-9 * max(1.0, abs(t))
    assert n_hit > 500


def _one_triangle_scene(v, albedo=0.6, lights=((0.3, 0.4, 1.0),), spheres=(), radii=()):
    e3 = np.zeros((0, 3))
    ld = np.array(lights, dtype=np.float64).reshape(-1, 3)
    sp = np.array(spheres, dtype=np.float64).reshape(-1, 3)
    s = scenegen.Scene(sp, np.array(radii, dtype=np.float64),
                       np.full((len(radii), 3), 0.5, np.float32), e3, e3.copy(), np.zeros(0),
                       np.zeros((0, 3), np.float32), ld, np.ones_like(ld))
    v = np.asarray(v, dtype=np.float64).reshape(-1, 3, 3)
    return scenegen.with_triangles(s, v, np.full((v.shape[0], 3), albedo, np.float32))


def test_normal(oracle_mod):
    s = _one_triangle_scene([[V0, V1, V2]])
    o = np.array([0.25, 0.25, 5.0])
    d = np.array([0.0, 0.0, -1.0])
    n = oracle_mod.normal(s, 0, o, d, 5.0)
    assert np.allclose(n, [0.0, 0.0, 1.0], atol=0)
    s = _one_triangle_scene([[V0, V2, V1]])  # reversed winding
    assert np.allclose(oracle_mod.normal(s, 0, o, d, 5.0), [0.0, 0.0, -1.0], atol=0)


def test_grid_equals_brute_force_mixed(oracle_mod):
    s = scenegen.mixed_tiny_scene()
    cam = scenegen.Camera((0.0, 4.0, 30.0), (0.0, -2.0, 0.0), (0.0, 1.0, 0.0), 50.0, 96, 80)
    p = scenegen.Params(ao_samples=8, seed=3)
    brute = oracle_mod.render(s, cam, p, grid=None)
    n_tri = s.n_spheres + s.n_cylinders
    assert (brute["hit_id"] >= n_tri).sum() > 500  # triangles are seen
    for lam in (1.0, 4.0, 24.0):
        g = oracle_mod.render(s, cam, p, grid=lam)
        for k in ("hit_id", "ao_mask", "light_mask", "t", "rgb"):
            assert np.array_equal(brute[k], g[k]), (lam, k)
    assert brute["counters"]["tri_tests"] > 0


def test_lit_triangle_closed_form(oracle_mod):
    # a large triangle in the plane z = 0, seen from above and from below
    big = [[-50.0, -50.0, 0.0], [50.0, -50.0, 0.0], [0.0, 60.0, 0.0]]
    L = np.array([0.3, 0.4, 1.0])
    Ln = L / np.linalg.norm(L)
    s = _one_triangle_scene([big], albedo=0.6, lights=[L])
    alb = float(np.float32(0.6))
    for eye, lit in (((2.0, 1.0, 20.0), True), ((2.0, 1.0, -20.0), False)):
        cam = scenegen.Camera(eye, (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 40.0, 32, 32)
        out = oracle_mod.render(s, cam, scenegen.Params(ao_samples=0, light_rescale=0.3,
                                                        skylight=0.5), grid=None)
        hit = out["hit_id"] == 0
        assert hit.all()
        # seen from below, the normal faces down, away from the light
        want = alb * (0.3 * (Ln[2] if lit else 0.0) + 0.5)
        assert np.abs(out["rgb"] - want).max() < 1e-12


def test_ao_beside_sphere_on_triangle(oracle_mod):
    # probe P on a large triangle (plane z = 0, N = +z); occluder: unit sphere
    # at distance 3 along N -> cosine-weighted visibility 1 - (1/3)^2 = 8/9
    big = [[-50.0, -50.0, 0.0], [50.0, -50.0, 0.0], [0.0, 60.0, 0.0]]
    P = np.array([0.0, 0.0, 0.0])
    s = _one_triangle_scene([big], albedo=1.0, lights=[], spheres=[[0.0, 0.0, 3.0]], radii=[1.0])
    eye = P + 10.0 * np.array([1.0, 0.0, 1.0]) / math.sqrt(2.0)
    cam = scenegen.Camera(tuple(eye), tuple(P), (0.0, 1.0, 0.0), 1e-3, 1, 1)
    S = 65536
    out = oracle_mod.render(s, cam, scenegen.Params(ao_samples=S, seed=8), grid=None)
    n_s = 1
    assert out["hit_id"][0, 0] == n_s  # the triangle (after the sphere)
    ao = 1.0 - out["ao_occluded"][0, 0] / S
    expect = 8.0 / 9.0
    assert abs(ao - expect) <= 4.0 * math.sqrt(expect * (1 - expect) / S), ao
