"""Pins of the light rule (reading A8 with its threshold; the paper names
the -rescale_lights option and no shading model, Sec. 2): a light counts,
and casts its shadow ray, when N.L > 2^-40.

- A face exactly perpendicular to a light (N.L = 0) casts no shadow ray.
- A face whose N.L is rounding noise of zero (about 1e-15: an unrotated
  icosphere face perpendicular to a light) casts none either; with the
  plain test N.L > 0 it would, and that ray would run along the surface.
- A light tilted 1e-9 above the face casts its ray, and lights the face by
  rescale * 1e-9 * I.
"""
import math

import numpy as np

import oracle
import scenegen


def _floor_scene(light):
    """A large triangle in the plane y = 0 (normal +-y) and one light."""
    tri = np.array([[[-50.0, 0.0, -50.0], [50.0, 0.0, -50.0], [0.0, 0.0, 60.0]]])
    e3 = np.zeros((0, 3))
    s = scenegen.Scene(e3, np.zeros(0), np.zeros((0, 3), np.float32), e3, e3, np.zeros(0),
                       np.zeros((0, 3), np.float32), np.array([light], dtype=np.float64),
                       np.ones((1, 3)))
    return scenegen.with_triangles(s, tri, np.full((1, 3), 0.5, np.float32))


def _top_view(W=16, H=12):
    return scenegen.Camera((0.0, 20.0, 5.0), (0.0, 0.0, 0.0), (0.0, 0.0, -1.0), 40.0, W, H)


def test_perpendicular_light_casts_nothing():
    s = _floor_scene((1.0, 0.0, 0.0))  # N.L = 0 exactly
    p = scenegen.Params(ao_samples=4, seed=1)
    r = oracle.render(s, _top_view(), p, grid=None)
    assert (r["hit_id"] == 0).all()
    assert r["counters"]["shadow_rays"] == 0
    assert (r["light_mask"] == 0).all()
    # nothing occludes the sky over the floor: colour = albedo * skylight
    np.testing.assert_allclose(r["rgb"], 0.5, rtol=0, atol=1e-12)


def test_tilted_light_counts():
    eps = 1e-9
    s = _floor_scene((1.0, eps, 0.0))
    p = scenegen.Params(ao_samples=4, seed=1)
    r = oracle.render(s, _top_view(), p, grid=None)
    n_hit = int((r["hit_id"] >= 0).sum())
    assert r["counters"]["shadow_rays"] == n_hit
    c = eps / math.sqrt(1.0 + eps * eps)
    np.testing.assert_allclose(r["rgb"], 0.5 * (0.3 * c + 1.0), rtol=0, atol=1e-15)


def _dot(a, b):
    return (a[0] * b[0] + a[1] * b[1]) + a[2] * b[2]


def _unit(v):
    m = math.sqrt(_dot(v, v))
    return [v[0] / m, v[1] / m, v[2] / m]


def test_noise_level_light_casts_nothing():
    # An unrotated icosphere blob (subdivision 2): some faces are
    # perpendicular to the first light up to rounding.  Their N.L, formed
    # in the oracle's order of operations (unit e1 x e2, unit light), is a
    # positive noise value of about 1e-15 for at least one face: with the
    # plain test N.L > 0 that face would send shadow rays along itself.
    verts, faces = scenegen.icosphere(2)
    ctr = np.array([3.0, 1.0, -2.0])
    tri = (ctr + 4.0 * verts[faces]).reshape(-1, 3, 3)
    e3 = np.zeros((0, 3))
    ld, lc = scenegen._lights(2)
    s = scenegen.with_triangles(
        scenegen.Scene(e3, np.zeros(0), np.zeros((0, 3), np.float32), e3, e3, np.zeros(0),
                       np.zeros((0, 3), np.float32), ld, lc), tri)
    L = [_unit(list(map(float, l))) for l in ld]
    pick = None
    for k in range(tri.shape[0]):
        v0, v1, v2 = (list(map(float, x)) for x in tri[k])
        e1 = [v1[q] - v0[q] for q in range(3)]
        e2 = [v2[q] - v0[q] for q in range(3)]
        c = [e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
             e1[0] * e2[1] - e1[1] * e2[0]]
        n = _unit(c)  # outward: the faces wind counter-clockwise from outside
        nl = [_dot(n, l) for l in L]
        if any(0.0 < x <= 2.0 ** -40 for x in nl):
            pick = (k, n, nl)
            break
    assert pick is not None
    k, n, nl = pick
    cen = tri[k].mean(axis=0)
    up = np.cross(n, [0.3, 0.5, 0.8])
    cam = scenegen.Camera(tuple(cen + 30.0 * np.array(n)), tuple(cen), tuple(up), 0.5, 3, 3)
    p = scenegen.Params(ao_samples=0, seed=1)
    r = oracle.render(s, cam, p, grid=None)
    on_face = int((r["hit_id"] == k).sum())
    assert r["hit_id"][1, 1] == k and on_face == 9
    # only the lights with N.L > 2^-40 send rays
    lit = sum(1 for x in nl if x > 2.0 ** -40)
    assert r["counters"]["shadow_rays"] == lit * on_face
    assert (r["light_mask"] & sum(1 << i for i, x in enumerate(nl) if x <= 2.0 ** -40) == 0).all()
