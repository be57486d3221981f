"""Pins of the oracle's Phong highlight (a shading option: strength k_s,
exponent n; white, added after the albedo-scaled diffuse and sky terms).
  * k_s = 0 is the plain renderer bit for bit, whatever n;
  * at the mirror point (light behind the camera, the sphere's pole seen by
    the centre ray) the highlight is exactly rescale * k_s;
  * the brightest highlight pixel is where the reflection law puts it: the
    point whose normal bisects the light and eye directions, found by an
    independent fixed-point solve and projected through the camera;
  * the highlight is a power law: (H_n1 / c)^(n2 / n1) = H_n2 / c per pixel;
  * it never exceeds rescale * k_s and vanishes where the light is shadowed.
CPU only."""
import math

import numpy as np

import scenegen


def _scene(spheres, radii, lights, albedo=0.3):
    spheres = np.array(spheres, dtype=np.float64).reshape(-1, 3)
    radii = np.array(radii, dtype=np.float64)
    ld = np.array(lights, dtype=np.float64).reshape(-1, 3)
    z3 = np.zeros((0, 3))
    return scenegen.Scene(spheres, radii, np.full((len(radii), 3), albedo, np.float32),
                          z3, z3.copy(), np.zeros(0), np.zeros((0, 3), np.float32),
                          ld, np.ones_like(ld))


def _p(**kw):
    base = dict(ao_samples=0, light_rescale=0.3, skylight=0.5, seed=3)
    base.update(kw)
    return scenegen.Params(**base)


def _highlight(oracle_mod, s, cam, ks, n, grid=None):
    on = oracle_mod.render(s, cam, _p(specular=ks, shininess=n), grid=grid)
    off = oracle_mod.render(s, cam, _p(), grid=grid)
    return on, off, on["rgb"][..., 0] - off["rgb"][..., 0]


def test_zero_strength_is_plain(oracle_mod):
    s, c, p = scenegen.tiny_workload()
    base = oracle_mod.render(s, c, p, grid=4.0)
    for n in (1.0, 20.0, 300.0):
        q = scenegen.Params(**{**p.__dict__, "specular": 0.0, "shininess": n})
        out = oracle_mod.render(s, c, q, grid=4.0)
        for k in ("rgb", "hit_id", "ao_mask", "light_mask"):
            assert np.array_equal(out[k], base[k]), (n, k)


def test_mirror_point_closed_form(oracle_mod):
    s = _scene([[0.0, 0.0, 0.0]], [3.0], lights=[[0.0, 0.0, 1.0]], albedo=0.3)
    cam = scenegen.Camera((0.0, 0.0, 20.0), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 30.0, 41, 41)
    out = oracle_mod.render(s, cam, _p(specular=0.4, shininess=35.0))
    # centre ray: d = -z, hits the pole, N = L = V: diffuse 1, mirror R.V = 1
    want = float(np.float32(0.3)) * (0.3 * 1.0 + 0.5) + 0.3 * 0.4
    assert abs(out["rgb"][20, 20, 0] - want) < 1e-12, (out["rgb"][20, 20], want)


def test_highlight_follows_reflection_law(oracle_mod):
    r = 3.0
    eye = np.array([0.0, 0.0, 20.0])
    L = np.array([1.0, 1.0, 2.0]) / math.sqrt(6.0)
    s = _scene([[0.0, 0.0, 0.0]], [r], lights=[L])
    W = H = 161
    fov = 20.0
    cam = scenegen.Camera(tuple(eye), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), fov, W, H)
    ks, n = 0.5, 60.0
    _, off, h = _highlight(oracle_mod, s, cam, ks, n)
    # the highlight peak: N(P) bisects L and the direction to the eye
    N = L + eye / np.linalg.norm(eye)
    N /= np.linalg.norm(N)
    for _ in range(200):
        P = r * N
        V = (eye - P) / np.linalg.norm(eye - P)
        N = (L + V) / np.linalg.norm(L + V)
    P = r * N
    # project P: camera looks down -z with up +y, so right = +x
    d = (P - eye) / np.linalg.norm(P - eye)
    th = math.tan(math.radians(fov / 2))
    x = d[0] / -d[2]
    y = d[1] / -d[2]
    px = (x / (th * W / H) + 1.0) * W / 2.0
    py = (1.0 - y / th) * H / 2.0
    j, i = np.unravel_index(np.argmax(h), h.shape)
    assert abs((i + 0.5) - px) <= 1.0 and abs((j + 0.5) - py) <= 1.0, ((i, j), (px, py))
    c = 0.3 * ks
    assert h.max() <= c + 1e-12
    assert h.max() >= 0.95 * c
    assert np.all(h[off["hit_id"] < 0] == 0)


def test_power_law(oracle_mod):
    s = _scene([[0.0, 0.0, 0.0]], [3.0], lights=[[0.3, 0.5, 1.0]])
    cam = scenegen.Camera((0.0, 0.0, 20.0), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 25.0, 64, 64)
    ks = 0.2
    c = 0.3 * ks
    _, _, h1 = _highlight(oracle_mod, s, cam, ks, 8.0)
    _, _, h2 = _highlight(oracle_mod, s, cam, ks, 32.0)
    lit = h1 > 1e-6 * c
    assert lit.sum() > 300
    lhs = (h1[lit] / c) ** 4
    assert np.allclose(lhs, h2[lit] / c, rtol=1e-6, atol=1e-12)


def test_no_highlight_in_shadow(oracle_mod):
    # a small sphere between the big one and the light shadows part of it
    L = np.array([0.0, 0.0, 1.0])
    s = _scene([[0.0, 0.0, 0.0], [0.0, 0.0, 6.0]], [3.0, 0.8], lights=[L])
    cam = scenegen.Camera((0.0, 8.0, 20.0), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 30.0, 96, 96)
    on, off, h = _highlight(oracle_mod, s, cam, 0.5, 4.0)
    shadowed = (off["hit_id"] == 0) & ((off["light_mask"] & 1) == 1)
    assert shadowed.sum() > 30
    assert np.all(h[shadowed] == 0)
    assert np.array_equal(on["light_mask"], off["light_mask"])
    assert (h[(off["hit_id"] == 0) & ~shadowed] > 0).sum() > 100
