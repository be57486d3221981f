"""Pins of the oracle's transparency (the -trans_vmd option of the paper's
rendering commands, read as front-to-back compositing of up to max_layers
surfaces; shadow and AO rays see every primitive as opaque).
  * without layers (max_layers <= 1), or with every opacity 1, the renderer
    is the opaque one bit for bit;
  * closed form on the axis through a transparent sphere in front of an
    opaque one: front face, inside of the back face (lit only by the sky: the
    sphere shadows its own far side), then the opaque sphere (in the
    transparent sphere's shadow): alpha C0 + (1 - alpha) alpha C1 +
    (1 - alpha)^2 C2, and with two layers the background in place of C2;
  * pixels whose first surface is opaque are the opaque renderer's.
CPU only."""
import numpy as np

import scenegen


def _scene(spheres, radii, albedo, opacity, lights):
    spheres = np.array(spheres, dtype=np.float64).reshape(-1, 3)
    radii = np.array(radii, dtype=np.float64)
    alb = np.array(albedo, dtype=np.float32).reshape(-1, 1).repeat(3, axis=1)
    ld = np.array(lights, dtype=np.float64).reshape(-1, 3)
    z3 = np.zeros((0, 3))
    return scenegen.Scene(spheres, radii, np.ascontiguousarray(alb), z3, z3.copy(), np.zeros(0),
                          np.zeros((0, 3), np.float32), ld, np.ones_like(ld),
                          sph_opacity=np.array(opacity, dtype=np.float32),
                          cyl_opacity=np.zeros(0, np.float32))


def test_opaque_cases_are_plain(oracle_mod):
    s, c, p = scenegen.tiny_workload()
    base = oracle_mod.render(s, c, p, grid=4.0)
    rng = np.random.default_rng(4)
    st = scenegen.Scene(**{**s.__dict__,
                           "sph_opacity": rng.uniform(0.2, 0.9, s.n_spheres).astype(np.float32)})
    so = scenegen.Scene(**{**s.__dict__, "sph_opacity": np.ones(s.n_spheres, np.float32)})
    cases = [(st, 0), (st, 1), (so, 8)]
    for sc, L in cases:
        q = scenegen.Params(**{**p.__dict__, "max_layers": L})
        out = oracle_mod.render(sc, c, q, grid=4.0)
        for k in ("rgb", "hit_id", "ao_mask", "light_mask", "t"):
            assert np.array_equal(out[k], base[k]), (L, k)
    # and with layers on, a transparent scene really differs
    q = scenegen.Params(**{**p.__dict__, "max_layers": 8})
    out = oracle_mod.render(st, c, q, grid=4.0)
    assert np.array_equal(out["hit_id"], base["hit_id"])
    assert np.abs(out["rgb"] - base["rgb"]).max() > 0.05


def test_axis_closed_form(oracle_mod):
    a1, a2, alpha = 0.7, 0.5, 0.4
    lam, sky = 0.3, 0.6
    s = _scene([[0.0, 0.0, 0.0], [0.0, 0.0, -10.0]], [2.0, 3.0], [a1, a2], [alpha, 1.0],
               lights=[[0.0, 0.0, 1.0]])
    cam = scenegen.Camera((0.0, 0.0, 30.0), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 30.0, 31, 31)
    bg = (0.1, 0.2, 0.3)
    f1, f2 = float(np.float32(a1)), float(np.float32(a2))
    fa = float(np.float32(alpha))
    C0 = f1 * (lam * 1.0 + sky)  # front pole: lit head-on, AO = 1 (S = 0)
    C1 = f1 * sky                # inside of the back pole: the sphere shadows it
    C2 = f2 * sky                # opaque sphere: in the transparent sphere's shadow
    for L, want in ((8, [fa * C0 + (1 - fa) * fa * C1 + (1 - fa) ** 2 * C2] * 3),
                    (2, [fa * C0 + (1 - fa) * fa * C1 + (1 - fa) ** 2 * b for b in bg]),
                    (1, [C0] * 3)):
        p = scenegen.Params(ao_samples=0, light_rescale=lam, skylight=sky, max_layers=L,
                            background=bg)
        out = oracle_mod.render(s, cam, p, grid=None)
        got = out["rgb"][15, 15]
        assert np.allclose(got, want, rtol=0, atol=1e-12), (L, got, want)
        assert out["hit_id"][15, 15] == 0 and abs(out["t"][15, 15] - 28.0) < 1e-12
        assert out["light_mask"][15, 15] == 0


def test_opaque_first_surface_unchanged(oracle_mod):
    s = _scene([[0.0, 0.0, 0.0], [3.0, 0.0, -10.0]], [2.0, 5.0], [0.7, 0.5], [0.4, 1.0],
               lights=[[0.3, 0.2, 1.0]])
    cam = scenegen.Camera((0.0, 0.0, 30.0), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 30.0, 64, 64)
    p1 = scenegen.Params(ao_samples=16, seed=9, max_layers=1)
    p8 = scenegen.Params(ao_samples=16, seed=9, max_layers=8)
    o1 = oracle_mod.render(s, cam, p1, grid=None)
    o8 = oracle_mod.render(s, cam, p8, grid=None)
    for k in ("hit_id", "ao_mask", "light_mask", "t"):
        assert np.array_equal(o1[k], o8[k]), k
    back = o1["hit_id"] == 1
    front = o1["hit_id"] == 0
    assert back.sum() > 100 and front.sum() > 100
    assert np.array_equal(o1["rgb"][back], o8["rgb"][back])
    assert np.abs(o1["rgb"][front] - o8["rgb"][front]).max() > 0.01


def _sphere_roots(c, r, o, d):
    q = o - c
    b = q @ d
    disc = b * b - (q @ q - r * r)
    if disc < 0:
        return None
    sq = np.sqrt(disc)
    return -b - sq, -b + sq


def test_every_pixel_closed_form(oracle_mod):
    # Each camera ray through the transparent sphere meets: its front face
    # (entry root), the inside of its far face (exit root; any light ray from
    # there crosses the sphere, so only the sky lights it), then the opaque
    # sphere behind or the background; the opaque sphere is lit unless the
    # transparent one (opaque to shadow rays) lies on the way to the light.
    c0, r0 = np.array([0.0, 0.0, 0.0]), 2.0
    c1, r1 = np.array([1.0, 0.5, -8.0]), 4.0
    a1, a2, alpha = 0.7, 0.5, 0.35
    lam, sky = 0.3, 0.6
    Ld = np.array([0.2, -0.3, 1.0])
    L = Ld / np.linalg.norm(Ld)
    s = _scene([c0, c1], [r0, r1], [a1, a2], [alpha, 1.0], lights=[Ld])
    cam = scenegen.Camera((0.0, 0.0, 30.0), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 25.0, 41, 41)
    bg = np.array([0.05, 0.1, 0.15])
    p = scenegen.Params(ao_samples=0, light_rescale=lam, skylight=sky, max_layers=8,
                        background=tuple(bg))
    out = oracle_mod.render(s, cam, p, grid=None)
    f1, f2, fa = (float(np.float32(x)) for x in (a1, a2, alpha))

    def opaque_colour(o, d):
        h = _sphere_roots(c1, r1, o, d)
        if h is None or h[1] <= 1e-4:
            return bg
        t = h[0] if h[0] > 1e-4 else h[1]
        P = o + t * d
        N = (P - c1) / r1
        if N @ d > 0:
            N = -N
        lit = 0.0
        if N @ L > 0:
            sh = _sphere_roots(c0, r0, P, L)
            blocked = sh is not None and sh[1] > 1e-4
            lit = 0.0 if blocked else N @ L
        return np.full(3, f2 * (lam * lit + sky))

    n_through = 0
    for j in range(cam.height):
        for i in range(cam.width):
            o, d = oracle_mod.camera_ray(cam, i, j)
            h = _sphere_roots(c0, r0, o, d)
            if h is None or h[0] <= 0:
                want = opaque_colour(o, d)
                # an opaque first surface: the transparent sphere only shadows
            else:
                n_through += 1
                P0 = o + h[0] * d
                N0 = (P0 - c0) / r0
                C0 = f1 * (lam * max(0.0, N0 @ L) + sky)
                C1 = f1 * sky
                P1 = o + h[1] * d
                C2 = opaque_colour(P1, d)
                want = fa * C0 + (1 - fa) * fa * C1 + (1 - fa) ** 2 * C2
            assert np.allclose(out["rgb"][j, i], want, rtol=0, atol=1e-9), (i, j, out["rgb"][j, i], want)
    assert n_through > 100
