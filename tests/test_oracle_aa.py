"""Pins of the oracle's antialiasing (several primary samples per pixel).

Sample 0 of a pixel is its centre, so one sample is the plain renderer; the
other samples sit at uniform random points of the pixel square, and the
pixel's colour is the mean of its samples' colours.  What pins it:
  * the sub-pixel camera map agrees with the pixel-centre camera and with the
    closed-form angle of the image corner;
  * the offsets are uniform on the pixel square (chi-squared) on a 2^-24 grid;
  * a lone sphere lit only by the sky (AO off, so a hit pixel is its albedo)
    gives, per pixel, the covered fraction of the pixel square, which a fine
    sub-pixel grid computes from the closed-form silhouette of a sphere seen
    from a point (a cone of half-angle asin(r / D)) -- per pixel within a
    binomial bound and, summed over the edge pixels, without bias;
  * every primary sample draws its own AO directions: with one AO ray per
    sample, the mean over many samples still converges to the closed-form
    cosine-weighted visibility 8/9 beside a sphere.
CPU only."""
import math

import numpy as np
import pytest

import scenegen


def _scene(spheres, radii, lights=(), albedo=0.5):
    spheres = np.array(spheres, dtype=np.float64).reshape(-1, 3)
    radii = np.array(radii, dtype=np.float64)
    ld = np.array(lights, dtype=np.float64).reshape(-1, 3)
    z3 = np.zeros((0, 3))
    return scenegen.Scene(spheres, radii, np.full((len(radii), 3), albedo, np.float32),
                          z3, z3.copy(), np.zeros(0), np.zeros((0, 3), np.float32),
                          ld, np.ones_like(ld))


def test_one_sample_is_the_plain_renderer(oracle_mod):
    s, c, p = scenegen.tiny_workload()
    c = scenegen.Camera(c.eye, c.lookat, c.up, c.fovy_deg, 40, 32)
    base = oracle_mod.render(s, c, p, grid=4.0)
    for a in (0, 1):
        q = scenegen.Params(**{**p.__dict__, "aa_samples": a})
        out = oracle_mod.render(s, c, q, grid=4.0)
        for k in ("rgb", "hit_id", "ao_mask", "light_mask", "ao_occluded", "t"):
            assert np.array_equal(out[k], base[k]), (a, k)
        assert out["counters"] == base["counters"]


def test_camera_ray_at_matches_centre_and_corner(oracle_mod):
    cam = scenegen.Camera((1.0, 2.0, 30.0), (0.5, -1.0, 0.0), (0.0, 1.0, 0.0), 50.0, 33, 21)
    for i, j in ((0, 0), (16, 10), (32, 20), (7, 13)):
        o0, d0 = oracle_mod.camera_ray(cam, i, j)
        o1, d1 = oracle_mod.camera_ray_at(cam, i + 0.5, j + 0.5)
        assert np.array_equal(o0, o1) and np.array_equal(d0, d1)
    # the image corners lie atan(th * sqrt(aspect^2 + 1)) off the view axis
    th = math.tan(math.radians(25.0))
    a = 33 / 21
    f = np.subtract(cam.lookat, cam.eye)
    f /= np.linalg.norm(f)
    want = math.atan(th * math.sqrt(a * a + 1.0))
    for px, py in ((0.0, 0.0), (33.0, 0.0), (0.0, 21.0), (33.0, 21.0)):
        _, d = oracle_mod.camera_ray_at(cam, px, py)
        assert abs(math.acos(min(1.0, float(d @ f))) - want) < 1e-12
    # the image centre is the view axis
    _, d = oracle_mod.camera_ray_at(cam, 16.5, 10.5)
    assert np.allclose(d, f, atol=1e-15)


def test_offsets_uniform_on_pixel_square(oracle_mod):
    assert oracle_mod.aa_offset(123, 0, 5, 99) == (0.5, 0.5)
    n = 1 << 15
    xs = np.empty(n)
    ys = np.empty(n)
    for q in range(n):
        xs[q], ys[q] = oracle_mod.aa_offset(q // 8, 1 + q % 8, 3, 0x1234_5678_9ABC)
    assert np.all((xs >= 0) & (xs < 1) & (ys >= 0) & (ys < 1))
    assert np.all(xs * 2**24 == np.floor(xs * 2**24)) and np.all(ys * 2**24 == np.floor(ys * 2**24))
    h, _, _ = np.histogram2d(xs, ys, bins=16, range=[[0, 1], [0, 1]])
    e = n / 256.0
    chi2 = float(((h - e) ** 2 / e).sum())
    # 255 degrees of freedom: mean 255, sd 22.6; 6 sd either side
    assert 255 - 6 * 22.6 < chi2 < 255 + 6 * 22.6, chi2
    # not the AO stream of the same pixel (different counter word 3)
    for q in range(64):
        assert oracle_mod.aa_offset(q, 3, 1, 7) != oracle_mod.ao_uniforms_aa(q, 3, 1, 0, 7)


def test_coverage_of_sphere_silhouette(oracle_mod):
    # Sphere (radius r) on the view axis at distance D: the rays that hit it
    # form a cone of half-angle asin(r / D), so image point (x, y) on the plane
    # at unit distance is covered iff x^2 + y^2 <= r^2 / (D^2 - r^2).
    r, D = 3.0, 20.0
    W = H = 40
    fov = 30.0
    A = 256
    alb = 0.5
    s = _scene([[0.0, 0.0, 0.0]], [r], albedo=alb)
    cam = scenegen.Camera((0.0, 0.0, D), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), fov, W, H)
    p = scenegen.Params(ao_samples=0, light_rescale=0.3, skylight=1.0, aa_samples=A, seed=5)
    out = oracle_mod.render(s, cam, p, grid=None)
    est = out["rgb"][..., 0] / alb
    assert np.array_equal(out["rgb"][..., 0], out["rgb"][..., 2])
    assert out["counters"]["primary_rays"] == W * H * A
    th = math.tan(math.radians(fov / 2))
    rho2 = r * r / (D * D - r * r)

    def covered(px, py):
        x = (2.0 * px / W - 1.0) * th * (W / H)
        y = (1.0 - 2.0 * py / H) * th
        return x * x + y * y <= rho2

    n_sub = 256
    sub = (np.arange(n_sub) + 0.5) / n_sub
    z_sum = 0.0
    var_sum = 0.0
    n_edge = 0
    for j in range(H):
        for i in range(W):
            corners = [covered(i + u, j + v) for u in (0.0, 1.0) for v in (0.0, 1.0)]
            if all(corners) or not any(corners):
                # the disc is convex and smaller than the frame: a pixel whose
                # corners agree lies wholly inside or outside it (none of these
                # pixels can hold the whole silhouette)
                want = 1.0 if all(corners) else 0.0
                assert est[j, i] == want, (i, j)
                continue
            gx, gy = np.meshgrid(i + sub, j + sub)
            f = float(covered(gx, gy).mean())
            sd = math.sqrt(max(f * (1 - f), 1e-4) / A)
            assert abs(est[j, i] - f) <= 4.5 * sd + 0.01, (i, j, est[j, i], f)
            z_sum += est[j, i] - f
            var_sum += f * (1 - f) / A
            n_edge += 1
    assert n_edge > 40
    # no bias over the silhouette (a shifted or scaled sample square shows here)
    assert abs(z_sum) <= 4.5 * math.sqrt(var_sum) + n_edge * 2e-3, (z_sum, var_sum, n_edge)
    # sample 0 is the pixel centre: hit ids follow the centre ray
    for j in range(H):
        for i in range(W):
            assert (out["hit_id"][j, i] == 0) == covered(i + 0.5, j + 0.5)


def test_each_sample_draws_its_own_ao(oracle_mod):
    # The probe of the AO closed form (visibility 8/9 beside a sphere) with a
    # field of view so narrow that every primary sample hits the same point:
    # one AO ray per sample, so only independent streams per sample converge.
    P = np.array([1.0, 0.0, 0.0])
    occ = P + 3.0 * np.array([1.0, 0.0, 0.0])
    s = _scene([[0.0, 0.0, 0.0], occ], [1.0, 1.0], albedo=1.0)
    eye = P + 10.0 * np.array([1.0, 1.0, 0.0]) / math.sqrt(2.0)
    cam = scenegen.Camera(tuple(eye), tuple(P), (0.0, 0.0, 1.0), 0.01, 1, 1)
    A = 16384
    p = scenegen.Params(ao_samples=1, light_rescale=0.3, skylight=1.0, aa_samples=A, seed=77)
    out = oracle_mod.render(s, cam, p, grid=None)
    assert out["counters"]["ao_rays"] == A
    expect = 8.0 / 9.0
    ao = float(out["rgb"][0, 0, 0])
    tol = 4.0 * math.sqrt(expect * (1 - expect) / A) + 2e-3
    assert abs(ao - expect) <= tol, (ao, expect, tol)
