"""Pins of the oracle's renderer: grid == brute force (bit exact), direct light
of a lone sphere in closed form, AO = 1 when nothing occludes, and the closed
form of the cosine-weighted visibility of a point beside a sphere.  CPU only."""
import math

import numpy as np
import pytest

import scenegen


def _scene(spheres, radii, cyls=(), lights=((0.0, 0.0, 1.0),), albedo=0.8):
    spheres = np.array(spheres, dtype=np.float64).reshape(-1, 3)
    radii = np.array(radii, dtype=np.float64)
    ca = np.array([c[0] for c in cyls], dtype=np.float64).reshape(-1, 3)
    cb = np.array([c[1] for c in cyls], dtype=np.float64).reshape(-1, 3)
    cr = np.array([c[2] for c in cyls], dtype=np.float64)
    ld = np.array(lights, dtype=np.float64).reshape(-1, 3)
    return scenegen.Scene(spheres, radii, np.full((len(radii), 3), albedo, np.float32),
                          ca, cb, cr, np.full((len(cr), 3), albedo, np.float32),
                          ld, np.ones_like(ld))


def test_grid_equals_brute_force_tiny(oracle_mod):
    s, c, p = scenegen.tiny_workload()
    brute = oracle_mod.render(s, c, p, grid=None)
    for lam in (0.5, 4.0, 30.0):
        grid = oracle_mod.render(s, c, p, grid=lam)
        for k in ("hit_id", "ao_mask", "light_mask", "ao_occluded"):
            assert np.array_equal(brute[k], grid[k]), (lam, k)
        assert np.array_equal(brute["t"], grid["t"])
        assert np.array_equal(brute["rgb"], grid["rgb"])
    assert (brute["hit_id"] >= 0).sum() > 2000


def test_grid_equals_brute_force_protein_sample(oracle_mod):
    s, c, p = scenegen.protein_workload()
    pix = scenegen.sample_pixels(c.width, c.height, 400, 11)
    brute = oracle_mod.render(s, c, p, grid=None, pix=pix)
    grid = oracle_mod.render(s, c, p, grid=4.0, pix=pix)
    for k in ("hit_id", "ao_mask", "light_mask", "t"):
        assert np.array_equal(brute[k], grid[k]), k
    assert (brute["hit_id"] >= 13159).sum() >= 0  # cylinders may or may not show
    assert (brute["hit_id"] >= 0).sum() > 100


def test_grid_equals_brute_force_cylinders(oracle_mod):
    # bare cylinders (no atoms) so that cylinder hits dominate
    rng = np.random.default_rng(5)
    pos, _ = scenegen.random_walk(300, 12.0, 9)
    s = _scene(np.zeros((0, 3)), [], cyls=[(pos[i], pos[i + 1], 0.4) for i in range(299)],
               lights=(scenegen.LIGHT0, scenegen.LIGHT1))
    cam = scenegen.Camera((0.0, 5.0, 45.0), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 50.0, 96, 80)
    p = scenegen.Params(ao_samples=6, seed=int(rng.integers(1 << 40)))
    brute = oracle_mod.render(s, cam, p, grid=None)
    grid = oracle_mod.render(s, cam, p, grid=3.0)
    for k in ("hit_id", "ao_mask", "light_mask", "t"):
        assert np.array_equal(brute[k], grid[k]), k
    assert (brute["hit_id"] >= 0).sum() > 300


def test_grid_structure(oracle_mod):
    s, _, _ = scenegen.protein_workload()
    g = oracle_mod.Grid(s, 4.0)
    lo, hi, res, n_refs = g.info()
    cb, refs = g.arrays()
    assert cb[0] == 0 and cb[-1] == n_refs and np.all(np.diff(cb.astype(np.int64)) >= 0)
    n_cells = int(np.prod(res.astype(np.int64)))
    assert n_cells == len(cb) - 1
    # ids ascend inside each cell and every primitive is listed somewhere
    seg = np.repeat(np.arange(n_cells), np.diff(cb.astype(np.int64)))
    inner = seg[1:] == seg[:-1]
    assert np.all(refs[1:][inner] > refs[:-1][inner])
    assert len(np.unique(refs)) == s.n_prims
    # every sphere is listed in the cell containing its centre
    h = (hi - lo) / res
    ijk = np.floor((s.sph_center - lo) / h).astype(np.int64)
    cid = (ijk[:, 2] * res[1] + ijk[:, 1]) * res[0] + ijk[:, 0]
    for k in range(0, s.n_spheres, 97):
        assert k in refs[cb[cid[k]]:cb[cid[k] + 1]]


def test_direct_light_lone_sphere_closed_form(oracle_mod):
    # no shadow is possible, S = 0 => AO := 1; the colour has a closed form
    c0 = np.array([0.5, -0.3, 0.2]); r0 = 3.0
    L = np.array([-0.5, 0.5, 1.0]); Ln = L / np.linalg.norm(L)
    s = _scene([c0], [r0], lights=[L], albedo=0.6)
    cam = scenegen.Camera((0.0, 0.0, 20.0), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 30.0, 64, 48)
    p = scenegen.Params(ao_samples=0, light_rescale=0.3, skylight=1.0)
    out = oracle_mod.render(s, cam, p)
    alb = np.float32(0.6)
    n_hit = 0
    for j in range(cam.height):
        for i in range(cam.width):
            o, d = oracle_mod.camera_ray(cam, i, j)
            q = o - c0
            bq = q @ d
            disc = bq * bq - (q @ q - r0 * r0)
            if disc < 0:
                assert out["hit_id"][j, i] == -1 and np.all(out["rgb"][j, i] == 0)
                continue
            n_hit += 1
            t = -bq - math.sqrt(disc)
            P = o + t * d
            N = (P - c0) / r0
            want = min(1.0, float(alb) * (0.3 * max(0.0, N @ Ln) + 1.0))
            assert np.all(np.abs(out["rgb"][j, i] - want) < 1e-12)
            assert out["light_mask"][j, i] == 0
    assert n_hit > 500


def test_ao_one_when_unoccluded(oracle_mod):
    s = _scene([[0.0, 0.0, 0.0]], [4.0], lights=[scenegen.LIGHT0])
    cam = scenegen.Camera((0.0, 0.0, 25.0), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 40.0, 48, 48)
    p = scenegen.Params(ao_samples=32, seed=1234)
    out = oracle_mod.render(s, cam, p)
    hit = out["hit_id"] >= 0
    assert hit.sum() > 300
    assert np.all(out["ao_mask"] == 0) and np.all(out["ao_occluded"] == 0)
    assert out["counters"]["ao_rays"] == 32 * hit.sum()


@pytest.mark.parametrize("alpha_deg,expect", [(0.0, 8.0 / 9.0), (60.0, 17.0 / 18.0)])
def test_ao_closed_form_beside_sphere(oracle_mod, alpha_deg, expect):
    # Probe P = (1,0,0) on the unit sphere, N = +x.  Occluder: radius 1 at
    # distance 3 along a direction alpha from N.  Cosine-weighted visibility
    # = 1 - cos(alpha) (r/d)^2 (occluder fully above the horizon).
    a = math.radians(alpha_deg)
    P = np.array([1.0, 0.0, 0.0])
    occ = P + 3.0 * np.array([math.cos(a), 0.0, math.sin(a)])
    s = _scene([[0.0, 0.0, 0.0], occ], [1.0, 1.0], lights=[])
    eye = P + 10.0 * np.array([1.0, 1.0, 0.0]) / math.sqrt(2.0)
    cam = scenegen.Camera(tuple(eye), tuple(P), (0.0, 0.0, 1.0), 10.0, 1, 1)
    S = 65536
    p = scenegen.Params(ao_samples=S, seed=77)
    out = oracle_mod.render(s, cam, p, grid=None)
    assert out["hit_id"][0, 0] == 0
    assert abs(out["t"][0, 0] - 10.0) < 1e-12
    ao = 1.0 - out["ao_occluded"][0, 0] / S
    tol = 4.0 * math.sqrt(expect * (1 - expect) / S)
    assert abs(ao - expect) <= tol, (ao, expect, tol)
    # the unweighted (uniform-solid-angle) reading would give a different value
    unweighted = 1.0 - (1.0 - math.cos(math.asin(1.0 / 3.0))) if alpha_deg == 0 else None
    if unweighted is not None:
        assert abs(ao - unweighted) > 10 * tol


def test_hemisphere_moments(oracle_mod):
    rng = np.random.default_rng(3)
    for _ in range(4):
        n = rng.standard_normal(3); n /= np.linalg.norm(n)
        cs = []
        for s in range(4000):
            u1, u2 = oracle_mod.ao_uniforms(s, 0, 0, 99)
            w = oracle_mod.ao_direction(n, u1, u2)
            assert abs(np.linalg.norm(w) - 1) < 1e-14
            cs.append(n @ w)
        cs = np.array(cs)
        assert np.all(cs > 0)
        # cosine-weighted: E[cos] = 2/3, E[cos^2] = 1/2
        assert abs(cs.mean() - 2 / 3) < 4 * math.sqrt(1 / 18 / len(cs))
        assert abs((cs ** 2).mean() - 0.5) < 4 * math.sqrt(1 / 12 / len(cs))
    # pole handling of the basis: n = -z and n = +z
    for nz in (-1.0, 1.0):
        w = oracle_mod.ao_direction(np.array([0.0, 0.0, nz]), 0.0, 0.0)
        assert np.allclose(w, [0, 0, nz])


def test_counters_brute_force(oracle_mod):
    # a ray that misses everything tests every primitive exactly once
    s = _scene([[0.0, 0.0, 0.0], [5.0, 0.0, 0.0]], [1.0, 1.0],
               cyls=[((0.0, 3.0, 0.0), (1.0, 3.0, 0.0), 0.2)])
    cnt = oracle_mod.Counters()
    t, k = oracle_mod.trace(s, None, (0.0, 10.0, -10.0), (0.0, 0.0, 1.0), counters=cnt)
    assert k == -1 and cnt.sph_tests == 2 and cnt.cyl_tests == 1 and cnt.rays_traced == 1
