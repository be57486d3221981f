"""Pins of the oracle's tie-break (reading A15: the paper is silent on equal
distances, Sec. 2; the nearest hit is the lexicographic minimum of (t, id),
so of two primitives hit at the same t the smaller global id wins).

Exact duplicates of spheres and cylinders are hit at bit-equal t, and so are
two spheres tangent at the point a ray enters them.  Every traversal the
oracle offers -- brute force in id order, brute force in any given order, and
its uniform grid at several densities -- must report the smaller id.  A
`<=` for `<`, a reversed id comparison, or a dropped tie clause (caught by
the descending visiting order) each fails a case here.
"""
import math

import numpy as np
import pytest

import oracle
import scenegen


def _dup_scene():
    """Spheres 0..5 and cylinders 6..9 with exact duplicates: sphere 1 == 3,
    sphere 4 == 5, cylinder 6 == 8; plus two spheres (0 and 2) tangent
    internally at (0, 0, -1), which a ray along +z from z = -10 enters at the
    same t = 9 exactly."""
    sc = np.array([[0.0, 0.0, 1.0],     # 0: radius 2, touches z = -1 on the axis
                   [6.0, 1.0, 0.5],     # 1
                   [0.0, 0.0, 0.0],     # 2: radius 1, touches z = -1 on the axis
                   [6.0, 1.0, 0.5],     # 3 == 1
                   [-5.0, -4.0, 2.0],   # 4
                   [-5.0, -4.0, 2.0]])  # 5 == 4
    sr = np.array([2.0, 1.25, 1.0, 1.25, 1.5, 1.5])
    ca = np.array([[-2.0, 6.0, -1.0], [3.0, -6.0, 0.0], [-2.0, 6.0, -1.0], [7.0, 7.0, 7.0]])
    cb = np.array([[2.0, 6.5, 1.0], [4.0, -3.0, 1.0], [2.0, 6.5, 1.0], [8.0, 8.0, 8.0]])
    cr = np.array([0.6, 0.4, 0.6, 0.3])
    ld, lc = scenegen._lights(1)
    return scenegen.Scene(sc, sr, scenegen.PALETTE[np.arange(6) % 4], ca, cb, cr,
                          scenegen.PALETTE[np.arange(4) % 4], ld, lc)


# (representative id, its duplicates); the representative is the smallest
GROUPS = [(1, (1, 3)), (4, (4, 5)), (6, (6, 8))]


def _aim(scene, k):
    """A ray from outside the scene at the middle of primitive k."""
    if k < scene.n_spheres:
        c = scene.sph_center[k]
    else:
        m = k - scene.n_spheres
        c = 0.5 * (scene.cyl_a[m] + scene.cyl_b[m])
    o = c + np.array([0.3, 0.2, -20.0])
    d = c - o
    return o, d / np.linalg.norm(d)


def _orders(n, seed=0):
    ids = np.arange(n)
    rng = np.random.default_rng(seed)
    return [ids, ids[::-1].copy(), rng.permutation(n), rng.permutation(n)]


@pytest.mark.parametrize("rep,dups", GROUPS)
def test_duplicates_report_smallest_id(rep, dups):
    scene = _dup_scene()
    n = scene.n_prims
    o, d = _aim(scene, rep)
    t_bf, k_bf = oracle.trace(scene, None, o, d)
    assert k_bf == rep and math.isfinite(t_bf)
    for order in _orders(n):
        t, k = oracle.trace_list(scene, order, o, d)
        assert (t, k) == (t_bf, rep), order
    # only the duplicates, largest first
    t, k = oracle.trace_list(scene, np.array(sorted(dups, reverse=True)), o, d)
    assert (t, k) == (t_bf, rep)
    for lam in (0.5, 4.0, 24.0):
        g = oracle.Grid(scene, lam)
        t, k = oracle.trace(scene, g, o, d)
        assert (t, k) == (t_bf, rep), lam


def test_tangent_spheres_equal_t():
    scene = _dup_scene()
    o, d = np.array([0.0, 0.0, -10.0]), np.array([0.0, 0.0, 1.0])
    # both roots are 9 exactly: 11 - 2 for sphere 0, 10 - 1 for sphere 2
    t0, t2 = oracle.hit_sphere(scene.sph_center[0], 2.0, o, d), oracle.hit_sphere(
        scene.sph_center[2], 1.0, o, d)
    assert t0 == t2 == 9.0
    for order in _orders(scene.n_prims, seed=1):
        assert oracle.trace_list(scene, order, o, d) == (9.0, 0)
    assert oracle.trace_list(scene, np.array([2, 0]), o, d) == (9.0, 0)
    assert oracle.trace(scene, None, o, d) == (9.0, 0)
    for lam in (0.5, 4.0, 24.0):
        assert oracle.trace(scene, oracle.Grid(scene, lam), o, d) == (9.0, 0)


def test_rendered_hit_ids_take_the_smallest_duplicate():
    scene = _dup_scene()
    cam = scenegen.Camera((0.0, 0.0, 30.0), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 50.0, 96, 96)
    params = scenegen.Params(ao_samples=4, seed=3)
    ref = oracle.render(scene, cam, params, grid=None)
    hid = ref["hit_id"]
    # the larger member of each duplicate group is never reported
    for rep, dups in GROUPS:
        assert (hid == rep).sum() > 20, rep
        for k in dups:
            if k != rep:
                assert not (hid == k).any(), k
    for lam in (0.5, 4.0, 24.0):
        g = oracle.render(scene, cam, params, grid=oracle.Grid(scene, lam))
        np.testing.assert_array_equal(g["hit_id"], hid)
        np.testing.assert_array_equal(g["rgb"], ref["rgb"])
