"""Render parity: the plain FP64 GPU path and the FP32 wavefront path against
the FP64 oracle, on the tiny scene, the 26,318-object protein-like scene at
965x1137 (full frame) and 3860x4548 (sampled pixels), ragged frame sizes and
degenerate cases."""
import math

import numpy as np
import pytest

import scenegen
from parity_util import assert_fp32_parity, compare, flat_at, frame_to_numpy

pytestmark = pytest.mark.gpu

OUT = ("rgb", "hit_id", "ao_mask", "light_mask")


@pytest.fixture(scope="module")
def tr():
    import paper_0801_1500_amd as tr
    tr.lib()
    return tr


@pytest.fixture(scope="module")
def protein(tr):
    s = scenegen.protein_scene()
    return s, tr.Scene(s)


def _gpu(tr, gscene, cam, params, precision, tune=None):
    import torch
    fr = tr.render(gscene, cam, params, precision=precision, outputs=OUT, tune=tune)
    torch.cuda.synchronize()
    return frame_to_numpy(fr)


def _ref(oracle_mod, scene, cam, params, pix=None, grid=4.0):
    return oracle_mod.render(scene, cam, params, grid=grid, pix=pix)


def _fp64_exact(m, got, ref):
    # the plain FP64 path reproduces the oracle: same hits, same decisions
    # (AO directions use the device's sin/cos, so allow a vanishing few flips)
    assert m["hit_mismatch"] == 0, m
    assert m["decision_flips"] <= max(2, m["decisions"] // 1000000), m
    assert m["max_abs_agree"] <= 1.2e-7, m  # float32 rounding of the FP64 colour


def test_tiny_fp64(tr, oracle_mod):
    s, c, p = scenegen.tiny_workload()
    print("tiny fp64", flush=True)
    got = _gpu(tr, tr.Scene(s), c, p, "fp64")
    ref = _ref(oracle_mod, s, c, p, grid=None)
    m = compare(got, ref, p.ao_samples, s.n_lights)
    _fp64_exact(m, got, ref)
    assert (got["hit_id"] >= 0).sum() > 2000


@pytest.mark.parametrize("prec", ["fp32", "fp32_resolve"])
def test_tiny_fp32(tr, oracle_mod, prec):
    s, c, p = scenegen.tiny_workload()
    print("tiny", prec, flush=True)
    got = _gpu(tr, tr.Scene(s), c, p, prec)
    ref = _ref(oracle_mod, s, c, p, grid=None)
    m = compare(got, ref, p.ao_samples, s.n_lights)
    print(m)
    assert_fp32_parity(m)


def test_protein_1mp_fp64(tr, oracle_mod, protein):
    s, gs = protein
    c = scenegen.protein_camera(scenegen.RES_1MP)
    p = scenegen.Params(ao_samples=16, seed=2)
    print("protein 1.1MP fp64", flush=True)
    got = _gpu(tr, gs, c, p, "fp64")
    ref = _ref(oracle_mod, s, c, p)
    m = compare(got, ref, 16, s.n_lights)
    print(m)
    _fp64_exact(m, got, ref)


def test_protein_1mp_fp32_resolve(tr, oracle_mod, protein):
    s, gs = protein
    c = scenegen.protein_camera(scenegen.RES_1MP)
    p = scenegen.Params(ao_samples=16, seed=2)
    print("protein 1.1MP fp32_resolve", flush=True)
    got = _gpu(tr, gs, c, p, "fp32_resolve")
    ref = _ref(oracle_mod, s, c, p)
    m = compare(got, ref, 16, s.n_lights)
    print(m)
    assert_fp32_parity(m)
    assert m["hit_agree"] >= 0.99999


@pytest.fixture(scope="module")
def protein_17mp_ref(oracle_mod, protein):
    """The oracle's whole 3860x4548 frame (all 17,555,280 pixels)."""
    s, _ = protein
    c = scenegen.protein_camera(scenegen.RES_17MP)
    p = scenegen.Params(ao_samples=16, seed=2)
    print("oracle 17.6MP full frame", flush=True)
    return _ref(oracle_mod, s, c, p)


@pytest.mark.parametrize("prec", ["fp32_resolve", "fp64"])
def test_protein_17mp_full(tr, protein, protein_17mp_ref, prec):
    # the whole 3860x4548 frame, in the launch shape the benchmark times,
    # against the oracle's whole frame, pixel by pixel
    s, gs = protein
    c = scenegen.protein_camera(scenegen.RES_17MP)
    p = scenegen.Params(ao_samples=16, seed=2)
    print("protein 17.6MP", prec, flush=True)
    got = _gpu(tr, gs, c, p, prec)
    m = compare(got, protein_17mp_ref, 16, s.n_lights)
    print(m, flush=True)
    assert m["n"] == 3860 * 4548
    if prec == "fp64":
        _fp64_exact(m, None, None)
    else:
        assert_fp32_parity(m)
    # every pixel written: hit ids valid, colour in [0, 1]
    assert got["hit_id"].min() >= -1 and got["hit_id"].max() < s.n_prims
    assert np.all(got["rgb"] >= 0) and np.all(got["rgb"] <= 1)


@pytest.mark.parametrize("W,H,tile_w", [(131, 77, 8), (67, 45, 16), (1, 1, 8), (5, 300, 32),
                                        (300, 5, 4), (131, 77, 64), (5, 300, 64)])
def test_ragged_frames(tr, oracle_mod, protein, W, H, tile_w):
    s, gs = protein
    c = scenegen.Camera((10.0, 20.0, 70.0), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 35.0, W, H)
    p = scenegen.Params(ao_samples=8, seed=5)
    print("ragged", W, H, tile_w, flush=True)
    got = _gpu(tr, gs, c, p, "fp32_resolve", tune={"tile_w": tile_w})
    ref = _ref(oracle_mod, s, c, p)
    m = compare(got, ref, 8, s.n_lights)
    assert m["hit_mismatch"] <= max(1, W * H // 10000), m
    assert m["max_abs_agree"] <= 1e-3, m
    got64 = _gpu(tr, gs, c, p, "fp64")
    _fp64_exact(compare(got64, ref, 8, s.n_lights), None, None)


def test_empty_scene(tr):
    s = scenegen.Scene(np.zeros((0, 3)), np.zeros(0), np.zeros((0, 3), np.float32),
                       np.zeros((0, 3)), np.zeros((0, 3)), np.zeros(0), np.zeros((0, 3), np.float32),
                       np.zeros((0, 3)), np.zeros((0, 3)))
    gs = tr.Scene(s)
    c = scenegen.Camera((0.0, 0.0, 10.0), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 50.0, 40, 30)
    p = scenegen.Params(ao_samples=4, background=(0.25, 0.5, 0.75))
    for prec in ("fp32_resolve", "fp64"):
        got = _gpu(tr, gs, c, p, prec)
        assert np.all(got["hit_id"] == -1)
        assert np.allclose(got["rgb"], [0.25, 0.5, 0.75])


@pytest.mark.parametrize("case", ["no_ao", "no_sky", "maxdist", "inside", "many_samples"])
def test_degenerate_params(tr, oracle_mod, case):
    s, c, p = scenegen.tiny_workload()
    if case == "no_ao":
        p.ao_samples = 0
    elif case == "no_sky":
        p.skylight = 0.0
    elif case == "maxdist":
        p.ao_maxdist = 2.5
    elif case == "inside":
        # eye inside the first sphere: back faces, unflipped skip rules
        c = scenegen.Camera(tuple(s.sph_center[0]), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 60.0, 48, 40)
    elif case == "many_samples":
        p.ao_samples = 100
        c = scenegen.Camera(c.eye, c.lookat, c.up, c.fovy_deg, 48, 48)
    print("degenerate", case, flush=True)
    gs = tr.Scene(s)
    out = OUT if p.ao_samples <= 32 else ("rgb", "hit_id", "light_mask")
    import torch
    ref = _ref(oracle_mod, s, c, p, grid=None)
    for prec in ("fp64", "fp32_resolve"):
        fr = frame_to_numpy(tr.render(gs, c, p, precision=prec, outputs=out))
        torch.cuda.synchronize()
        if "ao_mask" not in fr:
            fr["ao_mask"] = np.zeros_like(fr["hit_id"])
            ref = dict(ref)
            ref["ao_mask"] = np.zeros_like(ref["hit_id"])
        m = compare(fr, ref, min(p.ao_samples, 32), s.n_lights)
        print(prec, m, flush=True)
        if prec == "fp64":
            _fp64_exact(m, fr, ref)
        else:  # the same bar as every other frame
            assert_fp32_parity(m)


def test_deterministic_and_tune_independent(tr, protein):
    import torch
    s, gs = protein
    c = scenegen.Camera((0.0, 30.0, 100.0), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 50.0, 320, 240)
    p = scenegen.Params(ao_samples=16, seed=9)
    base = _gpu(tr, gs, c, p, "fp32_resolve")
    again = _gpu(tr, gs, c, p, "fp32_resolve")
    for k in OUT:
        assert np.array_equal(base[k], again[k]), k
    # the tile queue's stripe only changes which XCD takes a tile: 1 deals
    # single tiles round the XCDs, 1024 leaves six XCDs' queues empty (the
    # frame has 1200 tiles), so their waves take every tile from the others'
    for tune in ({"tile_w": 8}, {"tile_w": 4, "banks": 3, "waves_per_cu": 8, "refill_below": 16},
                 {"tile_w": 32, "banks": 2, "waves_per_cu": 32, "refill_below": 64},
                 {"tile_w": 16, "banks": 3, "waves_per_cu": 1, "refill_below": 1},
                 {"stripe": 1}, {"stripe": 1024, "waves_per_cu": 2}):
        other = _gpu(tr, gs, c, p, "fp32_resolve", tune=tune)
        for k in OUT:
            assert np.array_equal(base[k], other[k]), (tune, k)
    for bad in (3, 2048, -4):
        with pytest.raises(tr.TRError) as e:
            _gpu(tr, gs, c, p, "fp32_resolve", tune={"stripe": bad})
        assert e.value.status == -1 and "stripe" in str(e.value), bad
    # grid density never changes the frame
    gs2 = tr.Scene(s, cells_per_prim=3.0)
    other = _gpu(tr, gs2, c, p, "fp32_resolve")
    for k in OUT:
        assert np.array_equal(base[k], other[k]), ("lambda", k)


def test_stats_counts(tr, oracle_mod, protein):
    # exact per-pixel counts, and traversal op counts against the oracle's
    # walk of the same grid (the FP64 path walks it identically; the FP32
    # walk may differ at cell boundaries and near-tangent rays)
    import torch
    s, _ = protein
    gs = tr.Scene(s, cells_per_prim=4.0)  # the oracle walks the same grid
    c = scenegen.Camera((0.0, 0.0, 120.0), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 50.0, 200, 150)
    p = scenegen.Params(ao_samples=16, seed=2)
    ref = oracle_mod.render(s, c, p, grid=4.0)["counters"]
    for prec, tune, tol in (("fp32_resolve", {"count_ops": 1}, 0.02), ("fp64", None, 1e-4)):
        fr = tr.render(gs, c, p, precision=prec, outputs=OUT, stats=True, tune=tune)
        torch.cuda.synchronize()
        st = dict(zip(tr.STAT_NAMES, fr["stats"].cpu().tolist()))
        hits = int((fr["hit_id"] >= 0).sum().item())
        assert st["pixels"] == 200 * 150
        assert st["stalls"] == 0
        assert st["hit_pixels"] == hits
        assert st["ao_rays"] == 16 * hits
        assert st["rays_traced"] == st["pixels"] + st["ao_rays"] + st["shadow_rays"]
        keys = ("rays_traced", "cells", "sph_tests", "cyl_tests", "shadow_rays")
        if prec != "fp64":
            # the FP32 walk jumps over runs of empty cells: fewer cells, same tests
            keys = ("rays_traced", "sph_tests", "cyl_tests", "shadow_rays")
            assert st["cells"] < ref["cells"] and st["jumps"] > 0
        for k in keys:
            assert abs(st[k] - ref[k]) <= tol * ref[k] + 2, (prec, k, st[k], ref[k])
        # hits: the FP32 walk counts the hits it decides itself; a re-solved
        # test is counted as a re-solve, not as a hit
        for k in ("sph_hits", "cyl_hits"):
            assert ref[k] > 0
            assert abs(st[k] - ref[k]) <= tol * ref[k] + st["resolves"] + 2, (prec, k, st[k], ref[k])
        if prec == "fp64":
            assert st["resolves"] == 0
        else:
            n_tests = st["sph_tests"] + st["cyl_tests"]
            print("re-solves", st["resolves"], "of", n_tests, "tests", {
                k: st[k] for k in ("resolves_sph", "resolves_cyl", "resolves_nearest")})
            assert st["resolves"] <= 1e-3 * n_tests, st
            assert st["resolves_sph"] + st["resolves_cyl"] + st["resolves_tri"] == st["resolves"]
            assert st["resolves_nearest"] <= st["resolves"]
        if prec != "fp64":
            assert st["lane_iters"] <= 64 * st["wave_iters"]
            # a lane-iteration makes at most one test and at most one step (the
            # two together when the test is its cell's last); only the first
            # cell of each ray is entered outside the loop.  (Lane-iterations
            # also count lanes waiting for their work type to run.)
            assert st["lane_iters"] >= st["sph_tests"] + st["cyl_tests"]
            assert st["lane_iters"] >= st["cells"] - st["rays_traced"]
            assert 2 * st["lane_iters"] >= (st["cells"] + st["sph_tests"] + st["cyl_tests"]
                                            - st["rays_traced"])


def _limb_scene():
    # The farthest points from the grid box's centre, which the FP32 walk's
    # bounding sphere passes through (up to its padding), are a cylinder's
    # far end (+y) and, within 0.2% of it, a sphere's outer limb (-y); the
    # rest sits near the centre.
    centers = np.array([[0.0, 0.0, 0.0], [0.5, -7.0, 0.0], [1.0, 1.0, 0.5]])
    radius = np.array([1.0, 2.0, 0.75])
    cyl_a = np.array([[0.0, 1.5, 0.0], [0.5, 0.0, -0.5]])
    cyl_b = np.array([[0.0, 8.0, 0.0], [1.0, 1.0, 0.5]])
    cyl_r = np.array([0.5, 0.3])
    rng = np.random.default_rng(7)
    ld = np.array([[-0.5, 0.5, 1.0], [1.0, 2.0, 0.5]])
    ld /= np.linalg.norm(ld, axis=1, keepdims=True)
    return scenegen.Scene(centers, radius, rng.uniform(0.3, 1.0, (3, 3)).astype(np.float32),
                          cyl_a, cyl_b, cyl_r, rng.uniform(0.3, 1.0, (2, 3)).astype(np.float32),
                          ld, np.ones((2, 3)))


@pytest.mark.parametrize("view", ["cylinder_end", "sphere_limb", "cylinder_rim"])
def test_bounding_sphere_limb(tr, oracle_mod, view):
    """Rays that graze the outermost surfaces of the scene, where the walk's
    clip to the bounding sphere is tightest, find the oracle's hits: both
    FP32 precisions against brute force at the usual bar.  The rim view
    also aims at a cylinder's rim, where the cylinder touches its own
    bounding sphere (the walk's first test of a cylinder): the pixels are
    0.0013 apart, finer than that sphere's padding (0.003 in radius)."""
    s = _limb_scene()
    if view == "cylinder_end":  # the far end's rim, seen from the side
        c = scenegen.Camera((0.0, 8.0, 14.0), (0.0, 8.0, 0.0), (0.0, 1.0, 0.0), 12.0, 96, 96)
    elif view == "cylinder_rim":  # one point of that rim, rays tangent to the bounding sphere
        c = scenegen.Camera((0.5, 8.0, 14.0), (0.5, 8.0, 0.0), (0.0, 1.0, 0.0), 0.5, 96, 96)
    else:  # the far sphere's outer limb, seen from the side
        c = scenegen.Camera((0.5, -8.5, 15.0), (0.5, -8.5, 0.0), (0.0, 1.0, 0.0), 12.0, 96, 96)
    p = scenegen.Params(ao_samples=8, seed=3)
    print("limb", view, flush=True)
    ref = _ref(oracle_mod, s, c, p, grid=None)
    hits = (ref["hit_id"] >= 0).sum()
    assert 0.1 * 96 * 96 < hits < 0.9 * 96 * 96  # the silhouette crosses the frame
    gs = tr.Scene(s)
    for prec in ("fp32", "fp32_resolve"):
        got = _gpu(tr, gs, c, p, prec)
        m = compare(got, ref, p.ao_samples, s.n_lights)
        print(prec, m, flush=True)
        assert_fp32_parity(m)
