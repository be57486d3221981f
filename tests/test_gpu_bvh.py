"""The BVH walk (tune accel=1), the alternative acceleration structure: the
linear BVH built on the GPU is a valid tree over every primitive (checked on
the host: each node and primitive reached once, every box holding what is
below it); renders through it meet the FP32 bar against the oracle, match the
grid walk, and never overflow the traversal stack; argument errors."""
import numpy as np
import pytest

import scenegen
from parity_util import assert_fp32_parity, compare, frame_to_numpy

pytestmark = pytest.mark.gpu

OUT = ("rgb", "hit_id", "ao_mask", "light_mask")


@pytest.fixture(scope="module")
def tr():
    import paper_0801_1500_amd as tr
    tr.lib()
    return tr


def _prim_boxes(s):
    c, r = np.asarray(s.sph_center, np.float64).reshape(-1, 3), np.asarray(s.sph_radius, np.float64)
    boxes = [np.concatenate([c - r[:, None], c + r[:, None]], axis=1)]
    a, b = np.asarray(s.cyl_a, np.float64).reshape(-1, 3), np.asarray(s.cyl_b, np.float64).reshape(-1, 3)
    rho = np.asarray(s.cyl_radius, np.float64)[:, None]
    boxes.append(np.concatenate([np.minimum(a, b) - rho, np.maximum(a, b) + rho], axis=1))
    if s.n_triangles:
        tv = np.asarray(s.tri_v, np.float64).reshape(-1, 3, 3)
        boxes.append(np.concatenate([tv.min(axis=1), tv.max(axis=1)], axis=1))
    return np.concatenate(boxes)


def check_bvh(gs, s):
    nodes = gs.bvh_nodes()
    n = s.n_prims
    assert nodes.shape == (n - 1, 16)
    kids = nodes[:, 12:14].copy().view(np.int32)
    internal = kids[kids >= 0]
    leaves = -kids[kids < 0] - 1
    # every internal node but the root is a child exactly once; every
    # primitive is a leaf exactly once
    assert np.array_equal(np.sort(internal), np.arange(1, n - 1))
    assert np.array_equal(np.sort(leaves), np.arange(n))
    lo, hi, _, _ = gs.grid_info()
    org = 0.5 * (lo + hi)
    pb = _prim_boxes(s) - np.concatenate([org, org])
    box = [nodes[:, 0:6].astype(np.float64), nodes[:, 6:12].astype(np.float64)]
    for side in (0, 1):
        k = kids[:, side]
        b = box[side]
        leaf = k < 0
        # a leaf box holds its primitive's box
        p = pb[-k[leaf] - 1]
        assert np.all(b[leaf, :3] <= p[:, :3]) and np.all(b[leaf, 3:] >= p[:, 3:])
        # an internal child's box holds both of its own child boxes
        c = k[~leaf]
        for sub in (0, 1):
            inner = box[sub][c]
            assert np.all(b[~leaf, :3] <= inner[:, :3]) and np.all(b[~leaf, 3:] >= inner[:, 3:])
    # the depth the build reports (internal nodes on the longest root-to-leaf
    # path, which bounds the walk's stack) is the tree's, found top-down here
    depth = np.zeros(n - 1, np.int64)
    depth[0] = 1
    order = [0]
    for i in order:
        for c in kids[i]:
            if c >= 0:
                depth[c] = depth[i] + 1
                order.append(int(c))
    assert gs.bvh_depth() == int(depth.max())
    assert gs.bvh_depth() <= 48
    return nodes


def _duplicates_scene():
    # 3 x 1000 spheres on three points (equal Morton codes, split by their
    # sorted position) plus 200 spread ones
    rng = np.random.default_rng(12)
    pts = np.repeat(np.array([[0.0, 0.0, 0.0], [4.0, 1.0, -2.0], [-3.0, 2.5, 1.0]]), 1000, axis=0)
    c = np.concatenate([pts, rng.uniform(-12.0, 12.0, (200, 3))])
    r = np.concatenate([np.full(3000, 1.0), rng.uniform(0.4, 1.2, 200)])
    z3 = np.zeros((0, 3))
    ld = np.array([[0.3, 0.4, 1.0]])
    return scenegen.Scene(c, r, np.full((len(r), 3), 0.6, np.float32), z3, z3.copy(), np.zeros(0),
                          np.zeros((0, 3), np.float32), ld, np.ones_like(ld))


@pytest.mark.parametrize("which", ["tiny", "protein", "mixed", "duplicates"])
def test_bvh_structure(tr, which):
    s = {"tiny": lambda: scenegen.tiny_scene(seed=1), "protein": scenegen.protein_scene,
         "mixed": scenegen.mixed_tiny_scene, "duplicates": _duplicates_scene}[which]()
    print("bvh structure", which, flush=True)
    gs = tr.Scene(s)
    gs.build_bvh()
    check_bvh(gs, s)


def _render(tr, gs, c, p, accel, prec="fp32_resolve"):
    import torch
    fr = tr.render(gs, c, p, precision=prec, outputs=OUT, stats=True,
                   tune={"accel": accel, "count_ops": 1})
    torch.cuda.synchronize()
    return frame_to_numpy(fr)


@pytest.mark.parametrize("which", ["protein", "mixed"])
def test_bvh_walk_matches_oracle_and_grid(tr, oracle_mod, which):
    if which == "protein":
        s = scenegen.protein_scene()
        c0 = scenegen.protein_camera(scenegen.RES_1MP)
        c = scenegen.Camera(c0.eye, c0.lookat, c0.up, c0.fovy_deg, 241, 284)
    else:
        s = scenegen.mixed_tiny_scene()
        c = scenegen.Camera((0.0, 4.0, 30.0), (0.0, -2.0, 0.0), (0.0, 1.0, 0.0), 50.0, 128, 112)
    p = scenegen.Params(ao_samples=8, seed=2)
    gs = tr.Scene(s)
    gs.build_bvh()
    print("bvh walk", which, flush=True)
    got = _render(tr, gs, c, p, 1)
    st = dict(zip(tr.STAT_NAMES, got["stats"].tolist()))
    assert st["stack_overflows"] == 0 and st["stalls"] == 0
    ref = oracle_mod.render(s, c, p, grid=4.0)
    m = compare(got, ref, 8, s.n_lights)
    print(m)
    assert_fp32_parity(m)
    grid = _render(tr, gs, c, p, 0)
    same = (grid["hit_id"] == got["hit_id"]) & (grid["ao_mask"] == got["ao_mask"]) & \
           (grid["light_mask"] == got["light_mask"])
    assert same.mean() >= 0.9999
    # the same primitive tests give the same colours
    assert np.array_equal(grid["rgb"][same], got["rgb"][same])


def test_errors(tr):
    s = scenegen.tiny_scene(seed=1)
    gs = tr.Scene(s)
    c = scenegen.Camera((0.0, 0.0, 30.0), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 50.0, 32, 32)
    with pytest.raises(tr.TRError) as e:
        tr.render(gs, c, scenegen.Params(ao_samples=4), tune={"accel": 1})
    assert e.value.status == -1
    gs.build_bvh()
    st = scenegen.Scene(**{**s.__dict__, "sph_opacity": np.full(s.n_spheres, 0.5, np.float32)})
    gt = tr.Scene(st)
    gt.build_bvh()
    with pytest.raises(tr.TRError) as e:
        tr.render(gt, c, scenegen.Params(ao_samples=4, max_layers=3), tune={"accel": 1})
    assert e.value.status == -4
    with pytest.raises(tr.TRError) as e:
        tr.render(gs, c, scenegen.Params(ao_samples=4), tune={"accel": 2})
    assert e.value.status == -1


def _spheres(centres, radii):
    c = np.array(centres, dtype=np.float64).reshape(-1, 3)
    z3 = np.zeros((0, 3))
    ld = np.array([[0.3, 0.4, 1.0]])
    return scenegen.Scene(c, np.array(radii, dtype=np.float64),
                          np.full((len(radii), 3), 0.6, np.float32), z3, z3.copy(), np.zeros(0),
                          np.zeros((0, 3), np.float32), ld, np.ones_like(ld))


@pytest.mark.parametrize("n", [1, 2])
def test_bvh_one_and_two_primitives(tr, oracle_mod, n):
    # one primitive: no internal node, the walk tests it directly; two: the
    # root alone
    s = _spheres([[0.0, 0.0, 0.0], [2.5, 1.0, -3.0]][:n], [2.0, 1.5][:n])
    gs = tr.Scene(s)
    gs.build_bvh()
    assert gs.bvh_nodes().shape == (n - 1, 16)
    assert gs.bvh_depth() == n - 1
    c = scenegen.Camera((0.0, 0.0, 30.0), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 20.0, 64, 48)
    p = scenegen.Params(ao_samples=8, seed=4)
    print("bvh tiny", n, flush=True)
    got = _render(tr, gs, c, p, 1)
    ref = oracle_mod.render(s, c, p, grid=None)
    assert (ref["hit_id"] >= 0).sum() > 200
    assert_fp32_parity(compare(got, ref, 8, s.n_lights))
    grid = _render(tr, gs, c, p, 0)
    for k in OUT:
        assert np.array_equal(grid[k], got[k]), k


def test_bvh_duplicates_walk_equals_grid(tr):
    # equal codes and equal spheres: the BVH walk finds the same nearest hits
    # (ties to the lowest id) and occlusions as the grid walk
    s = _duplicates_scene()
    gs = tr.Scene(s)
    gs.build_bvh()
    assert 10 <= gs.bvh_depth() <= 48
    c = scenegen.Camera((0.0, 5.0, 40.0), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 45.0, 96, 80)
    p = scenegen.Params(ao_samples=8, seed=3)
    print("bvh duplicates", flush=True)
    got = _render(tr, gs, c, p, 1)
    grid = _render(tr, gs, c, p, 0)
    assert (grid["hit_id"] >= 0).sum() > 500
    for k in OUT:
        assert np.array_equal(grid[k], got[k]), k


def test_bvh_walk_with_options_and_batches(tr):
    # the BVH walk under antialiasing and the highlight agrees with the grid
    # walk; a batched tile-range launch of BVH frames equals each frame alone
    import torch
    s = scenegen.protein_scene()
    gs = tr.Scene(s)
    gs.build_bvh()
    c0 = scenegen.protein_camera(scenegen.RES_1MP)
    c = scenegen.Camera(c0.eye, c0.lookat, c0.up, c0.fovy_deg, 160, 190)
    p = scenegen.Params(ao_samples=8, seed=7, aa_samples=2, specular=0.5, shininess=16.0)
    print("bvh aa + highlight", flush=True)
    got = _render(tr, gs, c, p, 1)
    grid = _render(tr, gs, c, p, 0)
    same = (grid["hit_id"] == got["hit_id"]) & (grid["ao_mask"] == got["ao_mask"]) & \
           (grid["light_mask"] == got["light_mask"])
    assert same.mean() >= 0.9999
    err = np.abs(grid["rgb"].astype(np.float64) - got["rgb"]).max(axis=-1)
    assert float((err > 1e-6).mean()) <= 1e-3  # a sub-sample near-tie moves a pixel by <= 1/2
    cams = scenegen.orbit_cameras(3, dist=120.0, res=(96, 80))
    ps = [scenegen.Params(ao_samples=4, seed=9, view_id=k) for k in range(3)]
    frames = [tr.alloc_frame(cm, OUT) for cm in cams]
    print("bvh batch tiles", flush=True)
    tr.render_batch_tiles_into([gs] * 3, cams, ps, frames, [0] * 3,
                               [tr.tile_count(cm.width, cm.height, 8) for cm in cams],
                               tune={"accel": 1, "tile_w": 8})
    torch.cuda.synchronize()
    for cm, pp, fr in zip(cams, ps, frames):
        alone = frame_to_numpy(tr.render(gs, cm, pp, outputs=OUT, tune={"accel": 1}))
        torch.cuda.synchronize()
        f = frame_to_numpy(fr)
        for k in OUT:
            assert np.array_equal(f[k], alone[k]), k
