"""Batched renders (one persistent launch over many frames), tile-range
renders, and hipGraph replay: every frame identical, bit for bit, to the same
frame rendered alone."""
import numpy as np
import pytest

import scenegen
from parity_util import frame_to_numpy

pytestmark = pytest.mark.gpu

OUT = ("rgb", "hit_id", "ao_mask", "light_mask")


@pytest.fixture(scope="module")
def tr():
    import paper_0801_1500_amd as tr
    tr.lib()
    return tr


@pytest.fixture(scope="module")
def scenes(tr):
    a = scenegen.protein_scene()
    b = scenegen.random_walk_scene(3000, scenegen.serving_radius(6000), 101)
    return [tr.Scene(a), tr.Scene(b)]


def _jobs():
    cams = [scenegen.Camera((0.0, 0.0, 120.0), (0, 0, 0), (0, 1, 0), 50.0, 211, 173),
            scenegen.Camera((60.0, 10.0, 10.0), (0, 0, 0), (0, 1, 0), 50.0, 96, 200),
            scenegen.Camera((0.0, 0.0, 120.0), (0, 0, 0), (0, 1, 0), 40.0, 64, 64),
            scenegen.Camera((-40.0, 20.0, 80.0), (0, 0, 0), (0, 1, 0), 50.0, 150, 90)]
    params = [scenegen.Params(ao_samples=16, seed=2), scenegen.Params(ao_samples=7, seed=3),
              scenegen.Params(ao_samples=32, seed=4, view_id=3),
              scenegen.Params(ao_samples=4, seed=5, ao_maxdist=6.0)]
    which = [0, 1, 0, 1]
    return cams, params, which


def _alone(tr, scenes, cams, params, which):
    import torch
    out = []
    for c, p, w in zip(cams, params, which):
        out.append(frame_to_numpy(tr.render(scenes[w], c, p, outputs=OUT)))
    torch.cuda.synchronize()
    return out


def _same(a, b, tag):
    for k in OUT:
        assert np.array_equal(a[k], b[k]), (tag, k)


def test_batch_equals_alone(tr, scenes):
    import torch
    cams, params, which = _jobs()
    alone = _alone(tr, scenes, cams, params, which)
    frames = [tr.alloc_frame(c, OUT) for c in cams]
    tr.render_batch_into([scenes[w] for w in which], cams, params, frames)
    torch.cuda.synchronize()
    for i, f in enumerate(frames):
        _same(frame_to_numpy(f), alone[i], i)


def test_tile_ranges_compose(tr, scenes):
    import torch
    cams, params, which = _jobs()
    alone = _alone(tr, scenes, cams, params, which)
    frames = [tr.alloc_frame(c, OUT) for c in cams]
    for f in frames:
        f["rgb"].fill_(-1.0)
    ntiles = [tr.tile_count(c.width, c.height) for c in cams]
    # advance every job in steps of at most 37 tiles, several launches
    pos = [0] * len(cams)
    steps = 0
    while any(p < n for p, n in zip(pos, ntiles)):
        tb = list(pos)
        te = [min(p + 37, n) for p, n in zip(pos, ntiles)]
        tr.render_batch_tiles_into([scenes[w] for w in which], cams, params, frames, tb, te)
        pos = te
        steps += 1
    torch.cuda.synchronize()
    assert steps > 3
    for i, f in enumerate(frames):
        _same(frame_to_numpy(f), alone[i], i)


def test_graph_replay_and_update(tr, scenes):
    import torch
    sc = scenes[0]
    base_cams = scenegen.orbit_cameras(6, dist=130.0, res=(160, 120))
    params = [scenegen.Params(ao_samples=8, seed=4, view_id=k) for k in range(6)]
    frames = [tr.alloc_frame(c, OUT) for c in base_cams]
    g = tr.Graph([sc] * 6, base_cams, params, frames)
    alone = _alone(tr, [sc], base_cams, params, [0] * 6)
    for rep in range(3):
        for f in frames:
            f["rgb"].zero_()
        g.launch()
        torch.cuda.synchronize()
        for i, f in enumerate(frames):
            _same(frame_to_numpy(f), alone[i], (rep, i))
    # new cameras through the device job table, no re-capture
    cams2 = scenegen.orbit_cameras(6, dist=110.0, res=(160, 120))
    cams2 = cams2[3:] + cams2[:3]
    g.update(cams=cams2)
    alone2 = _alone(tr, [sc], cams2, params, [0] * 6)
    for rep in range(2):
        g.launch()
        torch.cuda.synchronize()
        for i, f in enumerate(frames):
            _same(frame_to_numpy(f), alone2[i], ("upd", rep, i))
    g.destroy()


def test_autotune_choice_is_bit_identical(tr, scenes):
    sc = scenes[1]
    c = scenegen.Camera((0.0, 0.0, 70.0), (0, 0, 0), (0, 1, 0), 50.0, 256, 256)
    p = scenegen.Params(ao_samples=8, seed=3)
    best, ms = tr.autotune(sc, c, p)
    assert ms > 0 and best["tile_w"] in (4, 8, 16, 32, 64)


def test_graph_autotune_keeps_frames(tr):
    # the graph is tuned on itself (grid density, then launch shape): every
    # candidate must leave the frames bit-identical, and the re-captured graph
    # renders the same frames as each job alone
    import torch
    walk = scenegen.random_walk_scene(3000, scenegen.serving_radius(6000), 101)
    prot = scenegen.protein_scene()
    a, b = tr.Scene(walk), tr.Scene(prot)
    cams = scenegen.orbit_cameras(4, dist=90.0, res=(160, 96))
    params = [scenegen.Params(ao_samples=8, seed=6, view_id=k) for k in range(4)]
    which = [a, b, a, b]
    alone = [frame_to_numpy(tr.render(s, c, p, outputs=OUT)) for s, c, p in zip(which, cams, params)]
    torch.cuda.synchronize()
    frames = [tr.alloc_frame(c, OUT) for c in cams]
    g = tr.Graph(which, cams, params, frames)
    tune, lam, ms = g.autotune(lambdas=(6.0, 24.0, 48.0))
    print("graph tune", tune, lam, ms, flush=True)
    assert ms > 0 and lam in (0.0, 6.0, 24.0, 48.0)
    assert tune["tile_w"] in (8, 16, 64) and tune["banks"] in (2, 3)
    assert tune["stripe"] in (16, 32, 64, 128, 256)
    if lam > 0:  # the scenes were left at the chosen density
        for s, src in ((a, walk), (b, prot)):
            assert np.array_equal(s.grid_info()[2], tr.Scene(src, cells_per_prim=lam).grid_info()[2])
    for f in frames:
        f["rgb"].zero_()
    g.launch()
    torch.cuda.synchronize()
    for i, f in enumerate(frames):
        _same(frame_to_numpy(f), alone[i], ("tuned graph", i))
    for bad in ((0.0,), (float("nan"),), (-3.0,)):
        with pytest.raises(tr.TRError) as e:
            g.autotune(lambdas=bad)
        assert e.value.status == -1
    g.destroy()
    # a BVH-walk graph: the grid rebuilds of the density search leave the
    # BVH valid, and the tuned graph still renders the frames of the walk
    a.build_bvh()
    b.build_bvh()
    alone = [frame_to_numpy(tr.render(s, c, p, outputs=OUT, tune={"accel": 1}))
             for s, c, p in zip(which, cams, params)]
    torch.cuda.synchronize()
    g = tr.Graph(which, cams, params, frames, tune={"accel": 1})
    tune, lam, ms = g.autotune(lambdas=(6.0,))
    assert tune["accel"] == 1 and ms > 0
    for f in frames:
        f["rgb"].zero_()
    g.launch()
    torch.cuda.synchronize()
    for i, f in enumerate(frames):
        _same(frame_to_numpy(f), alone[i], ("tuned bvh graph", i))
    g.destroy()


def test_measured_fp32_peak(tr):
    # non-packed FP32 FMAs: at most 128 flops per compute unit per clock
    m = tr.measure_fp32_peak()
    print("fp32 peak", m, flush=True)
    assert m["n_cus"] > 0 and m["clock_mhz"] > 0
    derived = m["n_cus"] * m["clock_mhz"] * 1e6 * 128 / 1e12
    assert 0.3 * derived < m["tflops"] <= 1.05 * derived, (m, derived)


def test_failing_batch_renders_nothing(tr, scenes):
    # every job is checked before anything is enqueued: an FP64 job ahead of
    # an invalid one is not rendered either
    import torch
    cams, params, which = _jobs()
    bad = scenegen.Camera(cams[1].eye, cams[1].lookat, cams[1].up, 0.0, 96, 200)  # fovy 0
    p64 = scenegen.Params(**{**params[0].__dict__})
    frames = [tr.alloc_frame(c, OUT) for c in (cams[0], bad)]
    for f in frames:
        f["rgb"].fill_(-7.0)
    with pytest.raises(tr.TRError) as e:
        tr.render_batch_into([scenes[0], scenes[1]], [cams[0], bad], [p64, params[1]], frames,
                             precision="fp64")
    assert e.value.status == -1
    torch.cuda.synchronize()
    assert bool((frames[0]["rgb"] == -7.0).all())


def test_graph_bvh_cross_stream_and_refresh(tr, scenes):
    import torch
    sc = tr.Scene(scenegen.random_walk_scene(3000, scenegen.serving_radius(6000), 101))
    sc.build_bvh()
    cams = scenegen.orbit_cameras(4, dist=60.0, res=(128, 96))
    params = [scenegen.Params(ao_samples=8, seed=6, view_id=k) for k in range(4)]
    frames = [tr.alloc_frame(c, OUT) for c in cams]
    # the BVH walk in a graph equals the BVH walk rendered alone
    g = tr.Graph([sc] * 4, cams, params, frames, tune={"accel": 1})
    alone = []
    for c, p in zip(cams, params):
        alone.append(frame_to_numpy(tr.render(sc, c, p, outputs=OUT, tune={"accel": 1})))
    torch.cuda.synchronize()
    g.launch()
    torch.cuda.synchronize()
    for i, f in enumerate(frames):
        _same(frame_to_numpy(f), alone[i], ("bvh", i))
    # update on one stream, replay on another: the replay sees the new table
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    cams2 = cams[2:] + cams[:2]
    alone2 = []
    for c, p in zip(cams2, params):
        alone2.append(frame_to_numpy(tr.render(sc, c, p, outputs=OUT, tune={"accel": 1})))
    torch.cuda.synchronize()
    g.update(cams=cams2, stream=s1)
    g.launch(stream=s2)
    torch.cuda.synchronize()
    for i, f in enumerate(frames):
        _same(frame_to_numpy(f), alone2[i], ("streams", i))
    # rebuilding the scene's grid and BVH, then re-reading the scenes (update
    # with no arguments), gives the same frames
    sc.rebuild(cells_per_prim=6.0)
    sc.build_bvh()
    g.update()
    for f in frames:
        f["rgb"].zero_()
    g.launch()
    torch.cuda.synchronize()
    for i, f in enumerate(frames):
        _same(frame_to_numpy(f), alone2[i], ("refresh", i))
    g.destroy()
    # a graph asking for the BVH walk of a scene without one is refused
    plain = tr.Scene(scenegen.tiny_scene(seed=1))
    c = scenegen.Camera((0.0, 0.0, 30.0), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 50.0, 32, 32)
    with pytest.raises(tr.TRError) as e:
        tr.Graph([plain], [c], [scenegen.Params(ao_samples=4)], [tr.alloc_frame(c, OUT)],
                 tune={"accel": 1})
    assert e.value.status == -1


def test_mixed_precision_batch(tr, scenes):
    # plain FP64 jobs (one launch each) and FP32 jobs (one wavefront launch)
    # in one batch call, antialiased jobs among them: each frame equals the
    # same job rendered alone
    import torch
    cams, params, which = _jobs()
    params = list(params)
    params[2] = scenegen.Params(**{**params[2].__dict__, "aa_samples": 3})
    params[3] = scenegen.Params(**{**params[3].__dict__, "aa_samples": 2})
    prec = ["fp64", "fp32_resolve", "fp64", "fp32_resolve"]
    frames = [tr.alloc_frame(c, OUT) for c in cams]
    print("mixed precision batch", flush=True)
    tr.render_batch_into([scenes[w] for w in which], cams, params, frames, precision=prec)
    torch.cuda.synchronize()
    for i, (c, p, w) in enumerate(zip(cams, params, which)):
        alone = frame_to_numpy(tr.render(scenes[w], c, p, precision=prec[i], outputs=OUT))
        torch.cuda.synchronize()
        _same(frame_to_numpy(frames[i]), alone, ("mixed", i))
