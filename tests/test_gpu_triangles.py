"""Triangles (the third primitive type) on the GPU against the oracle: the
grid build lists them exactly as the oracle's grid does; the plain FP64 path
reproduces the oracle; the FP32 wavefront path (triangle variant) meets the
FP32 bar on a scene of all three types, on a 26,560-triangle surface scene
of unrotated icosphere blobs (full small frame and sampled 17.6 MP pixels),
on an axis-aligned voxel surface and with transparent triangles; op counts;
scene files; graphs; argument errors."""
import os
import tempfile

import numpy as np
import pytest

import scenegen
from parity_util import assert_fp32_parity, compare, explain_flips, flat_at, frame_to_numpy

pytestmark = pytest.mark.gpu

OUT = ("rgb", "hit_id", "ao_mask", "light_mask")


@pytest.fixture(scope="module")
def tr():
    import paper_0801_1500_amd as tr
    tr.lib()
    return tr


@pytest.fixture(scope="module")
def surface(tr):
    s = scenegen.surface_scene()
    return s, tr.Scene(s)


def _gpu(tr, gscene, cam, params, precision, tune=None, stats=False):
    import torch
    fr = tr.render(gscene, cam, params, precision=precision, outputs=OUT, tune=tune, stats=stats)
    torch.cuda.synchronize()
    return frame_to_numpy(fr)


def _mixed_camera(w=128, h=112):
    return scenegen.Camera((0.0, 4.0, 30.0), (0.0, -2.0, 0.0), (0.0, 1.0, 0.0), 50.0, w, h)


def _surface_camera(res=(241, 284)):
    c = scenegen.protein_camera(scenegen.RES_1MP)
    return scenegen.Camera(c.eye, c.lookat, c.up, c.fovy_deg, res[0], res[1])


def _fp64_exact(m):
    assert m["hit_mismatch"] == 0, m
    assert m["decision_flips"] <= max(2, m["decisions"] // 1000000), m
    assert m["max_abs_agree"] <= 1.2e-7, m


@pytest.mark.parametrize("which,lam", [("mixed", 4.0), ("mixed", 24.0), ("surface", 24.0)])
def test_grid_matches_oracle(tr, oracle_mod, which, lam):
    s = scenegen.mixed_tiny_scene() if which == "mixed" else scenegen.surface_scene()
    print("triangle grid", which, lam, flush=True)
    cb, refs = tr.Scene(s, cells_per_prim=lam).grid_arrays()
    ocb, orefs = oracle_mod.Grid(s, cells_per_prim=lam).arrays()
    assert np.array_equal(cb, ocb)
    assert np.array_equal(refs, orefs)
    assert (refs >= s.n_spheres + s.n_cylinders).sum() > 0


def test_mixed_matches_oracle(tr, oracle_mod):
    s = scenegen.mixed_tiny_scene()
    c = _mixed_camera()
    p = scenegen.Params(ao_samples=8, seed=3)
    gs = tr.Scene(s)
    ref = oracle_mod.render(s, c, p, grid=None)
    assert (ref["hit_id"] >= s.n_spheres + s.n_cylinders).sum() > 1000
    ms = {}
    for prec in ("fp64", "fp32_resolve", "fp32"):
        print("mixed", prec, flush=True)
        ms[prec] = compare(_gpu(tr, gs, c, p, prec), ref, 8, s.n_lights)
        print(ms[prec])
    _fp64_exact(ms["fp64"])
    assert_fp32_parity(ms["fp32_resolve"])
    # FP32 alone (no FP64 re-solve) cannot decide the near-grazing tests this
    # scene is full of (open cylinders seen from inside, triangle edges):
    # the re-solve exists for them.  Hits and colours still meet the bar; the
    # decisions get ten times the budget.
    m = ms["fp32"]
    assert m["hit_agree"] >= 0.9999 and m["decision_agree"] >= 0.999, m
    assert m["max_abs_agree"] <= 1e-3 and m["rms_agree"] <= 1e-4, m


@pytest.mark.parametrize("prec", ["fp32_resolve", "fp64"])
def test_surface_small_matches_oracle(tr, oracle_mod, surface, prec):
    s, gs = surface
    c = _surface_camera()
    p = scenegen.Params(ao_samples=8, seed=2)
    print("surface 241x284", prec, flush=True)
    got = _gpu(tr, gs, c, p, prec)
    ref = oracle_mod.render(s, c, p, grid=4.0)
    m = compare(got, ref, 8, s.n_lights)
    print(m)
    assert (ref["hit_id"] >= 0).mean() > 0.2
    if prec == "fp64":
        _fp64_exact(m)
    else:
        # the FP32 bar; hits on an edge shared by two faces are re-solved in
        # FP64 for each face, but the two roots are kept as floats, which can
        # tie where the FP64 reference orders the faces by one ulp (then the
        # smaller id wins): 1 pixel of 68,444 on these blobs
        assert_fp32_parity(m)


def _degenerate_faces(s):
    """Faces whose FP64 unit normal has a z component, or a dot product
    with a light, within 1e-9 of zero: decisions that hold for the whole
    face and that FP32 rounding alone would take at random."""
    t = np.asarray(s.tri_v, dtype=np.float64)
    n = np.cross(t[:, 1] - t[:, 0], t[:, 2] - t[:, 0])
    n /= np.linalg.norm(n, axis=1)[:, None]
    ld = s.light_dir / np.linalg.norm(s.light_dir, axis=1)[:, None]
    return int((np.abs(n[:, 2]) <= 1e-9).sum()), int((np.abs(n @ ld.T) <= 1e-9).any(axis=1).sum())


@pytest.mark.parametrize("which", ["icosphere", "voxel"])
@pytest.mark.parametrize("prec", ["fp32_resolve", "fp64"])
def test_symmetric_surfaces_match_oracle(tr, oracle_mod, which, prec):
    """Blobs that keep the icosahedron's orientation, and voxel surfaces
    whose normals are the axis directions (with a light along +z, exactly
    perpendicular to the faces along x and y): whole faces whose facing,
    N.L > 0 or AO basis (the sign of N.z) rest on a zero.  The FP32 path
    takes those decisions from the FP64 vertices, so no rotation of the
    input is needed to meet the bar."""
    s = scenegen.surface_scene() if which == "icosphere" else scenegen.voxel_surface_scene()
    nz0, nl0 = _degenerate_faces(s)
    print(which, prec, "faces with N.z ~ 0:", nz0, "with N.L ~ 0:", nl0, flush=True)
    assert nz0 > 100
    if which == "voxel":
        assert nl0 > 100
    gs = tr.Scene(s)
    c = _surface_camera()
    p = scenegen.Params(ao_samples=8, seed=2)
    got = _gpu(tr, gs, c, p, prec)
    ref = oracle_mod.render(s, c, p, grid=4.0)
    m = compare(got, ref, 8, s.n_lights)
    print(m)
    for line in explain_flips(oracle_mod, s, c, got, ref):
        print(line, flush=True)
    assert (ref["hit_id"] >= 0).mean() > 0.04
    if prec != "fp64":
        st = _gpu(tr, gs, c, p, prec, tune={"count_ops": 1}, stats=True)["stats"]
        st = dict(zip(tr.STAT_NAMES, st.tolist()))
        print("signs decided in FP64:", st["signs_f64"], "of", st["hit_pixels"], "hit pixels",
              flush=True)
        assert st["signs_f64"] > 0
    if prec == "fp64":
        _fp64_exact(m)
    else:
        assert_fp32_parity(m)
    gs.destroy()


def test_surface_17mp_sampled(tr, oracle_mod, surface):
    s, gs = surface
    c = scenegen.protein_camera(scenegen.RES_17MP)
    p = scenegen.Params(ao_samples=16, seed=2)
    print("surface 17.6MP fp32_resolve", flush=True)
    got = _gpu(tr, gs, c, p, "fp32_resolve")
    pix = scenegen.sample_pixels(c.width, c.height, 20000, 37)
    ref = oracle_mod.render(s, c, p, grid=4.0, pix=pix)
    m = compare(flat_at(got, pix), ref, 16, s.n_lights)
    print(m)
    assert_fp32_parity(m)
    assert got["hit_id"].max() < s.n_prims


def test_transparent_triangles(tr, oracle_mod):
    s = scenegen.mixed_tiny_scene()
    op = np.full(s.n_triangles, 0.5, np.float32)
    op[-2:] = 1.0  # opaque floor
    st = scenegen.Scene(**{**s.__dict__, "tri_opacity": op})
    c = _mixed_camera()
    p = scenegen.Params(ao_samples=8, seed=3, max_layers=6)
    gst = tr.Scene(st)
    ref = oracle_mod.render(st, c, p, grid=None)
    for prec in ("fp64", "fp32_resolve"):
        print("glass triangles", prec, flush=True)
        got = _gpu(tr, gst, c, p, prec)
        m = compare(got, ref, 8, s.n_lights)
        print(m)
        if prec == "fp64":
            assert m["hit_mismatch"] == 0 and m["decision_flips"] <= 2, m
            err = np.abs(got["rgb"].astype(np.float64) - ref["rgb"]).max(axis=-1)
            assert float((err > 4e-7).mean()) <= 1e-3
        else:
            assert m["hit_agree"] >= 0.9999 and m["decision_agree"] >= 0.9999, m
            err = np.abs(got["rgb"].astype(np.float64) - ref["rgb"]).max(axis=-1)
            assert float((err > 1e-3).mean()) <= 10 * 6 * (1 + 8 + 1) * 1e-5


def test_op_counts(tr, oracle_mod, surface):
    s, _ = surface
    gs = tr.Scene(s, cells_per_prim=4.0)  # the oracle walks the same grid
    c = _surface_camera((200, 150))
    p = scenegen.Params(ao_samples=8, seed=2)
    ref = oracle_mod.render(s, c, p, grid=4.0)["counters"]
    assert ref["tri_tests"] > 0
    for prec, tune, tol in (("fp32_resolve", {"count_ops": 1}, 0.02), ("fp64", None, 1e-4)):
        fr = _gpu(tr, gs, c, p, prec, tune=tune, stats=True)
        st = dict(zip(tr.STAT_NAMES, fr["stats"].tolist()))
        for k in ("rays_traced", "tri_tests", "shadow_rays"):
            assert abs(st[k] - ref[k]) <= tol * ref[k] + 2, (prec, k, st[k], ref[k])


def test_scene_file_and_graph(tr):
    import torch
    s = scenegen.mixed_tiny_scene()
    op = np.full(s.n_triangles, 0.7, np.float32)
    st = scenegen.Scene(**{**s.__dict__, "tri_opacity": op})
    c = _mixed_camera()
    p = scenegen.Params(ao_samples=8, seed=3, max_layers=4)
    gst = tr.Scene(st)
    a = _gpu(tr, gst, c, p, "fp32_resolve")
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "mixed.trs")
        gst.save(path)
        loaded = tr.Scene.load(path)
        assert loaded.n_triangles == s.n_triangles
        b = _gpu(tr, loaded, c, p, "fp32_resolve")
    for k in OUT:
        assert np.array_equal(a[k], b[k]), k
    # a graph over a triangle scene (opaque rendering) equals the direct render
    gs = tr.Scene(s)
    q = scenegen.Params(ao_samples=8, seed=3)
    direct = _gpu(tr, gs, c, q, "fp32_resolve")
    fr = tr.alloc_frame(c, OUT, False)
    g = tr.Graph([gs], [c], [q], [fr])
    g.launch()
    torch.cuda.synchronize()
    g.destroy()
    f = frame_to_numpy(fr)
    for k in OUT:
        assert np.array_equal(direct[k], f[k]), k


def test_errors(tr):
    s = scenegen.mixed_tiny_scene()
    tv = np.array(s.tri_v, copy=True)
    tv[5, 1, 2] = np.inf
    with pytest.raises(tr.TRError) as e:
        tr.Scene(scenegen.Scene(**{**s.__dict__, "tri_v": tv}))
    assert e.value.status == -1
