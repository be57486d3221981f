"""The 1,000,000-object walk scene (ball radius 250): 64 camera views at
1920x1080 with 32 AO samples, captured once into a hipGraph and replayed;
sampled pixels of several views against the oracle, and FP64 on one view."""
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


def test_orbit_graph_parity(tr, oracle_mod):
    import torch
    print("generating the 1M-object scene", flush=True)
    scene = scenegen.orbit_scene()
    assert scene.n_prims == 1000000
    gs = tr.Scene(scene)
    cams = scenegen.orbit_cameras()
    params = scenegen.orbit_params()
    frames = [tr.alloc_frame(c, OUT) for c in cams]
    g = tr.Graph([gs] * len(cams), cams, params, frames)
    g.launch()
    torch.cuda.synchronize()
    print("graph launch done", flush=True)
    grid = oracle_mod.Grid(scene, 4.0)
    for v in (0, 17, 40):
        pix = scenegen.sample_pixels(cams[v].width, cams[v].height, 20000, 100 + v)
        ref = oracle_mod.render(scene, cams[v], params[v], grid=grid, pix=pix)
        m = compare(flat_at(frame_to_numpy(frames[v]), pix), ref, 32, scene.n_lights)
        print("view", v, m, flush=True)
        assert_fp32_parity(m)
        assert (ref["hit_id"] >= 0).mean() > 0.1  # sparse scene: ~20% of pixels hit
    # FP64 plain path on one view, same sample
    v = 17
    f64 = frame_to_numpy(tr.render(gs, cams[v], params[v], precision="fp64", outputs=OUT))
    torch.cuda.synchronize()
    pix = scenegen.sample_pixels(cams[v].width, cams[v].height, 20000, 100 + v)
    ref = oracle_mod.render(scene, cams[v], params[v], grid=grid, pix=pix)
    m = compare(flat_at(f64, pix), ref, 32, scene.n_lights)
    assert m["hit_mismatch"] == 0 and m["max_abs_agree"] <= 1.2e-7, m
    g.destroy()
