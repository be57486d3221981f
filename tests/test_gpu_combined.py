"""All options at once on a scene of all three primitive types: two
antialiasing samples, transparency (spheres and blob triangles at opacity
0.6, up to five surfaces), a Phong highlight and a background colour.  The
plain FP64 path reproduces the oracle; the FP32 path meets the FP32 bar on
the first surface with a budget for flipped decisions deeper down or in the
second sample; a batch mixing it with an opaque frame is bitwise the same."""
import numpy as np
import pytest

import scenegen
from parity_util import DECISION_AGREE_MIN, HIT_AGREE_MIN, compare, frame_to_numpy

pytestmark = pytest.mark.gpu

OUT = ("rgb", "hit_id", "ao_mask", "light_mask")


@pytest.fixture(scope="module")
def tr():
    import paper_0801_1500_amd as tr
    tr.lib()
    return tr


def _setup():
    s = scenegen.mixed_tiny_scene()
    top = np.full(s.n_triangles, 0.6, np.float32)
    top[-2:] = 1.0  # the floor stays opaque
    st = scenegen.Scene(**{**s.__dict__, "sph_opacity": np.full(s.n_spheres, 0.6, np.float32),
                           "tri_opacity": top})
    c = scenegen.Camera((0.0, 4.0, 30.0), (0.0, -2.0, 0.0), (0.0, 1.0, 0.0), 50.0, 96, 84)
    p = scenegen.Params(ao_samples=8, seed=3, aa_samples=2, max_layers=5, specular=0.3,
                        shininess=20.0, background=(0.1, 0.15, 0.2))
    return st, c, p


def _gpu(tr, gs, c, p, prec):
    import torch
    fr = tr.render(gs, c, p, precision=prec, outputs=OUT)
    torch.cuda.synchronize()
    return frame_to_numpy(fr)


def test_all_options_match_oracle(tr, oracle_mod):
    st, c, p = _setup()
    gs = tr.Scene(st)
    ref = oracle_mod.render(st, c, p, grid=None)
    g64 = _gpu(tr, gs, c, p, "fp64")
    m = compare(g64, ref, 8, st.n_lights)
    print("fp64", m)
    assert m["hit_mismatch"] == 0 and m["decision_flips"] <= 2, m
    err = np.abs(g64["rgb"].astype(np.float64) - ref["rgb"]).max(axis=-1)
    assert float((err > 4e-7).mean()) <= 2e-3, float(err.max())
    g32 = _gpu(tr, gs, c, p, "fp32_resolve")
    m = compare(g32, ref, 8, st.n_lights)
    print("fp32_resolve", m)
    assert m["hit_agree"] >= HIT_AGREE_MIN and m["decision_agree"] >= DECISION_AGREE_MIN, m
    err = np.abs(g32["rgb"].astype(np.float64) - ref["rgb"]).max(axis=-1)
    # 2 samples x up to 5 surfaces x (1 + 8 AO + 1 light) decisions at ~1e-5
    assert float((err > 1e-3).mean()) <= 10 * 2 * 5 * 10 * 1e-5, float((err > 1e-3).mean())


def test_batched_with_opaque_frame(tr):
    import torch
    st, c, p = _setup()
    gs = tr.Scene(st)
    plain = scenegen.Params(ao_samples=4, seed=9)
    alone = [_gpu(tr, gs, c, p, "fp32_resolve"), _gpu(tr, gs, c, plain, "fp32_resolve")]
    frames = [tr.alloc_frame(c, OUT, False) for _ in range(2)]
    tr.render_batch_into([gs, gs], [c, c], [p, plain], frames, precision="fp32_resolve")
    torch.cuda.synchronize()
    for a, f in zip(alone, frames):
        f = frame_to_numpy(f)
        for k in OUT:
            assert np.array_equal(a[k], f[k]), k
