"""The largest frame the boundary accepts: 46340 x 46340 = 2,147,395,600
pixels, just under the W*H < 2^31 - 1 limit (25.8 GB of RGB).  Both GPU
paths render it in one launch; sampled pixels (the first, the last, and a
seeded spread) meet the FP32 and FP64 bars against the oracle; every pixel is
counted; the 8-bit output of the whole frame matches its definition on the
samples.  A frame past the limit is rejected before any launch."""
import numpy as np
import pytest

import scenegen
from parity_util import assert_fp32_parity, compare

pytestmark = pytest.mark.gpu

OUT = ("rgb", "hit_id", "ao_mask", "light_mask")
SIDE = 46340


@pytest.fixture(scope="module")
def tr():
    import paper_0801_1500_amd as tr
    tr.lib()
    return tr


def _gather(torch, fr, idx):
    return {"rgb": fr["rgb"].view(-1, 3)[idx].cpu().numpy(),
            "hit_id": fr["hit_id"].view(-1)[idx].cpu().numpy(),
            "ao_mask": fr["ao_mask"].view(-1)[idx].cpu().numpy().view(np.uint32),
            "light_mask": fr["light_mask"].view(-1)[idx].cpu().numpy()}


def test_largest_frame(tr, oracle_mod):
    import torch
    s = scenegen.protein_scene()
    gs = tr.Scene(s)
    c0 = scenegen.protein_camera(scenegen.RES_1MP)
    c = scenegen.Camera(c0.eye, c0.lookat, c0.up, c0.fovy_deg, SIDE, SIDE)
    n = SIDE * SIDE
    assert n < 2 ** 31 - 1
    p = scenegen.Params(ao_samples=4, seed=11)
    pix = np.unique(np.concatenate([[0, n - 1], scenegen.sample_pixels(SIDE, SIDE, 20000, 23)]))
    ref = oracle_mod.render(s, c, p, grid=4.0, pix=pix)
    assert (ref["hit_id"] >= 0).mean() > 0.1
    idx = torch.from_numpy(pix).cuda()
    fr = tr.alloc_frame(c, OUT, stats=True)
    for prec in ("fp32_resolve", "fp64"):
        print("largest frame", SIDE, "x", SIDE, prec, flush=True)
        fr["stats"].zero_()
        tr.render_into(gs, c, p, fr, prec)
        torch.cuda.synchronize()
        st = dict(zip(tr.STAT_NAMES, fr["stats"].cpu().tolist()))
        assert st["pixels"] == n and st["stalls"] == 0, st
        m = compare(_gather(torch, fr, idx), ref, 4, s.n_lights)
        print(m, flush=True)
        if prec == "fp64":
            assert m["hit_mismatch"] == 0, m
            assert m["decision_flips"] <= max(2, m["decisions"] // 1000000), m
            assert m["max_abs_agree"] <= 1.2e-7, m
        else:
            assert_fp32_parity(m)
    # 8-bit output of the whole frame (6.4 G values): floor(clamp(v) * 255 + 1/2)
    q = tr.quantize_rgb8(fr["rgb"])
    torch.cuda.synchronize()
    v = fr["rgb"].view(-1, 3)[idx].cpu().numpy().astype(np.float64)
    want = np.floor(np.clip(v, 0.0, 1.0) * 255.0 + 0.5).astype(np.uint8)
    assert np.array_equal(q.view(-1, 3)[idx].cpu().numpy(), want)
    del fr, q
    torch.cuda.empty_cache()
    # one more row and column put W*H past the limit
    assert (SIDE + 1) ** 2 > 2 ** 31 - 2
    big = scenegen.Camera(c0.eye, c0.lookat, c0.up, c0.fovy_deg, SIDE + 1, SIDE + 1)
    small = {"rgb": torch.empty(3, device="cuda")}
    # the binding refuses the buffer for that frame; the library refuses the
    # frame size itself, before looking at any buffer
    with pytest.raises(ValueError):
        tr.render_into(gs, big, p, small, "fp32_resolve")
    import ctypes as C
    st = tr.lib().tr_render(gs.handle, C.byref(tr.make_camera(big)),
                            C.byref(tr.make_params(p, "fp32_resolve")),
                            C.byref(tr.frame_struct(small)), None)
    assert st == -1


def test_reference_total_past_32_bits_refused(tr):
    """14,000 identical cylinders spanning the scene list 4.8 G references
    at 24 cells per primitive: more than 2^32, whose 32-bit wrap (0.51 G)
    would pass the 2^29 limit (tests/test_grid_limits.py).  The build sums
    the total in 64 bits and refuses before the scan and the scatter; a
    normal scene still builds afterwards."""
    s = scenegen.stacked_cylinders()
    print("stacked cylinders", s.n_prims, flush=True)
    with pytest.raises(tr.TRError) as e:
        tr.Scene(s, cells_per_prim=24.0)
    assert e.value.status == -4
    assert "references" in str(e.value)
    gs = tr.Scene(scenegen.tiny_scene())
    gs.destroy()
