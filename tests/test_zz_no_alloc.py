"""tr_render_batch_noalloc (the batch render that allocates nothing) through
the C ABI, against tr_render_batch on the same jobs: bit-identical frames
and counters, on two calls in a row, the second with fewer and smaller
jobs; a job table past the limit and an antialiased job are refused before
anything is rendered."""
import ctypes as C

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


def _abi_call(tr, entry, scenes, cams, params, frames, precision="fp32_resolve"):
    """Call a batch entry point of the C ABI directly (ctypes arrays)."""
    n, sc, cm, pr, fr = tr._arrays(scenes, cams, params, frames, precision)
    if entry == "tr_render_batch_noalloc":
        return tr.lib().tr_render_batch_noalloc(n, sc, cm, pr, fr, None, None)
    return tr.lib().tr_render_batch(n, sc, cm, pr, fr, None)


def _jobs(first):
    s_tiny, c_tiny, p_tiny = scenegen.tiny_workload()
    s_prot = scenegen.protein_scene()
    if first:
        cams = [c_tiny, scenegen.protein_camera((241, 284)), scenegen.protein_camera(scenegen.RES_1MP)]
        params = [p_tiny, scenegen.Params(ao_samples=16, seed=2), scenegen.Params(ao_samples=8, seed=5)]
        scenes = ["tiny", "protein", "protein"]
    else:
        cams = [scenegen.Camera(c_tiny.eye, c_tiny.lookat, c_tiny.up, c_tiny.fovy_deg, 67, 45)]
        params = [scenegen.Params(ao_samples=4, seed=9)]
        scenes = ["tiny"]
    return scenes, cams, params, {"tiny": s_tiny, "protein": s_prot}


def test_noalloc_equals_batch_twice(tr, oracle_mod):
    import torch
    gpu = {}
    for first in (True, False):
        names, cams, params, host = _jobs(first)
        for k in set(names):
            if k not in gpu:
                gpu[k] = tr.Scene(host[k])
        scenes = [gpu[k] for k in names]
        print("no-alloc batch", "first" if first else "second", len(names), "jobs",
              [(c.width, c.height) for c in cams], flush=True)
        got, want = [], []
        for entry, out in (("tr_render_batch_noalloc", got), ("tr_render_batch", want)):
            frames = []
            for c in cams:
                f = tr.alloc_frame(c, OUT, stats=False)
                for v in f.values():
                    v.fill_(7)  # whatever is not written shows
                frames.append(f)
            st = torch.zeros(tr.STAT_COUNT, dtype=torch.int64, device="cuda")
            for f in frames:
                f["stats"] = st
            assert _abi_call(tr, entry, scenes, cams, params, frames) == 0, tr.lib().tr_last_error()
            torch.cuda.synchronize()
            out.append(([frame_to_numpy({k: f[k] for k in OUT}) for f in frames],
                        st.cpu().numpy().copy()))
        (g_frames, g_st), (w_frames, w_st) = got[0], want[0]
        for gf, wf in zip(g_frames, w_frames):
            for k in OUT:
                assert np.array_equal(gf[k], wf[k]), k
        # the exact counters agree (traversal counters need a counting launch)
        names_st = dict(zip(tr.STAT_NAMES, range(tr.STAT_COUNT)))
        for k in ("pixels", "hit_pixels", "ao_rays", "shadow_rays", "rays_traced"):
            assert g_st[names_st[k]] == w_st[names_st[k]], k
        assert g_st[names_st["pixels"]] == sum(c.width * c.height for c in cams)
        # and the first job meets the FP32 bar against the oracle
        ref = oracle_mod.render(host[names[0]], cams[0], params[0], grid=4.0)
        assert_fp32_parity(compare(g_frames[0], ref, params[0].ao_samples, host[names[0]].n_lights))


def test_noalloc_refusals(tr):
    import torch
    s, c, p = scenegen.tiny_workload()
    gs = tr.Scene(s)
    n = tr.NOALLOC_MAX_JOBS + 1
    frames = [tr.alloc_frame(c, ("rgb",)) for _ in range(n)]
    for f in frames:
        f["rgb"].fill_(7)
    assert _abi_call(tr, "tr_render_batch_noalloc", [gs] * n, [c] * n, [p] * n, frames) == -1
    aa = scenegen.Params(ao_samples=4, seed=1, aa_samples=2)
    assert _abi_call(tr, "tr_render_batch_noalloc", [gs, gs], [c, c], [p, aa], frames[:2]) == -4
    torch.cuda.synchronize()
    for f in frames:
        assert (f["rgb"] == 7).all()
