"""Antialiasing (several primary samples per pixel) on the GPU against the
oracle: one sample is the plain renderer bit for bit; the plain FP64 path
reproduces the oracle's sample positions, AO streams and mean; the FP32
wavefront path agrees within the FP32 tolerance, with a budget for the rare
sub-sample whose decision flips; batches, launch shapes and errors."""

import numpy as np
import pytest

import scenegen
from parity_util import DECISION_AGREE_MIN, HIT_AGREE_MIN, compare, flat_at, frame_to_numpy

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


def _params(p, **kw):
    return scenegen.Params(**{**p.__dict__, **kw})


def _gpu(tr, gscene, cam, params, precision, tune=None):
    import torch
    fr = tr.render(gscene, cam, params, precision=precision, outputs=OUT, tune=tune)
    torch.cuda.synchronize()
    return frame_to_numpy(fr)


def _small_protein_camera():
    c = scenegen.protein_camera(scenegen.RES_1MP)
    return scenegen.Camera(c.eye, c.lookat, c.up, c.fovy_deg, 241, 284)


def _aa_fp32_parity(m, got, ref, A, S):
    # Sample 0 (the pixel centre) carries hit id and masks: the FP32 bar on
    # hits and decisions (its colour is mixed with the other samples').
    assert m["hit_agree"] >= HIT_AGREE_MIN, m
    assert m["decision_agree"] >= DECISION_AGREE_MIN, m
    # A sub-sample's hit or AO decision may flip like any FP32 ray (about 1e-5
    # per ray); such a pixel moves by up to 1/A.  Expected share of pixels
    # with a flipped sub-sample: (A - 1) * (1 + S) * 1e-5; allow 10x.
    g = np.asarray(got["rgb"], np.float64).reshape(-1, 3)
    r = np.asarray(ref["rgb"], np.float64).reshape(-1, 3)
    err = np.abs(g - r).max(axis=1)
    bad = float((err > 1e-3).mean())
    budget = 10 * (A - 1) * (1 + S) * 1e-5
    assert bad <= budget, (bad, budget)
    ok = err <= 1e-3
    assert float(np.sqrt((err[ok] ** 2).mean())) <= 1e-4


@pytest.mark.parametrize("prec", ["fp32_resolve", "fp64"])
def test_one_sample_is_plain(tr, protein, prec):
    s, gs = protein
    c = _small_protein_camera()
    p = scenegen.Params(ao_samples=8, seed=2)
    print("aa one sample", prec, flush=True)
    base = _gpu(tr, gs, c, p, prec)
    for a in (0, 1):
        got = _gpu(tr, gs, c, _params(p, aa_samples=a), prec)
        for k in OUT:
            assert np.array_equal(got[k], base[k]), (a, k)


def test_tiny_fp64_matches_oracle(tr, oracle_mod):
    s, c, p = scenegen.tiny_workload()
    p = _params(p, aa_samples=4)
    print("aa tiny fp64", flush=True)
    got = _gpu(tr, tr.Scene(s), c, p, "fp64")
    ref = oracle_mod.render(s, c, p, grid=None)
    m = compare(got, ref, p.ao_samples, s.n_lights)
    print(m)
    assert m["hit_mismatch"] == 0, m
    assert m["decision_flips"] <= 2, m
    # every sample reproduced: float rounding of the FP64 colours and of the
    # float sum of four of them
    err = np.abs(got["rgb"].astype(np.float64) - ref["rgb"]).max(axis=2)
    assert float((err > 4e-7).mean()) <= 1e-3, float(err.max())
    # the mean really mixes samples: edge pixels differ from the centre render
    plain = _gpu(tr, tr.Scene(s), c, _params(p, aa_samples=1), "fp64")
    assert int((np.abs(plain["rgb"] - got["rgb"]).max(axis=2) > 0.05).sum()) > 50


def test_tiny_fp32_matches_oracle(tr, oracle_mod):
    s, c, p = scenegen.tiny_workload()
    A = 4
    p = _params(p, aa_samples=A)
    print("aa tiny fp32_resolve", flush=True)
    got = _gpu(tr, tr.Scene(s), c, p, "fp32_resolve")
    ref = oracle_mod.render(s, c, p, grid=None)
    m = compare(got, ref, p.ao_samples, s.n_lights)
    print(m)
    _aa_fp32_parity(m, got, ref, A, p.ao_samples)


@pytest.mark.parametrize("prec", ["fp32_resolve", "fp64"])
def test_protein_small_matches_oracle(tr, oracle_mod, protein, prec):
    s, gs = protein
    c = _small_protein_camera()
    A, S = 4, 8
    p = scenegen.Params(ao_samples=S, seed=2, aa_samples=A)
    print("aa protein 241x284", prec, flush=True)
    got = _gpu(tr, gs, c, p, prec)
    ref = oracle_mod.render(s, c, p, grid=4.0)
    m = compare(got, ref, S, s.n_lights)
    print(m)
    if prec == "fp64":
        assert m["hit_mismatch"] == 0 and m["decision_flips"] <= 2, m
        err = np.abs(got["rgb"].astype(np.float64) - ref["rgb"]).max(axis=2)
        assert float((err > 4e-7).mean()) <= 1e-3, float(err.max())
    else:
        _aa_fp32_parity(m, got, ref, A, S)


def test_protein_17mp_sampled(tr, oracle_mod, protein):
    # full 3860x4548 frame with 4 primary samples per pixel; the oracle
    # computes a seeded sample of its pixels one by one
    s, gs = protein
    c = scenegen.protein_camera(scenegen.RES_17MP)
    A, S = 4, 16
    p = scenegen.Params(ao_samples=S, seed=2, aa_samples=A)
    print("aa protein 17.6MP fp32_resolve", flush=True)
    got = _gpu(tr, gs, c, p, "fp32_resolve")
    pix = scenegen.sample_pixels(c.width, c.height, 4000, 23)
    ref = oracle_mod.render(s, c, p, grid=4.0, pix=pix)
    sub = flat_at(got, pix)
    m = compare(sub, ref, S, s.n_lights)
    print(m)
    _aa_fp32_parity(m, sub, ref, A, S)
    assert np.all(got["rgb"] >= 0) and np.all(got["rgb"] <= 1)


def test_batch_and_tunes_are_bitwise(tr, protein):
    import torch
    s, gs = protein
    c = _small_protein_camera()
    ps = [scenegen.Params(ao_samples=8, seed=2, aa_samples=3),
          scenegen.Params(ao_samples=4, seed=9, view_id=3),
          scenegen.Params(ao_samples=8, seed=5, aa_samples=2)]
    print("aa batch", flush=True)
    alone = [_gpu(tr, gs, c, p, "fp32_resolve") for p in ps]
    frames = [tr.alloc_frame(c, OUT, False) for _ in ps]
    tr.render_batch_into([gs] * 3, [c] * 3, ps, frames, precision="fp32_resolve")
    torch.cuda.synchronize()
    for a, f in zip(alone, frames):
        f = frame_to_numpy(f)
        for k in OUT:
            assert np.array_equal(a[k], f[k]), k
    # a different launch shape gives the same bits
    t = _gpu(tr, gs, c, ps[0], "fp32_resolve",
             tune=dict(tile_w=16, banks=3, waves_per_cu=12, refill_below=40, stripe=8))
    for k in OUT:
        assert np.array_equal(alone[0][k], t[k]), k
    # FP64 jobs of a batch take the plain path, antialiased as alone
    f64 = [tr.alloc_frame(c, OUT, False) for _ in range(2)]
    tr.render_batch_into([gs] * 2, [c] * 2, [ps[2], ps[1]], f64, precision="fp64")
    torch.cuda.synchronize()
    one = _gpu(tr, gs, c, ps[2], "fp64")
    for k in OUT:
        assert np.array_equal(one[k], frame_to_numpy(f64[0])[k]), k


def test_errors(tr, protein):
    s, gs = protein
    c = _small_protein_camera()
    for a in (-1, 257):
        with pytest.raises(tr.TRError) as e:
            tr.render(gs, c, scenegen.Params(ao_samples=4, aa_samples=a), outputs=("rgb",))
        assert e.value.status == -1
    fr = tr.alloc_frame(c, ("rgb",), False)
    n = tr.tile_count(c.width, c.height)
    with pytest.raises(tr.TRError) as e:
        tr.render_batch_tiles_into([gs], [c], [scenegen.Params(aa_samples=2)], [fr], [0], [n])
    assert e.value.status == -4
    with pytest.raises(tr.TRError) as e:
        tr.Graph([gs], [c], [scenegen.Params(aa_samples=2)], [fr])
    assert e.value.status == -4
    g = tr.Graph([gs], [c], [scenegen.Params()], [fr])
    with pytest.raises(tr.TRError) as e:
        g.update(params=[scenegen.Params(aa_samples=2)])
    assert e.value.status == -4
    g.destroy()
