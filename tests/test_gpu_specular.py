"""The Phong highlight option on the GPU against the oracle: strength 0 is
the plain renderer bit for bit; the plain FP64 path reproduces the oracle;
the FP32 wavefront path meets the FP32 tolerance (tiny frame, a 241x284
protein frame, and sampled pixels of the 17.6 MP frame); argument errors."""
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


def _params(p, **kw):
    return scenegen.Params(**{**p.__dict__, **kw})


def _gpu(tr, gscene, cam, params, precision):
    import torch
    fr = tr.render(gscene, cam, params, precision=precision, outputs=OUT)
    torch.cuda.synchronize()
    return frame_to_numpy(fr)


def _small_protein_camera():
    c = scenegen.protein_camera(scenegen.RES_1MP)
    return scenegen.Camera(c.eye, c.lookat, c.up, c.fovy_deg, 241, 284)


@pytest.mark.parametrize("prec", ["fp32_resolve", "fp64"])
def test_zero_strength_is_plain(tr, protein, prec):
    s, gs = protein
    c = _small_protein_camera()
    p = scenegen.Params(ao_samples=8, seed=2)
    print("specular off", prec, flush=True)
    base = _gpu(tr, gs, c, p, prec)
    for n in (0.0, 7.0):
        got = _gpu(tr, gs, c, _params(p, specular=0.0, shininess=n), prec)
        for k in OUT:
            assert np.array_equal(got[k], base[k]), (n, k)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp32_resolve"])
def test_tiny_matches_oracle(tr, oracle_mod, prec):
    s, c, p = scenegen.tiny_workload()
    p = _params(p, specular=0.5, shininess=30.0)
    print("specular tiny", prec, flush=True)
    got = _gpu(tr, tr.Scene(s), c, p, prec)
    ref = oracle_mod.render(s, c, p, grid=None)
    m = compare(got, ref, p.ao_samples, s.n_lights)
    print(m)
    if prec == "fp64":
        assert m["hit_mismatch"] == 0 and m["decision_flips"] <= 2, m
        assert m["max_abs_agree"] <= 2.4e-7, m
    else:
        assert_fp32_parity(m)
    # the highlight is really there
    plain = oracle_mod.render(s, c, _params(p, specular=0.0), grid=None)
    assert int((ref["rgb"][..., 0] - plain["rgb"][..., 0] > 0.01).sum()) > 50


@pytest.mark.parametrize("prec", ["fp32_resolve", "fp64"])
def test_protein_small_matches_oracle(tr, oracle_mod, protein, prec):
    s, gs = protein
    c = _small_protein_camera()
    p = scenegen.Params(ao_samples=8, seed=2, specular=0.3, shininess=12.0)
    print("specular protein 241x284", prec, flush=True)
    got = _gpu(tr, gs, c, p, prec)
    ref = oracle_mod.render(s, c, p, grid=4.0)
    m = compare(got, ref, 8, s.n_lights)
    print(m)
    if prec == "fp64":
        assert m["hit_mismatch"] == 0 and m["decision_flips"] <= 2, m
        assert m["max_abs_agree"] <= 2.4e-7, m
    else:
        assert_fp32_parity(m)


def test_protein_17mp_sampled(tr, oracle_mod, protein):
    s, gs = protein
    c = scenegen.protein_camera(scenegen.RES_17MP)
    p = scenegen.Params(ao_samples=16, seed=2, specular=0.3, shininess=30.0)
    print("specular protein 17.6MP fp32_resolve", flush=True)
    got = _gpu(tr, gs, c, p, "fp32_resolve")
    pix = scenegen.sample_pixels(c.width, c.height, 20000, 29)
    ref = oracle_mod.render(s, c, p, grid=4.0, pix=pix)
    m = compare(flat_at(got, pix), ref, 16, s.n_lights)
    print(m)
    assert_fp32_parity(m)


def test_errors(tr, protein):
    s, gs = protein
    c = _small_protein_camera()
    bad = [dict(specular=-0.1), dict(specular=math.nan), dict(specular=math.inf),
           dict(specular=0.5, shininess=0.0), dict(specular=0.5, shininess=math.inf)]
    for kw in bad:
        with pytest.raises(tr.TRError) as e:
            tr.render(gs, c, scenegen.Params(ao_samples=4, **kw), outputs=("rgb",))
        assert e.value.status == -1, kw
    # the exponent is not read without a highlight
    tr.render(gs, c, scenegen.Params(ao_samples=4, specular=0.0, shininess=-1.0), outputs=("rgb",))
