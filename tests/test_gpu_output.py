"""GPU 8-bit frame output (tr_frame_quantize) against the oracle, bit for bit:
ragged sizes, unaligned buffers, edge values, a rendered frame, the full
17.6 MP frame size, and the host download + PPM encoding; the GPU Targa
writer (tr_frame_encode_tga) against the oracle's, byte for byte, on images
of every run structure and size limit and on rendered 1.1 MP and 17.6 MP
frames."""
import numpy as np
import pytest

import scenegen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tr():
    import paper_0801_1500_amd as tr
    tr.lib()
    return tr


EDGE = np.array([0.0, -0.0, 1.0, 0.5, 0.25, 0.75, 1.0 / 256, -1.0, 2.0, np.inf, -np.inf, np.nan,
                 1e-30, -1e-30, 0.99999994, 1.0000001], dtype=np.float32)


def _values(n, seed):
    rng = np.random.default_rng(seed)
    v = rng.uniform(-0.2, 1.2, n).astype(np.float32)
    b = ((np.arange(255) + 0.5) / 255.0).astype(np.float32)  # rounding boundaries
    k = min(n, 255)
    v[:k] = np.nextafter(b[:k], np.float32(rng.integers(0, 2)))
    v[-min(n, len(EDGE)):] = EDGE[:min(n, len(EDGE))]
    return v


@pytest.mark.parametrize("n", [1, 3, 4, 5, 1023, 1024, 4095, 4096, 4097, 65539, (1 << 20) + 7])
@pytest.mark.parametrize("shift_in,shift_out", [(0, 0), (1, 0), (0, 1), (3, 2)])
def test_quantize_bit_exact(tr, oracle_mod, n, shift_in, shift_out):
    import torch
    print("quantize case", n, shift_in, shift_out, flush=True)
    v = _values(n, n + 7 * shift_in)
    src = torch.zeros(n + 8, dtype=torch.float32, device="cuda")
    src[shift_in:shift_in + n] = torch.from_numpy(v).cuda()
    dst = torch.full((n + 8,), 77, dtype=torch.uint8, device="cuda")
    tr.quantize_rgb8(src[shift_in:shift_in + n], out=dst[shift_out:shift_out + n])
    torch.cuda.synchronize()
    d = dst.cpu().numpy()
    assert np.array_equal(d[shift_out:shift_out + n], oracle_mod.quantize_rgb8(v))
    # nothing written outside the range
    assert np.all(d[:shift_out] == 77) and np.all(d[shift_out + n:] == 77)


def test_quantize_empty_and_errors(tr):
    import ctypes as C
    import torch
    L = tr.lib()
    assert L.tr_frame_quantize(None, 0, None, None) == tr.TR_OK
    assert L.tr_frame_quantize(None, 5, None, None) == tr.TR_EINVAL
    assert L.tr_frame_quantize(None, -1, None, None) == tr.TR_EINVAL
    with pytest.raises(TypeError):
        tr.quantize_rgb8(torch.zeros(4, dtype=torch.float64, device="cuda"))


def test_quantize_full_frame_and_rendered(tr, oracle_mod):
    import torch
    # the 17.6 MP frame's size, every value checked
    H, W = scenegen.RES_17MP[1], scenegen.RES_17MP[0]
    g = torch.Generator(device="cuda").manual_seed(5)
    big = torch.rand((H, W, 3), generator=g, device="cuda", dtype=torch.float32) * 1.2 - 0.1
    q = tr.quantize_rgb8(big)
    torch.cuda.synchronize()
    assert q.shape == (H, W, 3) and q.dtype == torch.uint8
    assert np.array_equal(q.cpu().numpy(), oracle_mod.quantize_rgb8(big.cpu().numpy()))
    # a rendered frame, downloaded to pinned memory and encoded
    s, c, p = scenegen.tiny_workload()
    gs = tr.Scene(s)
    fr = tr.render(gs, c, p, precision="fp32_resolve", outputs=("rgb",))
    host, ev = tr.frame_to_host_rgb8(fr)
    ev.synchronize()
    want = oracle_mod.quantize_rgb8(fr["rgb"].cpu().numpy())
    assert np.array_equal(host.numpy(), want)
    ppm = tr.encode_ppm(host)
    head = b"P6\n%d %d\n255\n" % (c.width, c.height)
    assert ppm[:len(head)] == head and ppm[len(head):] == want.tobytes()


# ---- Targa file (tr_frame_encode_tga) against the oracle's writer, byte for byte

def _tga_images():
    import sys
    import os
    sys.path.insert(0, os.path.dirname(__file__))
    from test_oracle_tga import _random_image
    rng = np.random.default_rng(77)
    out = []
    for h, w in ((1, 1), (1, 2), (2, 3), (3, 63), (2, 64), (2, 65), (4, 127), (3, 128), (3, 129),
                 (5, 300), (9, 1000), (1, 65535), (65535, 1), (64, 4097)):
        out.append(("runs", h, w, _random_image(rng, h, w)))
        out.append(("noise", h, w, rng.integers(0, 256, (h, w, 3), dtype=np.uint8)))
        out.append(("flat", h, w, np.full((h, w, 3), 17, np.uint8)))
    return out


def test_tga_bit_exact(tr, oracle_mod):
    import torch
    for kind, h, w, img in _tga_images():
        print("tga case", kind, h, w, flush=True)
        got = tr.encode_tga(torch.from_numpy(img).cuda())
        torch.cuda.synchronize()
        want = oracle_mod.tga_encode(img)
        assert got.numel() == len(want), (kind, h, w)
        assert got.cpu().numpy().tobytes() == want, (kind, h, w)


def test_tga_rendered_frames(tr, oracle_mod):
    # the full path: render, quantise, encode, all on the GPU; the oracle
    # encodes the same 8-bit image; an independent decoder reads the file
    import io

    import torch
    from PIL import Image
    s = scenegen.protein_scene()
    gs = tr.Scene(s)
    for res in (scenegen.RES_1MP, scenegen.RES_17MP):
        cam = scenegen.protein_camera(res)
        print("tga frame", res, flush=True)
        fr = tr.render(gs, cam, scenegen.Params(ao_samples=16, seed=2), outputs=("rgb",))
        q = tr.quantize_rgb8(fr["rgb"])
        f = tr.encode_tga(q)
        torch.cuda.synchronize()
        img = q.cpu().numpy()
        data = f.cpu().numpy().tobytes()
        assert data == oracle_mod.tga_encode(img)
        assert len(data) < img.size  # the background compresses
        if res == scenegen.RES_1MP:
            assert np.array_equal(np.asarray(Image.open(io.BytesIO(data))), img)


def test_tga_errors_and_reuse(tr, oracle_mod):
    import torch
    img = np.zeros((4, 300, 3), np.uint8)
    img[:, ::2] = 200
    d = torch.from_numpy(img).cuda()
    want = oracle_mod.tga_encode(img)
    small = torch.empty(len(want) - 1, dtype=torch.uint8, device="cuda").fill_(9)
    with pytest.raises(tr.TRError) as e:
        tr.encode_tga(d, out=small)
    assert e.value.status == -1
    torch.cuda.synchronize()
    assert bool((small == 9).all())  # nothing written
    exact = torch.empty(len(want), dtype=torch.uint8, device="cuda")
    assert tr.encode_tga(d, out=exact).cpu().numpy().tobytes() == want
    with pytest.raises(ValueError):
        tr.tga_max_bytes(65536, 1)
    wide = torch.zeros((1, 65536, 3), dtype=torch.uint8, device="cuda")
    with pytest.raises(ValueError):  # no buffer size exists for it
        tr.encode_tga(wide)
    with pytest.raises(tr.TRError) as e:  # the library refuses it too
        tr.encode_tga(wide, out=torch.empty(16, dtype=torch.uint8, device="cuda"))
    assert e.value.status == -1
    # the per-stream scratch grows and shrinks across calls on one stream
    for h in (3, 700, 2):
        im = np.random.default_rng(h).integers(0, 3, (h, 50, 3), dtype=np.uint8) * 100
        assert tr.encode_tga(torch.from_numpy(im).cuda()).cpu().numpy().tobytes() == \
            oracle_mod.tga_encode(im)


def test_write_tga_file(tr, oracle_mod, tmp_path):
    # render -> Targa file on disk; an independent decoder reads it back as
    # the 8-bit image of the frame
    import torch
    from PIL import Image
    s, c, p = scenegen.tiny_workload()
    fr = tr.render(tr.Scene(s), c, p, outputs=("rgb",))
    path = str(tmp_path / "tiny.tga")
    n = tr.write_tga(fr, path)
    torch.cuda.synchronize()
    q = tr.quantize_rgb8(fr["rgb"]).cpu().numpy()
    data = open(path, "rb").read()
    assert len(data) == n and data == oracle_mod.tga_encode(q)
    assert np.array_equal(np.asarray(Image.open(path)), q)
