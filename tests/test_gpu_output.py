"""GPU 8-bit frame output (tr_frame_quantize) against the oracle, bit for bit:
ragged sizes, unaligned buffers, edge values, a rendered frame, the full
17.6 MP frame size, and the host download + PPM encoding."""
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
