"""Pins of the oracle's Targa file writer (run-length true colour, the
"Image I/O" phase of Table 5; the file format is a reading):
  * hand-worked bytes of a two-row image (header, run, raw and run packets,
    footer);
  * 128-pixel splits of long runs and long raw stretches, a run of 129
    (128 + a run packet of 1), and rows never joined by a packet;
  * an independent decoder (Pillow) reads random images with every kind of
    run back to the exact pixels, in the right orientation and channel
    order, and a quantised render of the tiny scene too;
  * closed-form sizes of all-distinct and all-equal images; size limits.
CPU only."""
import io
import math

import numpy as np
import pytest
from PIL import Image

import scenegen

FOOTER = b"\x00" * 8 + b"TRUEVISION-XFILE.\x00"


def _decode(data: bytes) -> np.ndarray:
    img = Image.open(io.BytesIO(data))
    assert img.format == "TGA" and img.mode == "RGB"
    return np.asarray(img)


def test_hand_worked_bytes(oracle_mod):
    a = np.zeros((2, 6, 3), np.uint8)
    a[0, :3] = [10, 20, 30]
    a[0, 3] = [1, 2, 3]
    a[0, 4:] = [5, 5, 5]
    a[1] = np.arange(18).reshape(6, 3)
    want = bytes([0, 0, 10, 0, 0, 0, 0, 0, 0, 0, 0, 0, 6, 0, 2, 0, 24, 0x20])
    want += bytes([0x82, 30, 20, 10])              # run of 3
    want += bytes([0x00, 3, 2, 1])                 # one raw pixel
    want += bytes([0x81, 5, 5, 5])                 # run of 2
    want += bytes([0x05]) + bytes(a[1][:, ::-1].reshape(-1).tolist())  # raw 6
    want += FOOTER
    assert oracle_mod.tga_encode(a) == want


def _packets(body: bytes):
    """(kind, count) of each packet in a body of 24-bit packets."""
    out, i = [], 0
    while i < len(body):
        h = body[i]
        c = (h & 0x7F) + 1
        if h & 0x80:
            out.append(("run", c))
            i += 4
        else:
            out.append(("raw", c))
            i += 1 + 3 * c
    assert i == len(body)
    return out


def test_splits_and_rows(oracle_mod):
    run = np.tile(np.array([[[7, 8, 9]]], np.uint8), (1, 300, 1))
    assert _packets(oracle_mod.tga_encode(run)[18:-26]) == [("run", 128), ("run", 128), ("run", 44)]
    distinct = np.arange(600, dtype=np.uint16).astype(np.uint8).reshape(1, 200, 3)
    distinct[0, :, 0] = np.arange(200) % 256  # no two neighbours equal
    assert _packets(oracle_mod.tga_encode(distinct)[18:-26]) == [("raw", 128), ("raw", 72)]
    r129 = np.zeros((1, 131, 3), np.uint8)
    r129[0, 129] = [1, 1, 1]
    r129[0, 130] = [2, 2, 2]
    assert _packets(oracle_mod.tga_encode(r129)[18:-26]) == [("run", 128), ("run", 1), ("raw", 2)]
    # two rows of one colour: a packet per row, never one across the rows
    same = np.full((2, 5, 3), 200, np.uint8)
    assert _packets(oracle_mod.tga_encode(same)[18:-26]) == [("run", 5), ("run", 5)]


def _random_image(rng, h, w):
    """Rows of random colours with run lengths drawn from 1..300 (singles
    most often), some rows repeating the row above."""
    img = np.zeros((h, w, 3), np.uint8)
    for y in range(h):
        if y and rng.random() < 0.2:
            img[y] = img[y - 1]
            continue
        x = 0
        while x < w:
            n = int(rng.choice([1, 1, 1, 2, 3, 5, 127, 128, 129, 300]))
            img[y, x:x + n] = rng.integers(0, 4, 3) * 85  # few colours: equal neighbours happen
            x += n
    return img


@pytest.mark.parametrize("h,w", [(1, 1), (1, 2), (3, 1), (7, 64), (5, 65), (9, 129), (17, 700),
                                 (40, 333)])
def test_independent_decoder(oracle_mod, h, w):
    rng = np.random.default_rng(h * 1000 + w)
    img = _random_image(rng, h, w)
    data = oracle_mod.tga_encode(img)
    assert data[-26:] == FOOTER
    assert np.array_equal(_decode(data), img)
    # also a few noise images (almost no runs)
    noise = rng.integers(0, 256, (h, w, 3), dtype=np.uint8)
    assert np.array_equal(_decode(oracle_mod.tga_encode(noise)), noise)


def test_rendered_frame(oracle_mod):
    s, c, p = scenegen.tiny_workload()
    out = oracle_mod.render(s, c, p, grid=4.0)
    img = oracle_mod.quantize_rgb8(out["rgb"].astype(np.float32))
    data = oracle_mod.tga_encode(img)
    assert np.array_equal(_decode(data), img)
    assert len(data) < img.size  # the background compresses


def test_sizes_and_limits(oracle_mod):
    for h, w in ((3, 200), (2, 128), (1, 1000)):
        x = np.arange(w)
        img = np.stack([x % 256, x // 256, np.zeros(w, int)], axis=-1).astype(np.uint8)
        img = np.repeat(img[None], h, axis=0)
        assert len(oracle_mod.tga_encode(img)) == 44 + h * (3 * w + math.ceil(w / 128))
        assert len(oracle_mod.tga_encode(np.zeros((h, w, 3), np.uint8))) == 44 + h * 4 * math.ceil(w / 128)
    with pytest.raises(ValueError):
        oracle_mod.tga_encode(np.zeros((1, 65536, 3), np.uint8))
    big = oracle_mod.tga_encode(np.zeros((1, 65535, 3), np.uint8))
    assert big[12:14] == bytes([0xFF, 0xFF])
