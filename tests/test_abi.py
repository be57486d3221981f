"""The C-ABI library loads and exports every function include/tr.h declares,
and argument validation rejects bad input before any device work (no GPU
needed for these calls)."""
import ctypes as C
import math
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tr.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(tr_[a-z_0-9]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def tr():
    import paper_0801_1500_amd as tr
    if not os.path.exists(tr.LIB_PATH):
        from paper_0801_1500_amd import build
        build.build()
    return tr


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("tr_scene_build", "tr_render", "tr_render_batch", "tr_scene_destroy",
              "tr_last_error", "tr_abi_version"):
        assert n in names


def test_every_declared_symbol_exported(tr):
    L = tr.lib()
    for n in _declared():
        assert hasattr(L, n), n
    assert tr.abi_version() == 4


def test_stat_names_follow_the_header(tr):
    # the binding's stat names are the header's enum, in order
    import os
    import re
    hdr = open(os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                            "include", "tr.h")).read()
    start = hdr.index("TR_STAT_PIXELS = 0")
    body = hdr[start:hdr.index("TR_STAT_COUNT", start)]
    names = re.findall(r"^\s*TR_STAT_([A-Z0-9_]+)", body, re.M)
    assert [n.lower() for n in names] == tr.STAT_NAMES
    assert tr.STAT_COUNT == len(names)


def test_tile_count(tr):
    assert tr.tile_count(128, 128) == 256
    assert tr.tile_count(3860, 4548, 8) == 483 * 569
    assert tr.tile_count(65, 9, 16) == 5 * 3
    assert tr.tile_count(3860, 4548) == 61 * 4548  # default: 64 x 1 tiles
    assert tr.tile_count(3860, 4548, 64) == 61 * 4548
    with pytest.raises(ValueError):
        tr.tile_count(10, 10, 7)


def test_tga_bound_and_argument_errors(tr):
    # host-only: the size bound, and the checks that precede any device work
    import ctypes as C
    assert tr.tga_max_bytes(1, 1) == 44 + 4
    assert tr.tga_max_bytes(3860, 4548) == 44 + 4 * 3860 * 4548
    assert tr.tga_max_bytes(65535, 65535) == 44 + 4 * 65535 * 65535
    for w, h in ((0, 1), (1, 0), (65536, 1), (1, 65536), (-5, 3)):
        assert tr.lib().tr_tga_max_bytes(w, h) == -1
    L = tr.lib()
    n = C.c_int64(123)
    assert L.tr_frame_encode_tga(None, 4, 4, None, 0, C.byref(n), None) == -1  # NULL image
    assert n.value == 0
    assert L.tr_frame_encode_tga(None, 4, 4, None, 0, None, None) == -1       # NULL size
    buf = (C.c_uint8 * 16)()
    for w, h in ((0, 4), (4, 0), (65536, 1)):
        assert L.tr_frame_encode_tga(C.addressof(buf), w, h, None, 0, C.byref(n), None) == -1
    assert L.tr_frame_encode_tga(C.addressof(buf), 1, 1, None, 8, C.byref(n), None) == -1  # NULL out
    assert L.tr_frame_encode_tga(C.addressof(buf), 1, 1, C.addressof(buf), -1, C.byref(n), None) == -1


def test_frame_footprint(tr):
    import scenegen
    c = scenegen.protein_camera(scenegen.RES_17MP)
    p = scenegen.Params()
    assert tr.frame_footprint(c, p, 1) == 3860 * 4548 * 12
    assert tr.frame_footprint(c, p, 15) == 3860 * 4548 * 21


def _status(fn, *args):
    return fn(*args)


def test_scene_validation_rejects(tr):
    L = tr.lib()
    good_c = np.zeros((1, 3)); good_r = np.ones(1); rgb = np.ones((1, 3), np.float32)
    bad_r = np.array([0.0]); nan_c = np.array([[math.nan, 0.0, 0.0]])

    def build(center, radius, n_lights=0, cells=0.0, cyl=None):
        args = [1, center.ctypes.data, radius.ctypes.data, rgb.ctypes.data]
        if cyl is None:
            args += [0, None, None, None, None]
        else:
            a, b = cyl
            args += [1, a.ctypes.data, b.ctypes.data, good_r.ctypes.data, rgb.ctypes.data]
        ld = np.array([[0.0, 0.0, 1.0]] * max(n_lights, 1))
        args += [n_lights, ld.ctypes.data, ld.ctypes.data, cells]
        d = tr.SceneDesc(*args)
        h = C.c_void_p()
        return L.tr_scene_build(C.byref(d), None, C.byref(h))

    assert build(good_c, bad_r) == tr.TR_EINVAL
    assert b"radius" in L.tr_last_error()
    assert build(nan_c, good_r) == tr.TR_EINVAL
    assert build(good_c, good_r, n_lights=9) == tr.TR_EINVAL
    assert build(good_c, good_r, cells=-1.0) == tr.TR_EINVAL
    z = np.zeros((1, 3))
    assert build(good_c, good_r, cyl=(z, z)) == tr.TR_EINVAL
    assert b"zero length" in L.tr_last_error()
    h = C.c_void_p()
    assert L.tr_scene_build(None, None, C.byref(h)) == tr.TR_EINVAL
    # 2^27 primitives exceed the traversal's record offsets (16 x id in a
    # signed 32-bit word; the count is checked before any array is read)
    big = tr.SceneDesc(1 << 26, good_c.ctypes.data, good_r.ctypes.data, rgb.ctypes.data,
                       1 << 26, good_c.ctypes.data, good_c.ctypes.data, good_r.ctypes.data,
                       rgb.ctypes.data, 0, None, None, 0.0)
    assert L.tr_scene_build(C.byref(big), None, C.byref(h)) == tr.TR_EINVAL
    assert b"too many primitives" in L.tr_last_error()


def test_render_validation_rejects(tr):
    import scenegen
    L = tr.lib()
    c = tr.make_camera(scenegen.protein_camera())
    p = tr.make_params(scenegen.Params())
    f = tr.Frame(None, None, None, None, None)
    # NULL scene / frame->rgb, checked before any device call
    assert L.tr_render(None, C.byref(c), C.byref(p), C.byref(f), None) == tr.TR_EINVAL
    assert L.tr_render_batch(0, None, None, None, None, None) == tr.TR_EINVAL
    assert L.tr_render_batch_tiles(1, None, None, None, None, None, None, None, None) == tr.TR_EINVAL
    assert L.tr_graph_launch(None, None) == tr.TR_EINVAL
    assert L.tr_debug_philox(-1, None, None, None, None) == tr.TR_EINVAL
    assert L.tr_autotune(None, None, None, None, None, None) == tr.TR_EINVAL


def test_default_tune(tr):
    t = tr.default_tune()
    assert t["tile_w"] in (4, 8, 16, 32, 64) and t["banks"] in (2, 3)


def test_scene_load_rejects_bad_files(tr, tmp_path):
    # every check runs before any device call
    import struct
    L = tr.lib()
    h = C.c_void_p()
    assert L.tr_scene_load(None, None, C.byref(h)) == tr.TR_EINVAL
    assert L.tr_scene_load(str(tmp_path / "missing.bin").encode(), None, C.byref(h)) == tr.TR_EINVAL
    short = tmp_path / "short.bin"
    short.write_bytes(b"TRSCENE1" + b"\0" * 8)
    assert L.tr_scene_load(str(short).encode(), None, C.byref(h)) == tr.TR_EINVAL
    assert b"too short" in L.tr_last_error()
    bad = tmp_path / "bad.bin"
    bad.write_bytes(b"NOTASCN1" + b"\0" * 32)
    assert L.tr_scene_load(str(bad).encode(), None, C.byref(h)) == tr.TR_EINVAL
    assert b"bad magic" in L.tr_last_error()
    # counts that need more bytes than the file has
    trunc = tmp_path / "trunc.bin"
    trunc.write_bytes(b"TRSCENE1" + struct.pack("<qqiid", 5, 0, 1, 0, 0.0) + b"\0" * 16)
    assert L.tr_scene_load(str(trunc).encode(), None, C.byref(h)) == tr.TR_EINVAL
    assert b"its counts need" in L.tr_last_error()
    neg = tmp_path / "neg.bin"
    neg.write_bytes(b"TRSCENE1" + struct.pack("<qqiid", -1, 0, 0, 0, 0.0))
    assert L.tr_scene_load(str(neg).encode(), None, C.byref(h)) == tr.TR_EINVAL
    assert b"bad counts" in L.tr_last_error()
    flags = tmp_path / "flags.bin"
    flags.write_bytes(b"TRSCENE1" + struct.pack("<qqiid", 0, 0, 0, 4, 0.0))
    assert L.tr_scene_load(str(flags).encode(), None, C.byref(h)) == tr.TR_EINVAL
    assert b"unknown flags" in L.tr_last_error()
    # a triangle section announced by flag bit 1 but missing, or too short
    tri = tmp_path / "tri.bin"
    tri.write_bytes(b"TRSCENE1" + struct.pack("<qqiid", 0, 0, 0, 2, 0.0))
    assert L.tr_scene_load(str(tri).encode(), None, C.byref(h)) == tr.TR_EINVAL
    assert b"its counts need" in L.tr_last_error()
    tri.write_bytes(b"TRSCENE1" + struct.pack("<qqiidq", 0, 0, 0, 2, 0.0, 3) + b"\0" * 8)
    assert L.tr_scene_load(str(tri).encode(), None, C.byref(h)) == tr.TR_EINVAL
    assert b"its counts need" in L.tr_last_error()
    # opacity arrays announced by flag bit 0 but missing
    opq = tmp_path / "opq.bin"
    opq.write_bytes(b"TRSCENE1" + struct.pack("<qqiid", 1, 0, 0, 1, 0.0) + b"\0" * 48)
    assert L.tr_scene_load(str(opq).encode(), None, C.byref(h)) == tr.TR_EINVAL
    assert b"its counts need" in L.tr_last_error()
    assert not h.value


def test_frame_buffers_checked_before_the_call(tr):
    """frame_struct with the camera refuses buffers whose dtype, layout or
    size do not match the frame (their addresses would let the kernel write
    out of bounds), before anything reaches the library; on this CPU-only
    host a well-formed tensor still fails the device check."""
    import torch
    cam = tr.Camera((C.c_double * 3)(0, 0, 30), (C.c_double * 3)(0, 0, 0), (C.c_double * 3)(0, 1, 0),
                    50.0, 7, 5)
    good = {"rgb": torch.zeros(5, 7, 3), "hit_id": torch.zeros(5, 7, dtype=torch.int32),
            "ao_mask": torch.zeros(5, 7, dtype=torch.int32),
            "light_mask": torch.zeros(5, 7, dtype=torch.uint8),
            "stats": torch.zeros(tr.STAT_COUNT, dtype=torch.int64)}
    bad = [
        ("rgb", torch.zeros(5, 7, 3, dtype=torch.float64), "dtype"),
        ("rgb", torch.zeros(5, 7, 2), "elements"),
        ("rgb", torch.zeros(7, 5, 3).transpose(0, 1), "contiguous"),
        ("hit_id", torch.zeros(5, 7), "dtype"),
        ("hit_id", torch.zeros(5, 8, dtype=torch.int32), "elements"),
        ("ao_mask", torch.zeros(5, 7, dtype=torch.int64), "dtype"),
        ("light_mask", torch.zeros(5, 7, dtype=torch.uint8)[:, :6], "contiguous"),
        ("stats", torch.zeros(3, dtype=torch.int64), "elements"),
    ]
    for key, val, what in bad:
        with pytest.raises(ValueError, match=what):
            tr.frame_struct({**good, key: val}, cam)
    with pytest.raises(ValueError, match="CUDA"):
        tr.frame_struct(good, cam)
    # without the camera (no check) only the addresses are taken
    tr.frame_struct(good)
