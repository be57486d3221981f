"""Python binding of libtr.so, the gfx950 ambient-occlusion ray caster.

Argument marshalling only: every step of scene building and rendering runs in
the library's HIP kernels.  PyTorch provides device memory (output tensors)
and streams.  Importing this module does not touch the GPU; the first call
loads libtr.so and raises if it is missing or no GPU is present.
"""
from __future__ import annotations

import ctypes as C
import math
import os
from typing import Dict, List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtr.so")

TR_OK, TR_EINVAL, TR_ENOMEM, TR_EDEVICE, TR_EUNSUPPORTED = 0, -1, -2, -3, -4
PREC_FP64, PREC_FP32, PREC_FP32_RESOLVE = 0, 1, 2
PRECISIONS = {"fp64": PREC_FP64, "fp32": PREC_FP32, "fp32_resolve": PREC_FP32_RESOLVE}

STAT_NAMES = ["pixels", "hit_pixels", "ao_rays", "shadow_rays", "rays_traced", "cells",
              "sph_tests", "sph_hits", "cyl_tests", "cyl_hits", "resolves", "wave_iters",
              "lane_iters", "refills", "jumps", "cycles_traverse", "cycles_total", "tri_tests",
              "tri_hits", "stack_overflows", "stalls", "resolves_sph", "resolves_cyl",
              "resolves_tri", "resolves_nearest", "signs_f64", "cells_ao", "tests_ao",
              "cells_shadow", "tests_shadow", "tests_own", "cycles_resolve", "cycles_finish",
              "cycles_refill"]
STAT_COUNT = len(STAT_NAMES)


class TRError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("tr status %d: %s" % (status, msg))
        self.status = status


class SceneDesc(C.Structure):
    _fields_ = [
        ("n_spheres", C.c_int64), ("sph_center", C.c_void_p), ("sph_radius", C.c_void_p),
        ("sph_rgb", C.c_void_p),
        ("n_cylinders", C.c_int64), ("cyl_a", C.c_void_p), ("cyl_b", C.c_void_p),
        ("cyl_radius", C.c_void_p), ("cyl_rgb", C.c_void_p),
        ("n_lights", C.c_int32), ("light_dir", C.c_void_p), ("light_rgb", C.c_void_p),
        ("cells_per_prim", C.c_double), ("sph_opacity", C.c_void_p), ("cyl_opacity", C.c_void_p),
        ("n_triangles", C.c_int64), ("tri_v0", C.c_void_p), ("tri_v1", C.c_void_p),
        ("tri_v2", C.c_void_p), ("tri_rgb", C.c_void_p), ("tri_opacity", C.c_void_p),
        ("max_skip", C.c_int32)]


class Camera(C.Structure):
    _fields_ = [("eye", C.c_double * 3), ("lookat", C.c_double * 3), ("up", C.c_double * 3),
                ("fovy_deg", C.c_double), ("width", C.c_int32), ("height", C.c_int32)]


class Params(C.Structure):
    _fields_ = [("light_rescale", C.c_double), ("skylight", C.c_double),
                ("ao_samples", C.c_int32), ("ao_maxdist", C.c_double), ("seed", C.c_uint64),
                ("view_id", C.c_uint32), ("precision", C.c_int32), ("background", C.c_float * 3),
                ("aa_samples", C.c_int32), ("specular", C.c_double), ("shininess", C.c_double),
                ("max_layers", C.c_int32)]


class Frame(C.Structure):
    _fields_ = [("rgb", C.c_void_p), ("hit_id", C.c_void_p), ("ao_mask", C.c_void_p),
                ("light_mask", C.c_void_p), ("stats", C.c_void_p)]


class Tune(C.Structure):
    _fields_ = [("tile_w", C.c_int32), ("banks", C.c_int32), ("waves_per_cu", C.c_int32),
                ("refill_below", C.c_int32), ("count_ops", C.c_int32),
                ("accel", C.c_int32), ("stripe", C.c_int32)]

    def as_dict(self):
        return {n: int(getattr(self, n)) for n, _ in self._fields_}


_lib = None


def lib():
    """Load libtr.so (raises if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libtr.so is not built (%s); run paper_0801_1500_amd/build.py" % LIB_PATH)
    # torch's HIP runtime must be the one libtr.so binds to (same soname), so
    # that torch streams and device memory are valid inside the library:
    # load torch first.
    import torch  # noqa: F401
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, st = C.c_void_p, C.c_int32, C.c_int64, C.c_int
    sig = {
        "tr_scene_build": ([C.POINTER(SceneDesc), vp, C.POINTER(vp)], st),
        "tr_scene_rebuild": ([vp, C.c_double, vp], st),
        "tr_scene_set_max_skip": ([vp, C.c_int32, vp], st),
        "tr_scene_build_bvh": ([vp, vp], st),
        "tr_scene_bvh_nodes": ([vp, vp, C.POINTER(i64), C.POINTER(C.c_int32), vp], st),
        "tr_scene_footprint": ([vp, C.POINTER(C.c_size_t)], st),
        "tr_scene_grid_info": ([vp, vp, vp, vp, C.POINTER(i64)], st),
        "tr_scene_grid_arrays": ([vp, vp, vp, vp], st),
        "tr_scene_walk_arrays": ([vp, vp, vp, C.POINTER(i64), vp], st),
        "tr_frame_quantize": ([vp, i64, vp, vp], st),
        "tr_frame_encode_tga": ([vp, i32, i32, vp, i64, C.POINTER(i64), vp], st),
        "tr_tga_max_bytes": ([i32, i32], i64),
        "tr_scene_save": ([vp, C.c_char_p, vp], st),
        "tr_scene_load": ([C.c_char_p, vp, C.POINTER(vp)], st),
        "tr_scene_destroy": ([vp], None),
        "tr_render": ([vp, C.POINTER(Camera), C.POINTER(Params), C.POINTER(Frame), vp], st),
        "tr_render_tuned": ([vp, C.POINTER(Camera), C.POINTER(Params), C.POINTER(Frame),
                             C.POINTER(Tune), vp], st),
        "tr_render_batch": ([i32, vp, vp, vp, vp, vp], st),
        "tr_render_batch_tiles": ([i32, vp, vp, vp, vp, vp, vp, C.POINTER(Tune), vp], st),
        "tr_render_batch_noalloc": ([i32, vp, vp, vp, vp, C.POINTER(Tune), vp], st),
        "tr_tile_count": ([i32, i32, i32], i64),
        "tr_frame_footprint": ([C.POINTER(Camera), C.POINTER(Params), C.c_uint32], C.c_size_t),
        "tr_graph_create": ([i32, vp, vp, vp, vp, C.POINTER(Tune), vp, C.POINTER(vp)], st),
        "tr_graph_update": ([vp, vp, vp, vp], st),
        "tr_graph_launch": ([vp, vp], st),
        "tr_graph_destroy": ([vp], None),
        "tr_graph_autotune": ([vp, i32, vp, vp, C.POINTER(Tune), C.POINTER(C.c_double),
                               C.POINTER(C.c_double)], st),
        "tr_autotune": ([vp, C.POINTER(Camera), C.POINTER(Params), vp, C.POINTER(Tune),
                         C.POINTER(C.c_double)], st),
        "tr_default_tune": ([C.POINTER(Tune)], st),
        "tr_measure_fp32_peak": ([vp, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                  C.POINTER(i32)], st),
        "tr_debug_philox": ([i64, vp, vp, vp, vp], st),
        "tr_debug_ao_dirs": ([i64, vp, vp, vp, C.c_uint32, C.c_uint64, vp, vp], st),
        "tr_last_error": ([], C.c_char_p),
        "tr_abi_version": ([], i32),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _lib = L
    return L


def _check(status: int):
    if status != TR_OK:
        raise TRError(status, lib().tr_last_error().decode(errors="replace"))


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("no GPU: the ray caster runs only on the HIP device")
    return torch


def _torch_stream(stream):
    """A torch stream object for a torch stream, a raw hipStream_t or None."""
    torch = _torch()
    if stream is None:
        return torch.cuda.current_stream()
    if hasattr(stream, "cuda_stream"):
        return stream
    return torch.cuda.ExternalStream(int(stream))


def _stream(stream) -> Optional[int]:
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else stream


def make_camera(cam) -> Camera:
    return Camera((C.c_double * 3)(*map(float, cam.eye)), (C.c_double * 3)(*map(float, cam.lookat)),
                  (C.c_double * 3)(*map(float, cam.up)), float(cam.fovy_deg), int(cam.width),
                  int(cam.height))


def make_params(p, precision="fp32_resolve") -> Params:
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    return Params(float(p.light_rescale), float(p.skylight), int(p.ao_samples),
                  float(p.ao_maxdist), int(p.seed) & ((1 << 64) - 1), int(p.view_id) & 0xFFFFFFFF,
                  prec, (C.c_float * 3)(*map(float, p.background)),
                  int(getattr(p, "aa_samples", 1)), float(getattr(p, "specular", 0.0)),
                  float(getattr(p, "shininess", 20.0)), int(getattr(p, "max_layers", 0)))


def make_tune(tune) -> Optional[Tune]:
    if tune is None:
        return None
    if isinstance(tune, Tune):
        return tune
    return Tune(int(tune.get("tile_w", 0)), int(tune.get("banks", 0)),
                int(tune.get("waves_per_cu", 0)), int(tune.get("refill_below", 0)),
                int(tune.get("count_ops", 0)),
                int(tune.get("accel", 0)),
                int(tune.get("stripe", 0)))


class Scene:
    """A scene resident on the current GPU (arrays + uniform grid)."""

    def __init__(self, scene, cells_per_prim: float = 0.0, stream=None, max_skip: int = 0):
        f64 = lambda a: np.ascontiguousarray(a, dtype=np.float64)
        f32 = lambda a: np.ascontiguousarray(a, dtype=np.float32)
        arrs = [f64(scene.sph_center), f64(scene.sph_radius), f32(scene.sph_rgb),
                f64(scene.cyl_a), f64(scene.cyl_b), f64(scene.cyl_radius), f32(scene.cyl_rgb),
                f64(scene.light_dir), f64(scene.light_rgb)]
        ops = [getattr(scene, k, None) for k in ("sph_opacity", "cyl_opacity", "tri_opacity")]
        ops = [None if o is None else f32(o).reshape(-1) for o in ops]
        tv = getattr(scene, "tri_v", None)
        tv = np.zeros((0, 3, 3)) if tv is None else f64(tv).reshape(-1, 3, 3)
        trgb = getattr(scene, "tri_rgb", None)
        trgb = np.zeros((0, 3), np.float32) if trgb is None else f32(trgb).reshape(-1, 3)
        n_t = int(tv.shape[0])
        arrs += [o if o is not None else np.zeros(0, np.float32) for o in ops[:2]]
        arrs += [np.ascontiguousarray(tv[:, q, :]) for q in range(3)] + [trgb]
        arrs += [ops[2] if ops[2] is not None else np.zeros(0, np.float32)]
        p = [a.ctypes.data if a.size else None for a in arrs]
        desc = SceneDesc(int(arrs[1].shape[0]), p[0], p[1], p[2], int(arrs[5].shape[0]), p[3],
                         p[4], p[5], p[6], int(arrs[7].reshape(-1, 3).shape[0]), p[7], p[8],
                         float(cells_per_prim), p[9], p[10], n_t, p[11], p[12], p[13], p[14],
                         p[15], int(max_skip))
        h = C.c_void_p()
        _check(lib().tr_scene_build(C.byref(desc), _stream(stream), C.byref(h)))
        self.handle = h
        self.n_spheres = int(arrs[1].shape[0])
        self.n_cylinders = int(arrs[5].shape[0])
        self.n_lights = int(arrs[7].reshape(-1, 3).shape[0])
        self.n_triangles = n_t

    @property
    def n_prims(self):
        return self.n_spheres + self.n_cylinders + self.n_triangles

    def save(self, path: str, stream=None):
        """Write the scene as a binary scene file (tr_scene_save)."""
        _check(lib().tr_scene_save(self.handle, os.fsencode(path), _stream(stream)))

    @classmethod
    def load(cls, path: str, stream=None) -> "Scene":
        """Build a scene from a binary scene file (tr_scene_load)."""
        import struct
        with open(path, "rb") as f:
            head = f.read(40)
        h = C.c_void_p()
        _check(lib().tr_scene_load(os.fsencode(path), _stream(stream), C.byref(h)))
        self = cls.__new__(cls)
        self.handle = h
        self.n_spheres, self.n_cylinders, self.n_lights, flags = struct.unpack_from("<qqii", head, 8)
        self.n_triangles = 0
        if flags & 2:  # triangle count right after the light arrays
            pad8 = lambda b: (b + 7) & ~7
            ns, nc, nl = self.n_spheres, self.n_cylinders, self.n_lights
            at = (40 + pad8(24 * ns) + pad8(8 * ns) + pad8(12 * ns) + 2 * pad8(24 * nc) +
                  pad8(8 * nc) + pad8(12 * nc) + 2 * pad8(24 * nl))
            with open(path, "rb") as f:
                f.seek(at)
                self.n_triangles = struct.unpack("<q", f.read(8))[0]
        return self

    def build_bvh(self, stream=None):
        """Linear BVH for the BVH walk (tune accel=1)."""
        _check(lib().tr_scene_build_bvh(self.handle, _stream(stream)))

    def bvh_nodes(self, stream=None):
        """BVH records: float32 [n_nodes, 16] (see tr_scene_bvh_nodes)."""
        n = C.c_int64(0)
        _check(lib().tr_scene_bvh_nodes(self.handle, None, C.byref(n), None, _stream(stream)))
        out = np.zeros((max(n.value, 0), 16), dtype=np.float32)
        if n.value > 0:
            _check(lib().tr_scene_bvh_nodes(self.handle, out.ctypes.data, C.byref(n), None,
                                            _stream(stream)))
        return out

    def bvh_depth(self) -> int:
        """Internal nodes on the BVH's longest root-to-leaf path (0: none built)."""
        n, d = C.c_int64(0), C.c_int32(0)
        _check(lib().tr_scene_bvh_nodes(self.handle, None, C.byref(n), C.byref(d), None))
        return d.value

    def set_max_skip(self, max_skip: int, stream=None):
        """Empty-space skipping cap (1 = plain 3D-DDA); rebuilds the grid."""
        _check(lib().tr_scene_set_max_skip(self.handle, int(max_skip), _stream(stream)))

    def rebuild(self, cells_per_prim: float = 0.0, stream=None):
        _check(lib().tr_scene_rebuild(self.handle, float(cells_per_prim), _stream(stream)))

    def footprint(self) -> int:
        b = C.c_size_t()
        _check(lib().tr_scene_footprint(self.handle, C.byref(b)))
        return int(b.value)

    def grid_info(self):
        lo = np.zeros(3); hi = np.zeros(3); res = np.zeros(3, dtype=np.int32)
        n = C.c_int64()
        _check(lib().tr_scene_grid_info(self.handle, lo.ctypes.data, hi.ctypes.data,
                                        res.ctypes.data, C.byref(n)))
        return lo, hi, res, int(n.value)

    def grid_arrays(self, stream=None):
        lo, hi, res, n_refs = self.grid_info()
        n_cells = int(res[0]) * int(res[1]) * int(res[2])
        cb = np.zeros(n_cells + 1, dtype=np.uint32)
        refs = np.zeros(max(n_refs, 1), dtype=np.uint32)
        _check(lib().tr_scene_grid_arrays(self.handle, cb.ctypes.data, refs.ctypes.data,
                                          _stream(stream)))
        return cb, refs[:n_refs]

    def walk_arrays(self, stream=None):
        """(cellinfo [n_cells, 2], wrefs) of the FP32 walk (see tr.h)."""
        lo, hi, res, n_refs = self.grid_info()
        n_cells = int(res[0]) * int(res[1]) * int(res[2])
        n = C.c_int64(0)
        _check(lib().tr_scene_walk_arrays(self.handle, None, None, C.byref(n), _stream(stream)))
        ci = np.zeros((n_cells, 2), dtype=np.int32)
        wr = np.zeros(max(n.value, 1), dtype=np.uint32)
        _check(lib().tr_scene_walk_arrays(self.handle, ci.ctypes.data, wr.ctypes.data, C.byref(n),
                                          _stream(stream)))
        return ci, wr[:n.value]

    def destroy(self):
        if getattr(self, "handle", None):
            lib().tr_scene_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def alloc_frame(cam, outputs: Sequence[str] = ("rgb",), stats: bool = False, device=None) -> dict:
    torch = _torch()
    dev = device if device is not None else torch.device("cuda", torch.cuda.current_device())
    H, W = int(cam.height), int(cam.width)
    out = {}
    if "rgb" in outputs:
        out["rgb"] = torch.empty((H, W, 3), dtype=torch.float32, device=dev)
    if "hit_id" in outputs:
        out["hit_id"] = torch.empty((H, W), dtype=torch.int32, device=dev)
    if "ao_mask" in outputs:
        out["ao_mask"] = torch.empty((H, W), dtype=torch.int32, device=dev)
    if "light_mask" in outputs:
        out["light_mask"] = torch.empty((H, W), dtype=torch.uint8, device=dev)
    if stats:
        out["stats"] = torch.zeros(STAT_COUNT, dtype=torch.int64, device=dev)
    return out


# Element type and values per pixel of each frame buffer (tr.h, tr_frame);
# ao_mask holds uint32 bits and may come as int32.
_FRAME_FIELDS = {"rgb": (("float32",), 3), "hit_id": (("int32",), 1),
                 "ao_mask": (("int32", "uint32"), 1), "light_mask": (("uint8",), 1)}


def frame_struct(frame: dict, cam=None) -> Frame:
    """The tr_frame of a dict of device tensors.  With the camera, every
    buffer present is checked before its address reaches the library: a CUDA
    tensor on the current device, contiguous, of the element type tr.h names
    and with W * H (* 3 for rgb) elements; stats needs STAT_COUNT 64-bit
    integers.  ValueError otherwise."""
    if cam is not None:
        import torch
        n_px = int(cam.width) * int(cam.height)
        want = {k: (dt, n_px * per) for k, (dt, per) in _FRAME_FIELDS.items()}
        want["stats"] = (("int64", "uint64"), STAT_COUNT)
        for k, v in frame.items():
            if v is None or k not in want:
                continue
            dts, numel = want[k]
            if str(v.dtype).replace("torch.", "") not in dts:
                raise ValueError("frame[%r]: dtype %s, expected %s" % (k, v.dtype, " or ".join(dts)))
            if not v.is_contiguous():
                raise ValueError("frame[%r] must be contiguous" % k)
            if v.numel() != numel:
                raise ValueError("frame[%r] has %d elements, expected %d" % (k, v.numel(), numel))
        for k, v in frame.items():
            if v is not None and k in want and (
                    not v.is_cuda or v.device.index != torch.cuda.current_device()):
                raise ValueError("frame[%r] must be a CUDA tensor on the current device" % k)
    g = lambda k: frame[k].data_ptr() if frame.get(k) is not None else None
    return Frame(g("rgb"), g("hit_id"), g("ao_mask"), g("light_mask"), g("stats"))


def quantize_rgb8(values, out=None, stream=None):
    """8-bit image of float values on the GPU (tr_frame_quantize):
    floor(clamp(v, 0, 1) * 255 + 1/2), NaN -> 0.  values: a CUDA float32
    tensor (e.g. a frame's rgb [H, W, 3]); returns a uint8 tensor of the same
    shape (out, if given, must be one)."""
    torch = _torch()
    if values.dtype != torch.float32 or not values.is_cuda:
        raise TypeError("values must be a CUDA float32 tensor")
    s = _torch_stream(stream)
    # allocations are made on the stream that uses them, so the caching
    # allocator does not hand their blocks out while that stream's work is
    # pending
    with torch.cuda.stream(s):
        v = values.contiguous()
        if out is None:
            out = torch.empty(v.shape, dtype=torch.uint8, device=v.device)
        elif out.dtype != torch.uint8 or out.numel() != v.numel() or not out.is_contiguous():
            raise ValueError("out must be a contiguous uint8 tensor of values' size")
    if v is not values:
        v.record_stream(s)
    _check(lib().tr_frame_quantize(v.data_ptr(), v.numel(), out.data_ptr(), _stream(s)))
    return out


def frame_to_host_rgb8(frame: dict, host=None, stream=None):
    """Quantise frame["rgb"] on the GPU and start its copy into pinned host
    memory (asynchronous on the stream).  Returns (host uint8 [H, W, 3],
    event): wait on the event before reading host."""
    torch = _torch()
    s = _torch_stream(stream)
    dev = quantize_rgb8(frame["rgb"], stream=s)
    if host is None:
        host = torch.empty(dev.shape, dtype=torch.uint8, pin_memory=True)
    with torch.cuda.stream(s):
        host.copy_(dev, non_blocking=True)
        ev = torch.cuda.Event()
        ev.record(s)
    # the 8-bit device image is freed on return: its block must not be
    # reused before the copy on s has read it
    dev.record_stream(s)
    return host, ev


def encode_ppm(rgb8) -> bytes:
    """Binary PPM (P6) of an 8-bit RGB image [H, W, 3] in host memory."""
    a = rgb8.numpy() if hasattr(rgb8, "numpy") else np.asarray(rgb8)
    if a.dtype != np.uint8 or a.ndim != 3 or a.shape[2] != 3:
        raise ValueError("rgb8 must be uint8 [H, W, 3]")
    return b"P6\n%d %d\n255\n" % (a.shape[1], a.shape[0]) + np.ascontiguousarray(a).tobytes()


def render_into(scene: Scene, cam, params, frame: dict, precision="fp32_resolve", tune=None,
                stream=None):
    c = make_camera(cam)
    p = make_params(params, precision)
    f = frame_struct(frame, cam)
    t = make_tune(tune)
    if t is None:
        _check(lib().tr_render(scene.handle, C.byref(c), C.byref(p), C.byref(f), _stream(stream)))
    else:
        _check(lib().tr_render_tuned(scene.handle, C.byref(c), C.byref(p), C.byref(f), C.byref(t),
                                     _stream(stream)))
    return frame


def render(scene: Scene, cam, params, precision="fp32_resolve",
           outputs: Sequence[str] = ("rgb", "hit_id", "ao_mask", "light_mask"), stats=False,
           tune=None, stream=None) -> dict:
    """Render one frame; returns device tensors (rgb [H,W,3] f32, hit_id
    [H,W] i32, ao_mask [H,W] (uint32 bits in an int32 tensor), light_mask
    [H,W] u8, stats [STAT_COUNT] i64)."""
    outputs = list(outputs)
    if "ao_mask" in outputs and params.ao_samples > 32:
        outputs.remove("ao_mask")
    frame = alloc_frame(cam, outputs, stats)
    return render_into(scene, cam, params, frame, precision, tune, stream)


def _arrays(scenes, cams, params, frames, precision):
    n = len(scenes)
    sc = (C.c_void_p * n)(*[s.handle.value for s in scenes])
    cm = (Camera * n)(*[make_camera(c) for c in cams])
    if isinstance(precision, (list, tuple)):
        pr = (Params * n)(*[make_params(p, q) for p, q in zip(params, precision)])
    else:
        pr = (Params * n)(*[make_params(p, precision) for p in params])
    fr = (Frame * n)(*[frame_struct(f, c) for f, c in zip(frames, cams)])
    return n, sc, cm, pr, fr


def render_batch_into(scenes: List[Scene], cams, params, frames: List[dict],
                      precision="fp32_resolve", stream=None):
    n, sc, cm, pr, fr = _arrays(scenes, cams, params, frames, precision)
    _check(lib().tr_render_batch(n, sc, cm, pr, fr, _stream(stream)))
    return frames


NOALLOC_MAX_JOBS = 16  # TR_NOALLOC_MAX_JOBS


def render_batch_noalloc_into(scenes: List[Scene], cams, params, frames: List[dict],
                              precision="fp32_resolve", tune=None, stream=None):
    """tr_render_batch_noalloc: the batch render that allocates nothing (job
    table in the library's static device memory; at most NOALLOC_MAX_JOBS
    jobs, no antialiasing)."""
    n, sc, cm, pr, fr = _arrays(scenes, cams, params, frames, precision)
    t = make_tune(tune)
    _check(lib().tr_render_batch_noalloc(n, sc, cm, pr, fr, C.byref(t) if t is not None else None,
                                         _stream(stream)))
    return frames


def render_batch_tiles_into(scenes, cams, params, frames, tile_begin, tile_end,
                            precision="fp32_resolve", tune=None, stream=None):
    n, sc, cm, pr, fr = _arrays(scenes, cams, params, frames, precision)
    tb = (C.c_int64 * n)(*map(int, tile_begin))
    te = (C.c_int64 * n)(*map(int, tile_end))
    t = make_tune(tune)
    _check(lib().tr_render_batch_tiles(n, sc, cm, pr, fr, tb, te,
                                       C.byref(t) if t is not None else None, _stream(stream)))
    return frames


def tga_max_bytes(width: int, height: int) -> int:
    """Bytes that always hold the Targa file of a width x height image."""
    n = lib().tr_tga_max_bytes(int(width), int(height))
    if n < 0:
        raise ValueError("Targa width and height must be 1..65535")
    return int(n)


def encode_tga(rgb8, out=None, stream=None):
    """Run-length Targa file of an 8-bit RGB image, on the GPU
    (tr_frame_encode_tga).  rgb8: a contiguous CUDA uint8 tensor [H, W, 3]
    (e.g. quantize_rgb8's output); out: optional CUDA uint8 buffer.  Returns
    a CUDA uint8 tensor holding exactly the file's bytes (a view of out when
    given), written on the stream."""
    torch = _torch()
    if rgb8.dtype != torch.uint8 or not rgb8.is_cuda or rgb8.dim() != 3 or rgb8.shape[2] != 3:
        raise TypeError("rgb8 must be a CUDA uint8 tensor [H, W, 3]")
    rgb8 = rgb8.contiguous()
    H, W = int(rgb8.shape[0]), int(rgb8.shape[1])
    if out is None:
        out = torch.empty(tga_max_bytes(W, H), dtype=torch.uint8, device=rgb8.device)
    n = C.c_int64(0)
    _check(lib().tr_frame_encode_tga(rgb8.data_ptr(), W, H, out.data_ptr(), out.numel(),
                                     C.byref(n), _stream(stream)))
    return out[:n.value]


def write_tga(frame, path: str, stream=None) -> int:
    """Write a rendered frame (a frame dict or its float rgb tensor) as a
    run-length Targa file: 8-bit conversion and encoding on the GPU, then
    the file's bytes are copied to host memory and written.  Returns the
    file size in bytes."""
    torch = _torch()
    rgb = frame["rgb"] if isinstance(frame, dict) else frame
    tga = encode_tga(quantize_rgb8(rgb, stream=stream), stream=stream)
    host = torch.empty(tga.numel(), dtype=torch.uint8, pin_memory=True)
    s = stream if stream is not None else torch.cuda.current_stream()
    with torch.cuda.stream(s):
        host.copy_(tga, non_blocking=True)
    s.synchronize()
    with open(path, "wb") as f:
        f.write(host.numpy().tobytes())
    return int(tga.numel())


def tile_count(width: int, height: int, tile_w: int = 0) -> int:
    n = lib().tr_tile_count(int(width), int(height), int(tile_w))
    if n < 0:
        raise ValueError("invalid tile arguments")
    return int(n)


def frame_footprint(cam, params, flags: int = 1) -> int:
    c = make_camera(cam)
    p = make_params(params)
    return int(lib().tr_frame_footprint(C.byref(c), C.byref(p), int(flags)))


class Graph:
    """A captured batch render (hipGraph) whose cameras/params can be
    updated between replays without re-capture."""

    def __init__(self, scenes, cams, params, frames, precision="fp32_resolve", tune=None,
                 stream=None):
        n, sc, cm, pr, fr = _arrays(scenes, cams, params, frames, precision)
        self._keep = (scenes, frames)
        self.precision = precision
        t = make_tune(tune)
        h = C.c_void_p()
        _check(lib().tr_graph_create(n, sc, cm, pr, fr, C.byref(t) if t is not None else None,
                                     _stream(stream), C.byref(h)))
        self.handle = h
        self.n = n

    def update(self, cams=None, params=None, stream=None):
        cm = (Camera * self.n)(*[make_camera(c) for c in cams]) if cams is not None else None
        pr = ((Params * self.n)(*[make_params(p, self.precision) for p in params])
              if params is not None else None)
        _check(lib().tr_graph_update(self.handle, cm, pr, _stream(stream)))

    def launch(self, stream=None):
        _check(lib().tr_graph_launch(self.handle, _stream(stream)))

    def autotune(self, lambdas=(), stream=None):
        """Tune the graph on itself: its scenes' grid density over `lambdas`
        (cells per primitive), then the launch shape.  Returns (tune dict,
        chosen density or 0.0 when the scenes kept their own, ms per replay);
        the graph and its scenes keep the choice."""
        lam = (C.c_double * max(len(lambdas), 1))(*[float(x) for x in lambdas])
        t, bl, ms = Tune(), C.c_double(), C.c_double()
        _check(lib().tr_graph_autotune(self.handle, len(lambdas), lam, _stream(stream),
                                       C.byref(t), C.byref(bl), C.byref(ms)))
        return t.as_dict(), float(bl.value), float(ms.value)

    def destroy(self):
        if getattr(self, "handle", None):
            lib().tr_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def autotune(scene: Scene, cam, params, precision="fp32_resolve", stream=None):
    c = make_camera(cam)
    p = make_params(params, precision)
    t = Tune()
    ms = C.c_double()
    _check(lib().tr_autotune(scene.handle, C.byref(c), C.byref(p), _stream(stream), C.byref(t),
                             C.byref(ms)))
    return t.as_dict(), float(ms.value)


def default_tune() -> dict:
    t = Tune()
    _check(lib().tr_default_tune(C.byref(t)))
    return t.as_dict()


def measure_fp32_peak(stream=None) -> dict:
    """Measured non-packed FP32 FMA rate of the current device (TFLOP/s),
    with the device's reported peak clock (MHz) and compute units."""
    tf, mhz, cus = C.c_double(), C.c_double(), C.c_int32()
    _check(lib().tr_measure_fp32_peak(_stream(stream), C.byref(tf), C.byref(mhz), C.byref(cus)))
    return {"tflops": float(tf.value), "clock_mhz": float(mhz.value), "n_cus": int(cus.value)}


def debug_philox(ctr, key, stream=None):
    """ctr [n,4] and key [n,2] uint32-valued int64/int32 device tensors."""
    torch = _torch()
    ctr = ctr.to(torch.int32).contiguous()
    key = key.to(torch.int32).contiguous()
    out = torch.empty_like(ctr)
    _check(lib().tr_debug_philox(int(ctr.shape[0]), ctr.data_ptr(), key.data_ptr(),
                                 out.data_ptr(), _stream(stream)))
    return out


def debug_ao_dirs(normals, pix, sample, view_id: int, seed: int, stream=None):
    torch = _torch()
    normals = normals.to(torch.float32).contiguous()
    pix = pix.to(torch.int32).contiguous()
    sample = sample.to(torch.int32).contiguous()
    w = torch.empty_like(normals)
    _check(lib().tr_debug_ao_dirs(int(pix.shape[0]), normals.data_ptr(), pix.data_ptr(),
                                  sample.data_ptr(), int(view_id) & 0xFFFFFFFF,
                                  int(seed) & ((1 << 64) - 1), w.data_ptr(), _stream(stream)))
    return w


def abi_version() -> int:
    return int(lib().tr_abi_version())
