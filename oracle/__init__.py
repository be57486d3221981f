"""Python access to the FP64 CPU oracle (oracle.c).

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
benchmark's CPU-baseline leg may import this package; the product path never
does.  It imports nothing from the HIP implementation.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2 -ffp-contract=off, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-fPIC", "-shared", "-D_GNU_SOURCE", "-Wall", "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


class Counters(C.Structure):
    _fields_ = [(n, C.c_uint64) for n in (
        "pixels", "primary_rays", "hit_pixels", "shadow_rays", "ao_rays", "rays_traced",
        "cells", "sph_tests", "sph_hits", "cyl_tests", "cyl_hits", "tri_tests", "tri_hits")]

    def as_dict(self):
        return {n: int(getattr(self, n)) for n, _ in self._fields_}


class _Scene(C.Structure):
    _fields_ = [
        ("n_spheres", C.c_int64), ("sph_center", C.c_void_p), ("sph_radius", C.c_void_p),
        ("sph_rgb", C.c_void_p),
        ("n_cylinders", C.c_int64), ("cyl_a", C.c_void_p), ("cyl_b", C.c_void_p),
        ("cyl_radius", C.c_void_p), ("cyl_rgb", C.c_void_p),
        ("n_lights", C.c_int32), ("light_dir", C.c_void_p), ("light_rgb", C.c_void_p),
        ("sph_opacity", C.c_void_p), ("cyl_opacity", C.c_void_p),
        ("n_triangles", C.c_int64), ("tri_v0", C.c_void_p), ("tri_v1", C.c_void_p),
        ("tri_v2", C.c_void_p), ("tri_rgb", C.c_void_p), ("tri_opacity", C.c_void_p)]


class _Camera(C.Structure):
    _fields_ = [("eye", C.c_double * 3), ("lookat", C.c_double * 3), ("up", C.c_double * 3),
                ("fovy_deg", C.c_double), ("width", C.c_int32), ("height", C.c_int32)]


class _Params(C.Structure):
    _fields_ = [("light_rescale", C.c_double), ("skylight", C.c_double),
                ("ao_samples", C.c_int32), ("ao_maxdist", C.c_double), ("seed", C.c_uint64),
                ("view_id", C.c_uint32), ("background", C.c_double * 3),
                ("aa_samples", C.c_int32), ("specular", C.c_double), ("shininess", C.c_double),
                ("max_layers", C.c_int32)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = C.CDLL(_LIB)
        vp, i64, i32, dbl = C.c_void_p, C.c_int64, C.c_int32, C.c_double
        L.or_philox4x32_10.argtypes = [vp, vp, vp]
        L.or_philox_many.argtypes = [i64, vp, vp, vp]
        L.or_ao_uniforms.argtypes = [C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint64,
                                     C.POINTER(dbl), C.POINTER(dbl)]
        L.or_ao_uniforms_aa.argtypes = [C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32,
                                        C.c_uint64, C.POINTER(dbl), C.POINTER(dbl)]
        L.or_aa_offset.argtypes = [C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint64,
                                   C.POINTER(dbl), C.POINTER(dbl)]
        L.or_camera_ray_at.argtypes = [C.POINTER(_Camera), dbl, dbl, vp, vp]
        L.or_ao_direction.argtypes = [vp, dbl, dbl, vp]
        L.or_camera_ray.argtypes = [C.POINTER(_Camera), i32, i32, vp, vp]
        L.or_hit_sphere.argtypes = [vp, dbl, vp, vp, dbl, dbl, C.POINTER(dbl)]
        L.or_hit_sphere.restype = C.c_int
        L.or_hit_cylinder.argtypes = [vp, vp, dbl, vp, vp, dbl, dbl, C.POINTER(dbl)]
        L.or_hit_cylinder.restype = C.c_int
        L.or_hit_triangle.argtypes = [vp, vp, vp, vp, vp, dbl, dbl, C.POINTER(dbl)]
        L.or_hit_triangle.restype = C.c_int
        L.or_normal.argtypes = [C.POINTER(_Scene), i64, vp, vp, dbl, vp]
        L.or_grid_new.argtypes = [C.POINTER(_Scene), dbl]
        L.or_grid_new.restype = vp
        L.or_grid_free.argtypes = [vp]
        L.or_grid_info.argtypes = [vp, vp, vp, vp, C.POINTER(i64)]
        L.or_grid_arrays.argtypes = [vp, vp, vp]
        L.or_trace.argtypes = [C.POINTER(_Scene), vp, vp, vp, dbl, dbl, i64, C.c_int,
                               C.POINTER(dbl), C.POINTER(i64), C.POINTER(Counters)]
        L.or_trace.restype = C.c_int
        L.or_trace_list.argtypes = [C.POINTER(_Scene), vp, i64, vp, vp, dbl, dbl, i64, C.c_int,
                                    C.POINTER(dbl), C.POINTER(i64)]
        L.or_trace_list.restype = C.c_int
        L.or_render.argtypes = [C.POINTER(_Scene), C.POINTER(_Camera), C.POINTER(_Params), vp,
                                i64, vp, vp, vp, vp, vp, vp, vp, C.POINTER(Counters), i32]
        L.or_render.restype = C.c_int
        L.or_max_threads.restype = C.c_int32
        L.or_quantize_rgb8.argtypes = [i64, vp, vp]
        L.or_tga_encode.argtypes = [vp, C.c_int32, C.c_int32, vp, i64]
        L.or_tga_encode.restype = i64
        _lib = L
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data


class OScene:
    """Holds a scenegen.Scene's arrays (contiguous, right dtypes) and the C
    struct pointing at them."""

    def __init__(self, scene):
        f64 = lambda a: np.ascontiguousarray(a, dtype=np.float64)
        f32 = lambda a: np.ascontiguousarray(a, dtype=np.float32)
        self.arrays = dict(
            sph_center=f64(scene.sph_center).reshape(-1, 3), sph_radius=f64(scene.sph_radius),
            sph_rgb=f32(scene.sph_rgb).reshape(-1, 3),
            cyl_a=f64(scene.cyl_a).reshape(-1, 3), cyl_b=f64(scene.cyl_b).reshape(-1, 3),
            cyl_radius=f64(scene.cyl_radius), cyl_rgb=f32(scene.cyl_rgb).reshape(-1, 3),
            light_dir=f64(scene.light_dir).reshape(-1, 3),
            light_rgb=f64(scene.light_rgb).reshape(-1, 3))
        for key in ("sph_opacity", "cyl_opacity", "tri_opacity"):
            v = getattr(scene, key, None)
            self.arrays[key] = None if v is None else f32(v).reshape(-1)
        tv = getattr(scene, "tri_v", None)  # [n_t, 3, 3]
        tv = np.zeros((0, 3, 3)) if tv is None else f64(tv).reshape(-1, 3, 3)
        for q in range(3):
            self.arrays["tri_v%d" % q] = np.ascontiguousarray(tv[:, q, :])
        trgb = getattr(scene, "tri_rgb", None)
        self.arrays["tri_rgb"] = (np.zeros((0, 3), np.float32) if trgb is None
                                  else f32(trgb).reshape(-1, 3))
        self.n_triangles = tv.shape[0]
        a = self.arrays
        self.n_spheres = a["sph_radius"].shape[0]
        self.n_cylinders = a["cyl_radius"].shape[0]
        self.c = _Scene(self.n_spheres, _ptr(a["sph_center"]), _ptr(a["sph_radius"]),
                        _ptr(a["sph_rgb"]), self.n_cylinders, _ptr(a["cyl_a"]), _ptr(a["cyl_b"]),
                        _ptr(a["cyl_radius"]), _ptr(a["cyl_rgb"]), a["light_dir"].shape[0],
                        _ptr(a["light_dir"]), _ptr(a["light_rgb"]),
                        _ptr(a["sph_opacity"]), _ptr(a["cyl_opacity"]), self.n_triangles,
                        _ptr(a["tri_v0"]), _ptr(a["tri_v1"]), _ptr(a["tri_v2"]),
                        _ptr(a["tri_rgb"]), _ptr(a["tri_opacity"]))


def _as_oscene(scene) -> OScene:
    return scene if isinstance(scene, OScene) else OScene(scene)


def _camera(cam) -> _Camera:
    return _Camera((C.c_double * 3)(*cam.eye), (C.c_double * 3)(*cam.lookat),
                   (C.c_double * 3)(*cam.up), float(cam.fovy_deg), int(cam.width),
                   int(cam.height))


def _params(p) -> _Params:
    return _Params(float(p.light_rescale), float(p.skylight), int(p.ao_samples),
                   float(p.ao_maxdist), int(p.seed) & ((1 << 64) - 1), int(p.view_id),
                   (C.c_double * 3)(*[float(x) for x in p.background]),
                   int(getattr(p, "aa_samples", 1)), float(getattr(p, "specular", 0.0)),
                   float(getattr(p, "shininess", 20.0)), int(getattr(p, "max_layers", 0)))


class Grid:
    """The oracle's own uniform grid over a scene (definition in oracle.c)."""

    def __init__(self, scene, cells_per_prim: float = 4.0):
        self.scene = _as_oscene(scene)
        self.handle = lib().or_grid_new(C.byref(self.scene.c), float(cells_per_prim))
        if not self.handle:
            raise MemoryError("or_grid_new failed")

    def __del__(self):
        if getattr(self, "handle", None):
            lib().or_grid_free(self.handle)
            self.handle = None

    def info(self):
        lo = np.zeros(3); hi = np.zeros(3); res = np.zeros(3, dtype=np.int32)
        n = C.c_int64()
        lib().or_grid_info(self.handle, _ptr(lo), _ptr(hi), _ptr(res), C.byref(n))
        return lo, hi, res, int(n.value)

    def arrays(self):
        lo, hi, res, n_refs = self.info()
        n_cells = int(res[0]) * int(res[1]) * int(res[2])
        cb = np.zeros(n_cells + 1, dtype=np.uint32)
        refs = np.zeros(max(n_refs, 0), dtype=np.uint32)
        lib().or_grid_arrays(self.handle, _ptr(cb), _ptr(refs))
        return cb, refs


def philox(ctr: np.ndarray, key: np.ndarray) -> np.ndarray:
    ctr = np.ascontiguousarray(ctr, dtype=np.uint32).reshape(-1, 4)
    key = np.ascontiguousarray(key, dtype=np.uint32).reshape(-1, 2)
    out = np.zeros_like(ctr)
    lib().or_philox_many(ctr.shape[0], _ptr(ctr), _ptr(key), _ptr(out))
    return out


def ao_uniforms(pix: int, s: int, view_id: int, seed: int):
    u1 = C.c_double(); u2 = C.c_double()
    lib().or_ao_uniforms(pix, s, view_id, seed & ((1 << 64) - 1), C.byref(u1), C.byref(u2))
    return u1.value, u2.value


def ao_uniforms_aa(pix: int, s: int, view_id: int, a: int, seed: int):
    u1 = C.c_double(); u2 = C.c_double()
    lib().or_ao_uniforms_aa(pix, s, view_id, a, seed & ((1 << 64) - 1), C.byref(u1), C.byref(u2))
    return u1.value, u2.value


def aa_offset(pix: int, a: int, view_id: int, seed: int):
    ox = C.c_double(); oy = C.c_double()
    lib().or_aa_offset(pix, a, view_id, seed & ((1 << 64) - 1), C.byref(ox), C.byref(oy))
    return ox.value, oy.value


def ao_direction(n, u1: float, u2: float) -> np.ndarray:
    n = np.ascontiguousarray(n, dtype=np.float64)
    w = np.zeros(3)
    lib().or_ao_direction(_ptr(n), float(u1), float(u2), _ptr(w))
    return w


def camera_ray(cam, i: int, j: int):
    o = np.zeros(3); d = np.zeros(3)
    c = _camera(cam)
    lib().or_camera_ray(C.byref(c), int(i), int(j), _ptr(o), _ptr(d))
    return o, d


def camera_ray_at(cam, px: float, py: float):
    """Ray through image position (px, py) in pixel units (i + 1/2 = centre)."""
    o = np.zeros(3); d = np.zeros(3)
    c = _camera(cam)
    lib().or_camera_ray_at(C.byref(c), float(px), float(py), _ptr(o), _ptr(d))
    return o, d


def hit_sphere(c, r, o, d, tmin=0.0, tmax=math.inf):
    c, o, d = (np.ascontiguousarray(x, dtype=np.float64) for x in (c, o, d))
    t = C.c_double()
    h = lib().or_hit_sphere(_ptr(c), float(r), _ptr(o), _ptr(d), tmin, tmax, C.byref(t))
    return t.value if h else None


def hit_cylinder(a, b, rho, o, d, tmin=0.0, tmax=math.inf):
    a, b, o, d = (np.ascontiguousarray(x, dtype=np.float64) for x in (a, b, o, d))
    t = C.c_double()
    h = lib().or_hit_cylinder(_ptr(a), _ptr(b), float(rho), _ptr(o), _ptr(d), tmin, tmax,
                              C.byref(t))
    return t.value if h else None


def hit_triangle(v0, v1, v2, o, d, tmin=0.0, tmax=math.inf):
    v0, v1, v2, o, d = (np.ascontiguousarray(x, dtype=np.float64) for x in (v0, v1, v2, o, d))
    t = C.c_double()
    h = lib().or_hit_triangle(_ptr(v0), _ptr(v1), _ptr(v2), _ptr(o), _ptr(d), tmin, tmax,
                              C.byref(t))
    return t.value if h else None


def normal(scene, k: int, o, d, t: float) -> np.ndarray:
    sc = _as_oscene(scene)
    o, d = (np.ascontiguousarray(x, dtype=np.float64) for x in (o, d))
    n = np.zeros(3)
    lib().or_normal(C.byref(sc.c), int(k), _ptr(o), _ptr(d), float(t), _ptr(n))
    return n


def trace(scene, grid: Optional[Grid], o, d, tmin=0.0, tmax=math.inf, skip=-1, any_hit=False,
          counters: Optional[Counters] = None):
    sc = grid.scene if grid is not None else _as_oscene(scene)
    o, d = (np.ascontiguousarray(x, dtype=np.float64) for x in (o, d))
    t = C.c_double(); k = C.c_int64()
    h = lib().or_trace(C.byref(sc.c), grid.handle if grid else None, _ptr(o), _ptr(d),
                       float(tmin), float(tmax), int(skip), int(bool(any_hit)), C.byref(t),
                       C.byref(k), C.byref(counters) if counters is not None else None)
    return (t.value, int(k.value)) if h else (math.inf, -1)


def trace_list(scene, order, o, d, tmin=0.0, tmax=math.inf, skip=-1, any_hit=False):
    """Brute force over the primitive ids of `order`, visited in that order."""
    sc = _as_oscene(scene)
    order = np.ascontiguousarray(order, dtype=np.int64)
    n_all = scene.n_spheres + scene.n_cylinders + getattr(scene, "n_triangles", 0)
    if order.size and (order.min() < 0 or order.max() >= n_all):
        raise ValueError("primitive id out of range")
    o, d = (np.ascontiguousarray(x, dtype=np.float64) for x in (o, d))
    t = C.c_double(); k = C.c_int64()
    h = lib().or_trace_list(C.byref(sc.c), _ptr(order), int(order.size), _ptr(o), _ptr(d),
                            float(tmin), float(tmax), int(skip), int(bool(any_hit)), C.byref(t),
                            C.byref(k))
    return (t.value, int(k.value)) if h else (math.inf, -1)


def render(scene, cam, params, grid=None, pix: Optional[np.ndarray] = None,
           n_threads: int = 0) -> dict:
    """Render all pixels (pix None) or the listed pixel indices j*W+i.
    grid: None => brute force; a Grid => that grid; a number => build a grid
    with that many cells per primitive."""
    if grid is not None and not isinstance(grid, Grid):
        grid = Grid(scene, float(grid))
    sc = grid.scene if grid is not None else _as_oscene(scene)
    n = cam.width * cam.height if pix is None else int(len(pix))
    if pix is not None:
        pix = np.ascontiguousarray(pix, dtype=np.int64)
    out = dict(rgb=np.zeros((n, 3)), hit_id=np.zeros(n, dtype=np.int32),
               ao_mask=np.zeros(n, dtype=np.uint32), ao_occluded=np.zeros(n, dtype=np.int32),
               light_mask=np.zeros(n, dtype=np.uint8), t=np.zeros(n))
    cnt = Counters()
    c = _camera(cam)
    p = _params(params)
    rc = lib().or_render(C.byref(sc.c), C.byref(c), C.byref(p), grid.handle if grid else None,
                         n, _ptr(pix), _ptr(out["rgb"]), _ptr(out["hit_id"]),
                         _ptr(out["ao_mask"]), _ptr(out["ao_occluded"]),
                         _ptr(out["light_mask"]), _ptr(out["t"]), C.byref(cnt), int(n_threads))
    if rc != 0:
        raise ValueError("or_render rejected its arguments")
    out["counters"] = cnt.as_dict()
    if pix is None:
        H, W = cam.height, cam.width
        out["rgb"] = out["rgb"].reshape(H, W, 3)
        for key in ("hit_id", "ao_mask", "ao_occluded", "light_mask", "t"):
            out[key] = out[key].reshape(H, W)
    return out


def quantize_rgb8(values: np.ndarray) -> np.ndarray:
    """8-bit output of float values: floor(clamp(v, 0, 1) * 255 + 1/2), NaN -> 0."""
    v = np.ascontiguousarray(values, dtype=np.float32)
    out = np.empty(v.shape, dtype=np.uint8)
    lib().or_quantize_rgb8(v.size, v.ctypes.data, out.ctypes.data)
    return out


def max_threads() -> int:
    return int(lib().or_max_threads())


def tga_encode(rgb8: np.ndarray) -> bytes:
    """Run-length Targa file of an 8-bit RGB image [H, W, 3] (definition in
    oracle.h)."""
    a = np.ascontiguousarray(rgb8, dtype=np.uint8)
    if a.ndim != 3 or a.shape[2] != 3:
        raise ValueError("image must be [H, W, 3] uint8")
    h, w = int(a.shape[0]), int(a.shape[1])
    n = lib().or_tga_encode(a.ctypes.data, w, h, None, 0)
    if n < 0:
        raise ValueError("width and height must be 1..65535")
    out = np.zeros(n, np.uint8)
    got = lib().or_tga_encode(a.ctypes.data, w, h, out.ctypes.data, n)
    assert got == n
    return out.tobytes()
