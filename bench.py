#!/usr/bin/env python3
"""Benchmark of the ambient-occlusion ray caster on one MI355X.

Workload: the 26,318-object protein-like scene (13,159 spheres + 13,159
cylinders, seeded random walk in a ball of radius 40) rendered at 3860x4548
(17.6 MP, the paper's high-resolution case; Sec. 2, Table 3) with 16 AO
samples per hit pixel, light rescale 0.3 and sky light 1.0, FP32 intersection
with FP64 re-solve of grazing hits.

One step = one pass of the whole hot path on the resident scene: the uniform
grid rebuilt on the GPU from the resident FP64 arrays (bounds, count, scan,
scatter, sort -- the "Preprocess" phase of Table 5) and the frame rendered
(the "Ray Tracing" phase).  value = (primary + AO) rays per second over the
timed steps.  The line also carries frames/s, p50/p99 frame latency, the plain
FP64 GPU path on the same frame, the render kernel's roofline position and
the CPU oracle's rate on a sample of the frame.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Algorithmic flop model of the grid method (FP32-equivalent operations; FMA
# = 2; add, mul, min, max, compare, sqrt, rcp, sin, cos = 1), per counted
# event: ray setup + DDA init, DDA step (a cell entered), sphere test (+ hit),
# cylinder test (+ hit), primary ray generation, normal + facing, per light,
# orthonormal basis, AO direction, final shade.
FLOP_COST = dict(ray_setup=40, cell=4, sph_test=22, sph_hit=4, cyl_test=45, cyl_hit=12,
                 primary_gen=20, normal=10, per_light=8, onb=12, ao_dir=23, shade=10)
# An empty-space jump (skipping up to 32 empty cells at once) is not in the
# table; the variant that prices each jump as a re-initialised DDA step is
# reported beside the table's figure, never in its place.
JUMP_COST = 16
PEAK_FP32_TFLOPS = 157.3          # MI355X FP32 vector peak (256 CU x 2.4 GHz x 256 flop/clk)
PEAK_FP32_NONPACKED_TFLOPS = 78.6  # without packed-FP32 issue
PEAK_HBM_GBS = 8000.0
GRID_LAMBDA = 24.0  # grid cells per primitive of the benchmarked scene (the library default)
ORBIT_LAMBDAS = (8.0, 16.0, 24.0, 32.0, 48.0)  # grid densities the orbit graph is tuned over


def algorithmic_flops(st: dict, n_lights: int, ao_on: bool, jump_cost: int = 0) -> float:
    c = FLOP_COST
    return float(c["ray_setup"] * st["rays_traced"] + c["cell"] * st["cells"]
                 + jump_cost * st.get("jumps", 0)
                 + c["sph_test"] * st["sph_tests"] + c["sph_hit"] * st["sph_hits"]
                 + c["cyl_test"] * st["cyl_tests"] + c["cyl_hit"] * st["cyl_hits"]
                 + c["primary_gen"] * st["pixels"] + c["normal"] * st["hit_pixels"]
                 + c["per_light"] * st["hit_pixels"] * n_lights
                 + (c["onb"] * st["hit_pixels"] if ao_on else 0)
                 + c["ao_dir"] * st["ao_rays"] + c["shade"] * st["pixels"])


def _current_profile(name: str):
    """A committed rocprofv3 summary under profiles/, or None when it is
    missing or was taken on another version of the kernel source."""
    import hashlib
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    prof = json.load(open(path))
    src = b"".join(open(os.path.join(ROOT, f), "rb").read() for f in prof["kernel_source_files"])
    if hashlib.sha256(src).hexdigest() != prof["kernel_source_sha256"]:
        return None
    return prof


def measured_traffic():
    """HBM bytes per render launch from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE summary (each scaled by a plain copy's reading), valid only
    while the kernel source is the one that was profiled; else None."""
    prof = _current_profile("render_wave_p17_traffic.json")
    return None if prof is None else prof["hbm_bytes_per_launch"]


def measured_issue():
    """Instruction-issue figures of the render kernel from the committed
    rocprofv3 SQ counter passes (same source-version rule): the share of
    VALU and SALU issue slots used and the active lanes per VALU
    instruction; else None."""
    prof = _current_profile("render_wave_p17_issue.json")
    if prof is None:
        return None
    d = prof["derived"]
    return {k: d[k] for k in ("valu_issue_frac", "salu_issue_frac", "active_lanes_per_valu_inst")}


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _rows_sample(oracle, scene, cam, params, grid, target_s: float, n_threads: int):
    """Render evenly spaced full rows sized to about target_s seconds."""
    import numpy as np
    W, H = cam.width, cam.height
    rows = np.arange(0, H, max(H // 8, 1))[:8]
    pix = (rows[:, None] * W + np.arange(W)[None, :]).reshape(-1)
    t0 = time.perf_counter()
    oracle.render(scene, cam, params, grid=grid, pix=pix, n_threads=n_threads)
    per_row = (time.perf_counter() - t0) / len(rows)
    n_rows = int(min(H, max(len(rows), target_s / max(per_row, 1e-9))))
    rows = np.unique(np.linspace(0, H - 1, n_rows).round().astype(np.int64))
    pix = (rows[:, None] * W + np.arange(W)[None, :]).reshape(-1)
    t0 = time.perf_counter()
    r = oracle.render(scene, cam, params, grid=grid, pix=pix, n_threads=n_threads)
    return r, time.perf_counter() - t0, len(rows)


def cpu_baseline(scene, cam, params, cells_per_prim: float, target_s: float = 20.0,
                 one_thread_s: float = 8.0) -> tuple:
    """The oracle, as it stands, on the same frame with the GPU's grid density:
    the whole frame on every host thread when that takes under target_s
    (else evenly spaced full rows sized to it), then evenly spaced rows on one
    thread for the per-core rate.  Returns (baseline record, the oracle's
    frame or None when sampled, its traversal counters)."""
    import oracle
    oracle.build(force=False)
    grid = oracle.Grid(scene, cells_per_prim)
    W, H = cam.width, cam.height
    threads = oracle.max_threads()
    # one calibration row batch decides whether the whole frame fits
    _, dt_rows, n_rows = _rows_sample(oracle, scene, cam, params, grid, 0.5, threads)
    if dt_rows / n_rows * H <= target_s:
        t0 = time.perf_counter()
        ref = oracle.render(scene, cam, params, grid=grid)
        dt, rows_used = time.perf_counter() - t0, H
    else:
        ref, dt, rows_used = _rows_sample(oracle, scene, cam, params, grid, target_s, threads)
    cnt = ref["counters"]
    rays = cnt["primary_rays"] + cnt["ao_rays"]
    r1, dt1, rows1 = _rows_sample(oracle, scene, cam, params, grid, one_thread_s, 1)
    c1 = r1["counters"]
    rays1 = c1["primary_rays"] + c1["ao_rays"]
    out = {"value": rays / dt, "unit": "rays/s", "cores": int(threads), "kind": "oracle",
           "sample": "%s of the same %dx%d frame (%d of %d rows), FP64 oracle on its uniform "
                     "grid at %g cells per primitive (the GPU's), OpenMP over pixels on %d "
                     "threads, %.1f s" % ("the whole" if rows_used == H else "evenly spaced rows",
                                           W, H, rows_used, H, cells_per_prim, threads, dt),
           "seconds": dt, "rays": rays, "shadow_rays": cnt["shadow_rays"],
           "cpu_model": _cpu_model(), "host_cpus": os.cpu_count(),
           "one_thread": {"value": rays1 / dt1, "unit": "rays/s", "rows": rows1,
                          "seconds": dt1, "rays": rays1}}
    return out, (ref if rows_used == H else None), cnt, dt


def orbit_measure(tr, torch, scenegen, launches: int = 3) -> dict:
    """64 views of the 1,000,000-object walk scene at 1920x1080, 32 AO
    samples, captured once into a hipGraph; the graph is timed with the
    default launch shape, then tuned on itself (grid density over ORBIT_LAMBDAS
    and launch shape, tr_graph_autotune) and timed again: the tuned figure is
    the orbit's."""
    scene = scenegen.orbit_scene()
    gs = tr.Scene(scene)
    cams = scenegen.orbit_cameras()
    params = scenegen.orbit_params()
    frames = [tr.alloc_frame(c, ("rgb",), stats=False) for c in cams]
    stats = torch.zeros(tr.STAT_COUNT, dtype=torch.int64, device="cuda")
    for f in frames:
        f["stats"] = stats
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def time_graph(g):
        g.launch()
        torch.cuda.synchronize()
        stats.zero_()
        e0.record()
        for _ in range(launches):
            g.launch()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / launches, dict(zip(tr.STAT_NAMES, stats.cpu().tolist()))

    g = tr.Graph([gs] * len(cams), cams, params, frames)
    ms_default, _ = time_graph(g)
    t0 = time.perf_counter()
    used, lam, _ = g.autotune(lambdas=ORBIT_LAMBDAS)
    tune_s = time.perf_counter() - t0
    ms, st = time_graph(g)
    g.destroy()
    gs.rebuild(GRID_LAMBDA)
    rays = (st["pixels"] + st["ao_rays"]) / launches
    # the sparse scene with and without empty-space skipping: 8 views per batch
    sub = [tr.alloc_frame(c, ("rgb",), stats=False) for c in cams[:8]]
    walks = walk_compare(tr, torch, gs, lambda: tr.render_batch_into(
        [gs] * 8, cams[:8], params[:8], sub), [(24.0, 32), (24.0, 1), (4.0, 32), (4.0, 1)], reps=2)
    bvh = bvh_measure(tr, torch, gs, lambda a: tr.render_batch_tiles_into(
        [gs] * 8, cams[:8], params[:8], sub, [0] * 8, [tr.tile_count(c.width, c.height, 8) for c in cams[:8]],
        tune={"accel": a, "tile_w": 8}), reps=2)
    # FP32 (+ FP64 re-solve) against the plain FP64 path, same 8-view batch
    prec = {}
    for name in ("fp32_resolve", "fp64"):
        tr.render_batch_into([gs] * 8, cams[:8], params[:8], sub, precision=name)
        torch.cuda.synchronize()
        e0.record()
        tr.render_batch_into([gs] * 8, cams[:8], params[:8], sub, precision=name)
        e1.record()
        torch.cuda.synchronize()
        prec[name + "_ms"] = e0.elapsed_time(e1)
    prec["fp64_over_fp32"] = prec["fp64_ms"] / prec["fp32_resolve_ms"]
    return {"workload": "1,000,000-object walk (ball radius 250), 64 views of 1920x1080 per "
                        "graph launch, 32 AO samples, FP32 + FP64 re-solve",
            "ms_per_launch": ms, "views_per_s": 64 * 1000.0 / ms, "rays_per_launch": rays,
            "tune": used, "cells_per_prim": lam if lam > 0 else GRID_LAMBDA,
            "lambdas_tried": list(ORBIT_LAMBDAS), "tuning_s": tune_s,
            "ms_per_launch_default_tune": ms_default,
            "rays_per_s": rays / (ms * 1e-3),
            "walk_8_views": walks, "bvh_8_views": bvh, "precision_8_views": prec}


def scene_ingest_measure(tr, torch, scene, name: str) -> dict:
    """Scene ingest (the "Parse" + "Preprocess" phases of Table 5): build from
    in-memory arrays, save as a binary scene file, and load it back (read +
    upload + GPU grid build), each timed to completion."""
    import tempfile
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    gs = tr.Scene(scene)
    torch.cuda.synchronize()
    build_ms = (time.perf_counter() - t0) * 1e3
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "scene.trs")
        t0 = time.perf_counter()
        gs.save(path)
        save_ms = (time.perf_counter() - t0) * 1e3
        nbytes = os.path.getsize(path)
        t0 = time.perf_counter()
        gl = tr.Scene.load(path)
        torch.cuda.synchronize()
        load_ms = (time.perf_counter() - t0) * 1e3
    del gs, gl
    return {"scene": name, "objects": scene.n_prims, "file_bytes": nbytes,
            "build_from_arrays_ms": build_ms, "save_ms": save_ms, "load_ms": load_ms,
            "load_MBps": nbytes / (load_ms * 1e-3) / 1e6}


def end_to_end_measure(tr, torch, scene, cam, params, prec, reps: int = 3) -> dict:
    """One 17.6 MP frame from a scene file to an image file in host memory,
    in the phases of Table 5: scene load (file read, upload and GPU grid
    build: the paper's parse + preprocess), ray tracing, and image I/O
    (8-bit conversion, Targa file on the GPU, download into pinned memory).
    Each phase is timed to completion; the best of reps runs is kept."""
    import tempfile
    best = None
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "scene.trs")
        tr.Scene(scene).save(path)
        frame = tr.alloc_frame(cam, ("rgb",))
        H, W = cam.height, cam.width
        buf = torch.empty(tr.tga_max_bytes(W, H), dtype=torch.uint8, device="cuda")
        host = torch.empty(tr.tga_max_bytes(W, H), dtype=torch.uint8, pin_memory=True)
        for k in range(reps + 1):  # run 0 warms the caches and the allocator
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            gs = tr.Scene.load(path)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            tr.render_into(gs, cam, params, frame, prec)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            q = tr.quantize_rgb8(frame["rgb"])
            tga = tr.encode_tga(q, out=buf)
            host[:tga.numel()].copy_(tga, non_blocking=True)
            torch.cuda.synchronize()
            t3 = time.perf_counter()
            run = {"scene_load_ms": (t1 - t0) * 1e3, "ray_tracing_ms": (t2 - t1) * 1e3,
                   "image_io_ms": (t3 - t2) * 1e3, "total_ms": (t3 - t0) * 1e3,
                   "image_bytes": int(tga.numel())}
            del gs
            if k > 0 and (best is None or run["total_ms"] < best["total_ms"]):
                best = run
    best["workload"] = ("protein-like 26,318 objects from a binary scene file to a Targa file in "
                        "host memory, 3860x4548, 16 AO samples")
    return best


def frame_output_measure(tr, torch, frame, reps: int = 20) -> dict:
    """8-bit output of the 17.6 MP frame on the GPU (tr_frame_quantize: 12 B
    read + 3 B written per pixel, HBM-bound), its asynchronous download to
    pinned host memory, the host PPM encoding, and the run-length Targa file
    written on the GPU (tr_frame_encode_tga, wall time per call including its
    wait for the size pass) with the download of the file."""
    rgb = frame["rgb"]
    q = tr.quantize_rgb8(rgb)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        tr.quantize_rgb8(rgb, out=q)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    nbytes = rgb.numel() * 4 + q.numel()
    host = torch.empty(q.shape, dtype=torch.uint8, pin_memory=True)
    host, ev = tr.frame_to_host_rgb8(frame, host=host)
    ev.synchronize()
    d0, d1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    d0.record()
    host.copy_(q, non_blocking=True)
    d1.record()
    torch.cuda.synchronize()
    d2h_ms = d0.elapsed_time(d1)
    t0 = time.perf_counter()
    ppm = tr.encode_ppm(host)
    enc_ms = (time.perf_counter() - t0) * 1e3
    # Targa file on the GPU, then its download
    H, W = int(q.shape[0]), int(q.shape[1])
    buf = torch.empty(tr.tga_max_bytes(W, H), dtype=torch.uint8, device=q.device)
    tga = tr.encode_tga(q, out=buf)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        tga = tr.encode_tga(q, out=buf)
    torch.cuda.synchronize()
    tga_ms = (time.perf_counter() - t0) * 1e3 / reps
    tga_host = torch.empty(tga.numel(), dtype=torch.uint8, pin_memory=True)
    d0.record()
    tga_host.copy_(tga, non_blocking=True)
    d1.record()
    torch.cuda.synchronize()
    tga_d2h_ms = d0.elapsed_time(d1)
    return {"quantize_ms": ms, "quantize_GBps": nbytes / (ms * 1e-3) / 1e9,
            "quantize_hbm_frac": nbytes / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS,
            "bytes": nbytes, "d2h_ms": d2h_ms, "d2h_GBps": q.numel() / (d2h_ms * 1e-3) / 1e9,
            "ppm_encode_ms": enc_ms, "ppm_bytes": len(ppm),
            "tga_encode_ms": tga_ms, "tga_bytes": int(tga.numel()),
            "tga_ratio": tga.numel() / float(q.numel()), "tga_d2h_ms": tga_d2h_ms}


def variant_measure(tr, torch, gs, cam, p, prec, workload: str, frames: int = 3) -> dict:
    """The 17.6 MP frame with a shading variant on (antialiasing, Phong
    highlight): ms per frame and counted (primary + AO) rays per second."""
    fr = tr.alloc_frame(cam, ("rgb",), stats=True)
    tr.render_into(gs, cam, p, fr, prec)
    torch.cuda.synchronize()
    fr["stats"].zero_()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(frames):
        tr.render_into(gs, cam, p, fr, prec)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / frames
    st = dict(zip(tr.STAT_NAMES, fr["stats"].cpu().tolist()))
    rays = (st["pixels"] + st["ao_rays"]) / frames
    return {"workload": workload, "ms_per_frame": ms, "frames_per_s": 1000.0 / ms,
            "rays_per_frame": rays, "rays_per_s": rays / (ms * 1e-3)}


def walk_compare(tr, torch, gs, render, configs, reps: int = 3) -> list:
    """Render time of the same frame(s) under other grid shapes: grid density
    (cells per primitive) and empty-space skipping cap (1 = the plain
    uniform-grid walk, no jumps).  The scene is rebuilt for each shape and
    restored to the defaults (24, 32) afterwards."""
    import numpy as np
    out = []
    for lam, cap in configs:
        gs.rebuild(lam)
        gs.set_max_skip(cap)
        render()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            render()
        e1.record()
        torch.cuda.synchronize()
        out.append({"cells_per_prim": lam, "max_skip": cap,
                    "grid_cells": int(np.prod(gs.grid_info()[2])),
                    "ms": e0.elapsed_time(e1) / reps})
    gs.rebuild(24.0)
    gs.set_max_skip(32)
    return out


def bvh_measure(tr, torch, gs, render_with, reps: int = 3) -> dict:
    """The BVH walk against the grid walk on the same frame(s): BVH build
    time (GPU, to completion), the tree's depth and render time of each walk
    (the BVH walk is refused on a tree deeper than its stack)."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    gs.build_bvh()
    build_ms = (time.perf_counter() - t0) * 1e3
    out = {"bvh_build_ms": build_ms, "bvh_depth": gs.bvh_depth()}
    for name, accel in (("grid_ms", 0), ("bvh_ms", 1)):
        if accel and out["bvh_depth"] > 48:
            out[name] = None
            continue
        render_with(accel)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            render_with(accel)
        e1.record()
        torch.cuda.synchronize()
        out[name] = e0.elapsed_time(e1) / reps
    return out


def variants_measure(tr, torch, scenegen, np, gs, scene, cam, params, prec, log):
    """The shading-variant frames (antialiasing, highlight, transparency) and
    the triangle surface frame, each at 17.6 MP."""
    import dataclasses
    aa = variant_measure(tr, torch, gs, cam, dataclasses.replace(params, aa_samples=4), prec,
                         "protein-like 26,318 objects, 3860x4548, 4 primary samples per pixel, "
                         "16 AO samples each, FP32 + FP64 re-solve")
    aa["aa_samples"] = 4
    log("antialiased frame", aa)
    spec = variant_measure(tr, torch, gs, cam,
                           dataclasses.replace(params, specular=0.3, shininess=30.0), prec,
                           "protein-like 26,318 objects, 3860x4548, 16 AO samples, Phong "
                           "highlight k_s 0.3, n 30, FP32 + FP64 re-solve")
    log("highlight frame", spec)
    glass = tr.Scene(scenegen.Scene(**{**scene.__dict__, "sph_opacity":
                                       np.full(scene.n_spheres, 0.5, np.float32)}))
    trans = variant_measure(tr, torch, glass, cam, dataclasses.replace(params, max_layers=4), prec,
                            "protein-like 26,318 objects, spheres at opacity 0.5 (cylinders "
                            "opaque), up to 4 surfaces per pixel, 3860x4548, 16 AO samples per "
                            "surface, FP32 + FP64 re-solve")
    del glass
    log("transparent frame", trans)
    surf_scene = scenegen.surface_scene()
    surf = tr.Scene(surf_scene)
    tris = variant_measure(tr, torch, surf, cam, params, prec,
                           "molecular-surface stand-in: 83 closed icosphere blobs on the protein "
                           "walk, 26,560 triangles, 3860x4548, 16 AO samples, FP32 + FP64 "
                           "re-solve")
    tris["build_ms"] = scene_ingest_measure(tr, torch, surf_scene, "surface")["build_from_arrays_ms"]
    del surf
    log("triangle surface frame", tris)
    return aa, spec, trans, tris


def serving_measure(tr, torch, scenegen, seconds: float, warmup: float = 5.0,
                    rate: float = 50.0, small_seconds: float = 20.0,
                    small_budget: int = 1920 * 1080 * 12, burst_jobs: int = 400) -> dict:
    """Render serving over a pool of 16 resident walk scenes of 2k-200k
    objects, requests at resolutions uniform over {256x256, 965x1137,
    1920x1080} with 4-32 AO samples:
    - Poisson arrivals (mean `rate` per second) at the 64 GB frame budget:
      `warmup` seconds of the stream, not reported, then `seconds` seconds;
    - the same arrival process for `small_seconds` under a forced small frame
      budget (`small_budget` bytes, one 1920x1080 frame), where a request
      that arrives while others are on the GPU waits for memory;
    - a burst of `burst_jobs` requests arriving at once, which keeps the GPU
      saturated: continuous batching under full load (latency here is the
      time from the burst to each job's completion)."""
    from paper_0801_1500_amd.serve import Job, Server
    pool = scenegen.serving_pool()
    gpool = [tr.Scene(s) for s in pool]
    radii = [scenegen.serving_radius(s.n_prims) for s in pool]

    def jobs_of(reqs, t_shift=0.0, at_once=False):
        return [Job(i, 0.0 if at_once else t - t_shift, si, cam, p)
                for i, (t, si, cam, p) in enumerate(reqs)]

    n_warm, n_main = int(round(warmup * rate)), int(round(seconds * rate))
    reqs = scenegen.serving_requests(radii, n_warm + n_main, rate_hz=rate, seed=3)
    srv = Server(gpool, hbm_budget=64 << 30)
    if n_warm:
        srv.run(jobs_of(reqs[:n_warm]), realtime=True)
    t_start = reqs[n_warm - 1][0] if n_warm else 0.0
    out = srv.run(jobs_of(reqs[n_warm:], t_shift=t_start), realtime=True).summary()
    out["workload"] = ("Poisson %.0f req/s, %d jobs over %.0f s after a %.0f s warm-up of %d jobs, "
                       "64 GB frame budget, 16 resident scenes of 2k-200k objects, 256x256 / "
                       "965x1137 / 1920x1080, 4-32 AO samples" % (rate, n_main, seconds, warmup,
                                                                   n_warm))
    if small_seconds > 0:
        sreqs = scenegen.serving_requests(radii, int(round(small_seconds * rate)), rate_hz=rate,
                                          seed=4)
        small = Server(gpool, hbm_budget=small_budget).run(jobs_of(sreqs), realtime=True).summary()
        small["workload"] = ("Poisson %.0f req/s, %d jobs, forced %.1f MiB frame budget "
                             "(one 1920x1080 frame)" % (rate, len(sreqs), small_budget / 2**20))
        out["small_budget"] = small
    if burst_jobs > 0:
        breqs = scenegen.serving_requests(radii, burst_jobs, rate_hz=rate, seed=5)
        burst = Server(gpool, hbm_budget=64 << 30).run(jobs_of(breqs, at_once=True),
                                                       realtime=False).summary()
        burst["workload"] = "%d requests arriving at once, 64 GB frame budget" % burst_jobs
        out["burst"] = burst
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--fp64-frames", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--autotune", action="store_true", help="autotune the launch shape first")
    ap.add_argument("--serve-warmup", type=float, default=5.0,
                    help="seconds of the serving stream before the measured window")
    ap.add_argument("--serve-small-seconds", type=float, default=20.0,
                    help="length of the forced small-budget serving run (0 = skip)")
    ap.add_argument("--serve-seconds", type=float, default=60.0,
                    help="length of the Poisson serving run (0 = skip)")
    ap.add_argument("--no-orbit", action="store_true", help="skip the 1M-object orbit run")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the shading-variant and triangle frames (profiling runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: this build has no multi-GPU path "
              "(pixels would shard by interleaved tiles with one frame gather; not built).",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_0801_1500_amd as tr
    import scenegen

    torch.cuda.set_device(0)
    scene = scenegen.protein_scene(seed=2)
    cam = scenegen.protein_camera(scenegen.RES_17MP)
    params = scenegen.Params(ao_samples=16, seed=2)
    prec = "fp32_resolve"
    gs = tr.Scene(scene, cells_per_prim=GRID_LAMBDA)
    stream = torch.cuda.current_stream()
    log = lambda *a: print("[bench]", *a, file=sys.stderr, flush=True)
    log("scene built", gs.grid_info()[2].tolist(), "refs", gs.grid_info()[3])

    tune = None
    tune_ms = None
    if args.autotune:
        tune, tune_ms = tr.autotune(gs, cam, params, precision=prec)
        print("autotuned", tune, "%.2f ms" % tune_ms, file=sys.stderr, flush=True)
    used_tune = dict(tune) if tune else tr.default_tune()

    # exact algorithmic op counts of this frame (one counting launch)
    cnt_frame = tr.alloc_frame(cam, ("rgb",), stats=True)
    tr.render_into(gs, cam, params, cnt_frame, prec, tune=dict(used_tune, count_ops=1))
    torch.cuda.synchronize()
    st = dict(zip(tr.STAT_NAMES, cnt_frame["stats"].cpu().tolist()))
    del cnt_frame
    ao_on = params.ao_samples > 0 and params.skylight > 0
    flops_frame = algorithmic_flops(st, scene.n_lights, ao_on)
    rays_frame = st["pixels"] + st["ao_rays"]

    log("counting launch done", st)
    frame = tr.alloc_frame(cam, ("rgb",), stats=True)

    def step():
        gs.rebuild()
        tr.render_into(gs, cam, params, frame, prec, tune=tune)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    frame["stats"].zero_()
    K = args.steps
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(K)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(K):
        ev[k][0].record(stream)
        gs.rebuild()
        ev[k][1].record(stream)
        tr.render_into(gs, cam, params, frame, prec, tune=tune)
        ev[k][2].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    log("timed %d steps in %.3f s" % (K, wall))
    step_ms = np.array([ev[k][0].elapsed_time(ev[k][2]) for k in range(K)])
    build_ms = np.array([ev[k][0].elapsed_time(ev[k][1]) for k in range(K)])
    render_ms = np.array([ev[k][1].elapsed_time(ev[k][2]) for k in range(K)])
    tst = dict(zip(tr.STAT_NAMES, frame["stats"].cpu().tolist()))
    rays_timed = tst["pixels"] + tst["ao_rays"]
    assert rays_timed == K * rays_frame, (rays_timed, K * rays_frame)
    ms_per_step = wall * 1000.0 / K
    value = rays_timed / wall

    kernel_ms = float(render_ms.mean())
    gpu_rgb = frame["rgb"].cpu().numpy()  # the last timed frame, for the parity block
    peak = tr.measure_fp32_peak()
    log("measured FP32 FMA peak", peak)

    # plain FP64 GPU path on the same frame
    fp64 = None
    if args.fp64_frames > 0:
        f64 = tr.alloc_frame(cam, ("rgb",))
        tr.render_into(gs, cam, params, f64, "fp64")
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.fp64_frames):
            tr.render_into(gs, cam, params, f64, "fp64")
        e1.record(stream)
        torch.cuda.synchronize()
        ms64 = e0.elapsed_time(e1) / args.fp64_frames
        fp64 = {"render_ms": ms64, "rays_per_s": rays_frame / (ms64 * 1e-3),
                "speedup_fp32_over_fp64": ms64 / float(render_ms.mean())}
        del f64
        log("fp64 plain path", fp64)

    aa = spec = trans = tris = walks = bvh = None
    if not args.no_variants:
        wf = tr.alloc_frame(cam, ("rgb",))

        walks = walk_compare(tr, torch, gs, lambda: tr.render_into(gs, cam, params, wf, prec),
                             [(24.0, 32), (24.0, 1), (4.0, 32), (4.0, 1)])
        log("grid shapes", walks)
        bvh = bvh_measure(tr, torch, gs, lambda a: tr.render_into(gs, cam, params, wf, prec,
                                                                  tune={"accel": a}))
        log("bvh walk", bvh)
        aa, spec, trans, tris = variants_measure(tr, torch, scenegen, np, gs, scene, cam, params,
                                                 prec, log)


    frame_out = frame_output_measure(tr, torch, frame)
    log("frame output", frame_out)
    e2e = end_to_end_measure(tr, torch, scene, cam, params, prec)
    log("end to end", e2e)
    ingest = [scene_ingest_measure(tr, torch, scene, "protein-like 26,318 objects")]
    if not args.no_orbit:
        ingest.append(scene_ingest_measure(tr, torch, scenegen.orbit_scene(),
                                           "1,000,000-object walk"))
    log("scene ingest", ingest)

    orbit = None
    if not args.no_orbit:
        log("orbit (1M objects, 64 views per graph launch) ...")
        orbit = orbit_measure(tr, torch, scenegen)
        log("orbit", orbit)
    serving = None
    if args.serve_seconds > 0:
        log("serving stream ...")
        serving = serving_measure(tr, torch, scenegen, args.serve_seconds, args.serve_warmup,
                                  small_seconds=args.serve_small_seconds)
        log("serving", serving)

    cpu = ref = ocnt = None
    if not args.no_cpu:
        log("cpu baseline (oracle) ...")
        cpu, ref, ocnt, _ = cpu_baseline(scene, cam, params, GRID_LAMBDA)
        log("cpu baseline", cpu)

    # roofline of the render kernel: the flop table over the kernel's own
    # counters, over the kernel's mean duration in the timed steps
    achieved = flops_frame / (kernel_ms * 1e-3) / 1e12
    flops_jump = algorithmic_flops(st, scene.n_lights, ao_on, JUMP_COST)
    roofline = {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / PEAK_FP32_TFLOPS, "traffic": measured_traffic(),
                "frac_nonpacked": achieved / PEAK_FP32_NONPACKED_TFLOPS,
                "peak_measured": peak["tflops"], "frac_measured": achieved / peak["tflops"],
                "peak_measured_how": "non-packed FP32 FMA chains on every lane, 32 waves per CU "
                                     "(tr_measure_fp32_peak), reported clock %.0f MHz, %d CUs"
                                     % (peak["clock_mhz"], peak["n_cus"]),
                "kernel": "k_render_wave", "kernel_ms": kernel_ms,
                "flop_per_frame": flops_frame, "flop_per_counted_ray": flops_frame / rays_frame,
                "flop_model": "cost table per op over the kernel's own counters: cells entered, "
                              "sphere/cylinder tests and hits, rays, pixels, hit pixels, lights, "
                              "AO directions; empty-space jumps not priced",
                "with_jump_cost": {"jump_cost": JUMP_COST, "flop_per_frame": flops_jump,
                                   "achieved": flops_jump / (kernel_ms * 1e-3) / 1e12,
                                   "frac": flops_jump / (kernel_ms * 1e-3) / 1e12 / PEAK_FP32_TFLOPS},
                "oracle_counts": None, "issue": measured_issue()}
    if ocnt is not None:
        # the same table over the oracle's plain-DDA counts at the GPU's grid
        # density (every cell on a ray's path is a step there), per counted ray
        o_rays = ocnt["primary_rays"] + ocnt["ao_rays"]
        f_ray = algorithmic_flops(ocnt, scene.n_lights, ao_on) / o_rays
        o_ach = f_ray * rays_frame / (kernel_ms * 1e-3) / 1e12
        roofline["oracle_counts"] = {"flop_per_counted_ray": f_ray,
                                     "flop_per_frame": f_ray * rays_frame, "achieved": o_ach,
                                     "frac": o_ach / PEAK_FP32_TFLOPS,
                                     "cells_per_counted_ray": ocnt["cells"] / o_rays,
                                     "counted_rays": o_rays}
    if roofline["traffic"] is not None:  # measured HBM bytes over the live kernel time
        roofline["hbm_GBps"] = roofline["traffic"] / (kernel_ms * 1e-3) / 1e9
        roofline["hbm_frac"] = roofline["hbm_GBps"] / PEAK_HBM_GBS
    parity = None
    if ref is not None:  # the GPU frame against the oracle's, whole frame
        d = np.abs(gpu_rgb.astype(np.float64) - ref["rgb"])
        parity = {"pixels": int(d.shape[0] * d.shape[1]), "max_abs_all": float(d.max()),
                  "rms_all": float(np.sqrt(np.mean(d * d))),
                  "frac_pixels_over_1e-3": float(np.mean(d.max(axis=2) > 1e-3))}
        del d, ref

    out = {
        "metric": "rays/sec (primary+AO) and frames/s at 17.6 MP AO; p50/p99 frame latency",
        "value": value, "unit": "rays/s", "n_gpus": 1, "steps": K, "warmup": args.warmup,
        "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "protein-like random walk, 13,159 spheres + 13,159 cylinders, "
                               "3860x4548, 16 AO samples, light rescale 0.3, sky light 1.0, "
                               "FP32 + FP64 re-solve; step = grid rebuild + render",
                   "width": cam.width, "height": cam.height, "ao_samples": params.ao_samples,
                   "precision": prec, "tune": used_tune, "parallelism": "1 GPU"},
        "fps": 1000.0 / ms_per_step,
        "frame_latency_ms_p50": float(np.percentile(step_ms, 50)),
        "frame_latency_ms_p99": float(np.percentile(step_ms, 99)),
        "render_ms_mean": float(render_ms.mean()), "build_ms_mean": float(build_ms.mean()),
        "rays_per_frame": rays_frame, "shadow_rays_per_frame": st["shadow_rays"],
        "hit_pixels": st["hit_pixels"], "op_counts": st,
        "render_only_rays_per_s": rays_frame / (render_ms.mean() * 1e-3),
        "fp64_plain": fp64,
        "walk_shapes": walks,
        "bvh_walk": bvh,
        "antialias": aa,
        "specular": spec,
        "transparency": trans,
        "triangles": tris,
        "frame_output": frame_out,
        "scene_ingest": ingest,
        "end_to_end": e2e,
        "orbit": orbit,
        "serving": serving,
        "roofline": roofline,
        "parity_vs_oracle": parity,
        "cpu_baseline": cpu,
        "paper_context": "Tachyon on 6144 Blue Gene/L processors: 2.6416 s per 17.6 MP AO frame "
                         "(0.379 frames/s), 822x a 3 GHz Pentium IV (Table 3)",
    }
    if tune_ms is not None:
        out["autotune_ms"] = tune_ms
    print(json.dumps(out))


if __name__ == "__main__":
    main()
